"""ORACLE (test infrastructure only): write the committed quadrature table of phi.

Usage:  python -m oracle.make_phi_table [radius] [stencil]

Evaluates phi(a, b), 0 <= b <= a <= radius (default 128), of the 5-point operator (or, with
stencil 9, of the isotropic 9-point operator) by the two-step quadrature of Section 3.2
(``oracle.phi.phi_table_quadrature``) and writes one line per entry,
``a b value`` with the value as an exact hexadecimal float.  Nothing but ``oracle/`` is used.
"""
from __future__ import annotations

import os
import sys
import time

# one BLAS thread per worker process: the workers already use every core
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

from oracle.phi import TABLE_RADIUS, octant_index, phi_table_quadrature, table_file


def main() -> None:
    radius = int(sys.argv[1]) if len(sys.argv) > 1 else TABLE_RADIUS
    stencil = int(sys.argv[2]) if len(sys.argv) > 2 else 5
    path = table_file(stencil)
    t0 = time.time()
    table = phi_table_quadrature(radius, stencil=stencil)
    with open(path, "w") as fh:
        fh.write("# phi(a,b) for 0 <= b <= a <= %d, %d-point operator, two-step quadrature of Section 3.2\n"
                 % (radius, stencil))
        fh.write("# written by: python -m oracle.make_phi_table %d %d\n" % (radius, stencil))
        for a in range(radius + 1):
            for b in range(a + 1):
                fh.write("%d %d %s\n" % (a, b, float(table[octant_index(a, b)]).hex()))
    print("wrote %s (%d entries) in %.1f s" % (path, len(table), time.time() - t0))


if __name__ == "__main__":
    main()
