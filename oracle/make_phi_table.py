"""ORACLE (test infrastructure only): write the committed quadrature table of phi.

Usage:  python -m oracle.make_phi_table [radius]

Evaluates phi(a, b), 0 <= b <= a <= radius (default 128), by the two-step quadrature of
Section 3.2 (``oracle.phi.phi_table_quadrature``) and writes one line per entry,
``a b value`` with the value as an exact hexadecimal float.  Nothing but ``oracle/`` is used.
"""
from __future__ import annotations

import os
import sys
import time

# one BLAS thread per worker process: the workers already use every core
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

from oracle.phi import TABLE_RADIUS, _TABLE_FILE, octant_index, phi_table_quadrature


def main() -> None:
    radius = int(sys.argv[1]) if len(sys.argv) > 1 else TABLE_RADIUS
    t0 = time.time()
    table = phi_table_quadrature(radius)
    with open(_TABLE_FILE, "w") as fh:
        fh.write("# phi(a,b) for 0 <= b <= a <= %d, two-step quadrature of Section 3.2\n" % radius)
        fh.write("# written by: python -m oracle.make_phi_table %d\n" % radius)
        for a in range(radius + 1):
            for b in range(a + 1):
                fh.write("%d %d %s\n" % (a, b, float(table[octant_index(a, b)]).hex()))
    print("wrote %s (%d entries) in %.1f s" % (_TABLE_FILE, len(table), time.time() - t0))


if __name__ == "__main__":
    main()
