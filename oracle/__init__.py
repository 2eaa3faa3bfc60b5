"""ORACLE -- test infrastructure only.

A plain, slow FP64 CPU implementation of what the lattice FMM computes: phi by the two-step
quadrature of Section 3.2 plus the expansion eq. (3.1) (``oracle.phi``), and the direct sum
u(t) = sum_s phi(t - s) f(s) of eq. (1.7) (``oracle.direct``, plain C with OpenMP); and the
two applications of Section 10 as dense FP64 solves on top of them (``oracle.extensions``:
the lattice with inclusions, eq. 10.1-10.4, and the Dirichlet problem, eq. 10.5-10.7).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the GPU library (``paper_1105_3505_amd``), and the
library never imports it.
"""
