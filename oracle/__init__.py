"""Plain FP64 CPU oracle for the Schwarz-preconditioned Wilson-clover solver.

TEST INFRASTRUCTURE ONLY. This package exists to check the HIP path. Only the test suite,
the smoke check in __graft_entry__ and the CPU-baseline leg of bench.py may import it; the
product path (the C-ABI library and its Python binding) never calls it and has no
fallback to it.

Everything here is NumPy on complex128, written for readability rather than speed:
full-lattice arrays in the canonical layout (x fastest, see `synthetic`), np.roll for the
nearest-neighbour shifts and boolean masks for the block structure. It shares no code,
table or constant with the GPU library.

Modules and what the paper fixes for them (arxiv 1502.04025, Sec. 3.1 "Algorithm and
implementation overview"; the paper names the operator and the algorithms but prints no
formula, so the standard definitions are spelled out in each module):
  gamma    Euclidean Dirac matrices in a chiral basis
  lattice  indexing, shifts with antiperiodic time, parity, Schwarz blocks and colours
  wilson   Wilson-clover operator, clover term, block-restricted operator, dense matrix
  sap      even-odd block operator, minimal residual, Schwarz alternating procedure
  fgmres   flexible GMRES(m) with restarts and a true-residual check
  mg       two-level aggregation multigrid with the Schwarz procedure as smoother

Parity pins (closed forms, invariants, library special cases) live in tests/test_oracle*.py.
"""
from . import gamma, lattice, wilson, sap, fgmres, mg  # noqa: F401
