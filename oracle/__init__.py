"""FP64 CPU oracle for TUCKET range queries (Qiu et al., PVLDB 17(13), 2024).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or
links anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's ``cpu_baseline`` leg use it.  It shares no code with the
HIP library (no headers, helpers, tables or generators) and imports nothing
from it.

It is a plain, slow, literal implementation of the paper:
  * tensor_ops  -- vec / mat_n / mode-n product / Frobenius norm (App. A);
  * tucker      -- Tucker-ALS (HOOI) with HOSVD init (Sec. 2, Eq. "als-mat");
  * tree        -- stream segment tree: Alg. "append", Alg. "insert",
                   Alg. "recall" (Secs. 4.2, 5.1, 6.2);
  * stitch      -- partial-hit approximation (Eq. "partial-tucker") and
                   Alg. "stitch" with Z^(1) materialised (Sec. 5.2);
  * evaluate    -- reconstruction error, subspace angles, brute-force hit
                   sets and brute-force Tucker-ALS for the checks.

Parity status: every function is pinned by ``tests/test_oracle_*.py``
against closed forms, the paper's worked example (Fig. "illust"), brute
force or library routines, except the stitched values on noisy data at
non-full rank, which no printed number fixes ("parity unpinned" beyond the
identity, invariant and special-case checks listed there).
"""

from . import tensor_ops, tucker, tree, stitch, evaluate  # noqa: F401
from .tree import StreamSegmentTree  # noqa: F401
