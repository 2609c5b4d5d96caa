"""Oracle: a plain, slow, float64 CPU implementation of direct BPA and HHFFBPA.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the GPU
library (``paper_2506_23568_amd``) and never imports it; the two meet only in
the seeded input generators of ``workloads``.

Modules
  geometry  analytic SDC/LLT maps of one subarray (Sec. III)
  plan      subarray tree, sampling grids and their preimages (Sec. IV-A)
  hhffbp    the factorised pipeline and eq. (4) direct BPA (Sec. II-A, IV-A)
  native    ctypes access to the C sums (oracle.c)
  brute     pure-Python loops for tiny cases

Parity unpinned: the exact HHFFBPA values of the paper's own implementation
(its interpolation kernel, oversampling and grid extent are not published);
the oracle's HHFFBPA is pinned to eq. (4) through error bounds and special
cases instead (tests/test_oracle_hhffbp.py).
"""
