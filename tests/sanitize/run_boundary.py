"""Runs the host-side boundary tests (tests/test_boundary.py) against the
library named on the command line: a build of libboba.so whose host code is
instrumented with AddressSanitizer and UndefinedBehaviorSanitizer.  Started by
tests/test_sanitizers.py in a process with the sanitizer runtime preloaded.
Every call either is a host-only query or fails validation before anything is
enqueued, so no GPU is needed."""
import inspect
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.join(ROOT, "tests")]

from paper_2306_10410_amd import boba  # noqa: E402

boba.LIB_PATH = sys.argv[1]
boba._lib = None
lib = boba.load()

import test_boundary  # noqa: E402

ran = 0
for name in sorted(dir(test_boundary)):
    if not name.startswith("test_"):
        continue
    fn = getattr(test_boundary, name)
    fn(lib) if "lib" in inspect.signature(fn).parameters else fn()
    ran += 1
# beyond the boundary tests: every workspace query over a spread of sizes
for n in (0, 1, 31, 32768, 32769, (1 << 20) + 3, 1 << 24, (1 << 25) + 7, (1 << 31) - 1):
    for m in (0, 1, 5, 1 << 20, (1 << 28) + 1, (1 << 31) - 1):
        for q in ("boba_reorder_workspace", "boba_reorder_relabel_workspace", "boba_relabel_bucketed_workspace",
                  "coo_to_csr_workspace", "spmv_csr_workspace", "boba_nbr_workspace", "boba_pagerank_workspace",
                  "boba_bin_by_dst_workspace"):
            getattr(lib, q)(n, m)
print(f"boundary ok: {ran} tests", flush=True)
