"""MI355X-native event-by-event proton CT reconstruction (arXiv:1707.05014).

The compute path is libpct.so (hand-written HIP kernels for gfx950, C ABI in
include/pct.h); ``paper_1707_05014_amd.api`` is its thin Python binding
(torch for device memory and streams).  Importing this package does not load
the library; the first API call does, and raises if it has not been built.
"""
