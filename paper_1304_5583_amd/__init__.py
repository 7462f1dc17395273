"""DFC-LRR on MI355X (gfx950): hand-written HIP kernels behind a C ABI.

``binding`` wraps the shared library (include/lrr.h); ``datagen`` draws the
seeded synthetic inputs.  Build the library with
``python -m paper_1304_5583_amd.build``.
"""
