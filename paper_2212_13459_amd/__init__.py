"""Localized (tiled, two-pass) style-transfer loss and gradient on MI355X (gfx950).

The compute path is libnst.so (hand-written HIP kernels behind a C ABI, declared in
include/nst.h).  ``nst`` is the thin Python binding; it refuses to run without the
built library.
"""
from .nst import (NST_BOTH, NST_CHECK_FINITE, NST_RESIDENT, NST_STEP1, NST_STEP2, NST_STRICT_HALO,  # noqa: F401
                  Context, MeanStdTerms, StyleEnergy, min_halo, plan, vgg19_desc, workspace_bytes)
