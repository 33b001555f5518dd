"""FP64 CPU oracle for the localized style-transfer loss and gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library.

What it computes (Galerne, Raad, Lezama, Morel, "Scaling Painting Style
Transfer", Sec. 3.1 and Sec. 4, Algorithm 1, Table 1):

* ``net``   : VGG-19 prefix geometry, pooling strides, receptive-field closed form
* ``ops``   : 3x3 zero-padded cross-correlation, its adjoint, 2x2/2 floor max pool
              and its backward, written as plain NumPy float64
* ``loss``  : whole-image forward, Gram matrices G = V^T V / n_p (Sec. 3.1),
              transfer energy (Eq. 1-3) and the augmented style loss with channel
              means and stds (Eq. 5), feature-loss seeds (Table 1, all four rows)
              and the hand-derived backward
* ``plan``  : the tile / halo / owned-feature plan (blocks with margin, Sec. 4.1)
* ``tiled`` : the two-pass localized loss and gradient (Algorithm 1)
* ``naive`` : pure-loop conv, pool and Gram for tiny pins

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, brute force, invariants and a library routine (torch CPU float64
autograd used as a checker only).  The energy value itself has no printed
worked example in the paper (parity of the value unpinned by a paper number;
pinned by the invariants and the independent cross-checks).
"""
from .net import NetSpec, vgg19, vgg19_tiny, receptive_fields, min_halo  # noqa: F401
from .loss import forward, gram, energy_terms, loss_grad, content_features, MeanStd, style_stats  # noqa: F401
from .plan import make_plan  # noqa: F401
from .tiled import tiled_loss_grad, tiled_style_grams, tiled_style_stats, tiled_content_features  # noqa: F401
