"""Host-only checks of the C ABI: it loads, exports every declared symbol, and its
integer tile plan matches the oracle's planner exactly.  No device calls."""
import ctypes
import os
import re
from ctypes import byref, c_int, c_size_t

import pytest

from oracle.net import min_halo as o_min_halo, vgg19, vgg19_tiny
from oracle.plan import make_plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nst.h")


@pytest.fixture(scope="module")
def L():
    from paper_2212_13459_amd import _lib
    return _lib.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nst_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("nst_style_grams", "nst_content_feats", "nst_loss_grad", "nst_plan", "nst_create"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_2212_13459_amd", "libnst.so"))
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_abi_version_and_strerror(L):
    assert L.nst_abi_version() == 2
    assert L.nst_strerror(0) == b"ok"
    assert L.nst_strerror(-7) == b"workspace too small"
    assert L.nst_strerror(-8) == b"non-finite value in an input"


def test_pool_avg_bits_must_be_pools(L):
    """nst_net_desc.pool_avg may only mark convs that a pool follows."""
    import ctypes
    from paper_2212_13459_amd.nst import vgg19_desc
    d = vgg19_desc(avg_pool=True)
    assert d.pool_avg == d.pool_after
    assert L.nst_min_halo(ctypes.byref(d)) == 155
    d.pool_avg = d.pool_after | 1   # conv1_1 is not followed by a pool
    assert L.nst_min_halo(ctypes.byref(d)) == -1


def test_min_halo_matches_oracle():
    from paper_2212_13459_amd.nst import min_halo, vgg19_desc
    assert min_halo(vgg19_desc()) == o_min_halo(vgg19()) == 155
    assert min_halo(vgg19_desc(tiny=True)) == o_min_halo(vgg19_tiny()) == 23


CASES = [(64, 64, 64, 23), (64, 64, 16, 0), (512, 512, 256, 155), (2048, 2048, 512, 155),
         (200, 328, 96, 155), (756, 1008, 1024, 155), (1512, 2016, 1024, 155), (3024, 4032, 1000, 155),
         (6048, 8064, 1024, 155), (4226, 5319, 1024, 155), (37, 53, 8, 0), (17, 5, 4, 7), (1, 1, 1, 0),
         (999, 7, 250, 300), (33, 1000, 1000, 3)]


@pytest.mark.parametrize("tiny", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_plan_matches_oracle_exactly(tiny, case):
    from paper_2212_13459_amd.nst import plan, vgg19_desc
    H, W, T, m = case
    net = vgg19_tiny() if tiny else vgg19()
    ours = plan(vgg19_desc(tiny=tiny), H, W, T, m)
    ref = make_plan(H, W, T, m, net.strides(), net.align())
    assert len(ours) == len(ref)
    for a, b in zip(ours, ref):
        assert a[:8] == (b.by0, b.by1, b.bx0, b.bx1, b.ey0, b.ey1, b.ex0, b.ex1)
        assert a[8] == b.own


def test_plan_capacity_and_errors(L):
    from paper_2212_13459_amd._lib import Tile
    from paper_2212_13459_amd.nst import vgg19_desc
    d = vgg19_desc()
    n = c_int(-1)
    arr = (Tile * 2)()
    assert L.nst_plan(byref(d), 512, 512, 128, 155, arr, 2, byref(n)) == -6   # ECAPACITY
    assert n.value == 16
    assert arr[1].bx0 == 128 and arr[1].bx1 == 256
    assert L.nst_plan(byref(d), 0, 512, 128, 155, arr, 2, byref(n)) == -2     # ESHAPE
    assert L.nst_plan(byref(d), 512, 512, 0, 155, arr, 2, byref(n)) == -2
    assert L.nst_plan(byref(d), 512, 512, 64, -1, arr, 2, byref(n)) == -2
    assert L.nst_plan(byref(d), 512, 512, 64, 0, None, 2, byref(n)) == -1      # EINVAL
    assert L.nst_plan(byref(d), 512, 512, 64, 0, arr, 2, None) == -1


def test_bad_descriptors_rejected(L):
    from paper_2212_13459_amd.nst import vgg19_desc
    d = vgg19_desc()
    d.c_in[0] = 4
    assert L.nst_min_halo(byref(d)) == -1
    d = vgg19_desc()
    d.c_out[3] = 100            # not 64 or a multiple of 128
    d.c_in[4] = 100
    assert L.nst_min_halo(byref(d)) == -1
    d = vgg19_desc()
    d.style_conv[1] = 0         # not increasing
    assert L.nst_min_halo(byref(d)) == -1
    d = vgg19_desc()
    d.style_conv[1] = 1         # style layer followed by a pool
    assert L.nst_min_halo(byref(d)) == -1
    d = vgg19_desc()
    d.n_style, d.content_conv = 0, -1
    assert L.nst_min_halo(byref(d)) == -1
    assert L.nst_min_halo(None) == -1


def test_workspace_sizes(L):
    from paper_2212_13459_amd.nst import vgg19_desc, workspace_bytes
    d = vgg19_desc()
    b1 = workspace_bytes(d, "bf16", 6048, 8064, 1024, 155, 1)
    b2 = workspace_bytes(d, "bf16", 6048, 8064, 1024, 155, 2)
    f1 = workspace_bytes(d, "fp32", 6048, 8064, 1024, 155, 1)
    assert 1.0e9 < b1 < 3.0e9 and b2 > b1 and f1 > b1
    out = c_size_t(0)
    assert L.nst_workspace_bytes(byref(d), 7, 64, 64, 64, 0, 1, byref(out)) == -1   # bad precision
    assert L.nst_workspace_bytes(byref(d), 0, 64, 64, 64, 0, 0, byref(out)) == -1   # batch < 1


def test_workspace_with_a_slot_per_tile():
    """tile_batch >= the tile count sizes one slot per tile (activations resident from
    Step 1 to Step 2): the same size for any such tile_batch, about nt slots."""
    from paper_2212_13459_amd.nst import plan, vgg19_desc, workspace_bytes
    d = vgg19_desc()
    nt = len(plan(d, 6048, 8064, 1024, 155))
    assert nt == 48
    all_tiles = workspace_bytes(d, "bf16", 6048, 8064, 1024, 155, nt)
    assert all_tiles == workspace_bytes(d, "bf16", 6048, 8064, 1024, 155, nt + 7)
    one = workspace_bytes(d, "bf16", 6048, 8064, 1024, 155, 1)
    two = workspace_bytes(d, "bf16", 6048, 8064, 1024, 155, 2)
    step = two - one          # one slot plus one tile's Gram-sum scratch
    assert (nt - 1) * step < all_tiles < nt * step
    # fewer tiles than the launch limit: the batch already holds every tile
    n_small = len(plan(d, 200, 328, 96, 155))
    assert workspace_bytes(d, "bf16", 200, 328, 96, 155, n_small) == \
        workspace_bytes(d, "bf16", 200, 328, 96, 155, 100)


def test_run_entry_points_validate_before_touching_the_device(L):
    assert L.nst_style_grams(None, None, 64, 64, 64, 0, None, None, 0, None) == -1
    assert L.nst_content_feats(None, None, 64, 64, 64, 0, None, None, 0, None) == -1
    assert L.nst_layer_feats(None, None, 64, 64, 64, 0, 0, None, None, 0, None) == -1
    assert L.nst_loss_grad(None, None, 64, 64, None, None, None, 1.0, 64, 0, 3, None, None, None, None, 0,
                           None) == -1
    L.nst_destroy(None)   # no-op
