"""Multiscale L-BFGS driver (Algorithm 2): schedules on the CPU; a short run on the GPU
whose every evaluation goes through libnst (StyleEnergy)."""
import numpy as np
import pytest
import torch

import synth
from paper_2212_13459_amd.multiscale import history_schedule, iteration_schedule, scale_sizes


def test_spst_schedules():
    # Sec. 5.2: SPST 600 then 300 per scale; SPST-fast divides by 3 with a floor of 30
    assert iteration_schedule(4) == [600, 300, 300, 300]
    assert iteration_schedule(4, fast=True) == [600, 200, 66, 30]
    assert iteration_schedule(6, fast=True) == [600, 200, 66, 30, 30, 30]
    assert iteration_schedule(1) == [600]
    assert history_schedule(3) == [100, 10, 10]
    with pytest.raises(ValueError):
        iteration_schedule(0)


def test_scale_sizes_halve_from_the_full_size():
    # Fig. 1: 6048 x 8064 over four scales
    assert scale_sizes(6048, 8064, 4) == [(756, 1008), (1512, 2016), (3024, 4032), (6048, 8064)]
    assert scale_sizes(101, 75, 3) == [(25, 18), (50, 37), (101, 75)]


@pytest.mark.gpu
@pytest.mark.parametrize("cpu_last", [False, True])
def test_multiscale_run_lowers_the_energy_at_every_scale(cpu_last):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_13459_amd import Context
    from paper_2212_13459_amd.multiscale import style_transfer
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    nst = Context(ws, bs, "bf16")
    c = torch.from_numpy(synth.image(320, 384, 8.0, synth.SEED_CONTENT)).cuda()
    s = torch.from_numpy(synth.image(288, 288, 8.0, synth.SEED_STYLE)).cuda()
    x, rec = style_transfer(nst, c, s, n_scales=2, iterations=[10, 5], history=[100, 10], T=256,
                            w_mean=[1.0] * 5, w_std=[1.0] * 5, alpha=1e-3, cpu_last=cpu_last)
    print(f"[multiscale cpu_last={cpu_last}] {rec}", flush=True)
    assert x.shape == c.shape and bool(torch.isfinite(x).all())
    assert [r["size"] for r in rec] == [(160, 192), (320, 384)]
    for r in rec:
        assert r["evaluations"] >= r["iterations"] and np.isfinite(r["E_last"])
        assert r["E_last"] < r["E_first"]
    nst.close()


@pytest.mark.gpu
def test_texture_synthesis_from_noise():
    """Sec. 6.2: no content layer, alpha = 0, white-noise start, augmented style loss."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_13459_amd import Context
    from paper_2212_13459_amd.multiscale import texture_synthesis
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    nst = Context(ws, bs, "bf16", with_content=False)
    v = torch.from_numpy(synth.image(256, 256, 8.0, synth.SEED_STYLE)).cuda()
    x, rec = texture_synthesis(nst, v, 384, 320, n_scales=3, iterations=[10, 5, 5], history=[100, 10, 10], T=256,
                               w_mean=[1.0] * 5, w_std=[1.0] * 5, seed=7)
    print(f"[texture] {rec}", flush=True)
    assert x.shape == (3, 384, 320) and bool(torch.isfinite(x).all())
    assert [r["size"] for r in rec] == [(96, 80), (192, 160), (384, 320)]
    for r in rec:
        assert r["E_last"] < r["E_first"]
    nst.close()
