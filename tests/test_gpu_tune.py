"""The launch parameters and the autotuner on the GPU: every candidate value
of every parameter gives the same ciphertexts bit for bit (plan modes 0 and
4, a 2^16 ring so that the radix choice of the 2^16 transforms is exercised,
and a small ring), and the autotuner returns a choice whose output is
unchanged."""
import numpy as np
import pytest

from checks import log

pytestmark = pytest.mark.gpu

NAMES = {"ntt16_radix": [16, 2], "ntt_fp64": [1, 0], "ntt_row_vals": [16, 8], "ntt_tile": [2048, 4096, 8192], "ntt_group": [0, 64, 256, 1024],
         "ks_rot_batch": [4, 8, 16, 32], "ks_overlap": [0, 1], "ks_amounts": [1, 2, 4, 8, 16]}


@pytest.fixture
def restore():
    from paper_2306_09189_amd import hecnn
    saved = {k: hecnn.tune_get(k) for k in NAMES}
    yield
    for k, v in saved.items():
        hecnn.tune_set(k, v)


def exports(img):
    return [img.shard_export(u) for u in range(img.info()[4])]


@pytest.mark.parametrize("logn,shape", [(16, (4, 112, 112)), (11, (8, 16, 16))])
def test_every_candidate_bit_exact(restore, logn, shape):
    from paper_2306_09189_amd import hecnn
    if logn == 16:
        ctx = hecnn.Context(16, 24, 60, 50, 8, 60, 3, 50, device=0)
        level = 4
    else:
        ctx = hecnn.Context(11, 8, 60, 40, 3, 60, 3, 40, device=0)
        level = 6
    ctx.keygen(31)
    rng = np.random.default_rng(logn)
    x = rng.uniform(-1, 1, shape)
    w = rng.normal(0, 0.05, (shape[0], shape[0], 3, 3))
    img = ctx.image_encrypt(x, level, 9)
    plan = ctx.conv2d_plan(img, w)
    ctx.gen_rotation_keys(plan.steps())
    for mode in (0, 4):
        plan.set_mode(mode)
        ref = exports(plan.run(img))
        for name, vals in NAMES.items():
            keep = hecnn.tune_get(name)
            for v in vals:
                hecnn.tune_set(name, v)
                got = exports(plan.run(img))
                assert all((a == b).all() for a, b in zip(got, ref)), (mode, name, v)
            hecnn.tune_set(name, keep)
        log("mode %d: all candidates bit-exact" % mode)
    plan.set_mode(4)
    ref = exports(plan.run(img))
    rep = ctx.autotune_conv(plan, img, reps=2)
    log(rep)
    assert rep.startswith("chosen ")
    assert all((a == b).all() for a, b in zip(exports(plan.run(img)), ref))
