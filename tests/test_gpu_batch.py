"""Batches of layer evaluations as one launch (hec_batch_*): images at
different levels (so different limb counts) each through its convolution and
rescale, run eagerly and as one captured HIP graph.  The graph's outputs
equal the eager ones bit for bit on the first launch and on replays with other
eager work in between; one item is also compared with the oracle."""
import numpy as np
import pytest

from checks import log
from oracle import ckks
from oracle import he_layers as hl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring():
    from paper_2306_09189_amd import hecnn
    ctx = hecnn.Context(11, 8, 60, 40, 3, 60, 3, 40, device=0)
    prm = ckks.Params(11, [60] + [40] * 8, [60] * 3, 3)
    ctx.keygen(17)
    return ctx, prm, ckks.Oracle(prm, 17)


def exports(img):
    return [img.shard_export(u) for u in range(img.info()[4])]


def test_batch_graph_equals_eager(ring):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = ring
    rng = np.random.default_rng(9)
    cases = [((4, 16, 16), 8, 0), ((8, 16, 16), 4, 2), ((2, 32, 32), 6, 4), ((16, 16, 16), 3, 4), ((4, 8, 8), 7, 3)]
    b = ctx.batch()
    inst = []
    for i, (shape, level, mode) in enumerate(cases):
        x = rng.uniform(-1, 1, shape)
        w = rng.normal(0, 0.1, (shape[0], shape[0], 3, 3))
        img = ctx.image_encrypt(x, level, 500 + i)
        plan = ctx.conv2d_plan(img, w)
        plan.set_mode(mode)
        ctx.gen_rotation_keys(plan.steps())
        assert b.add(plan, img) == i
        inst.append((x, w, img, plan, level))
    assert len(b) == len(cases)
    b.launch(graph=False)
    eager = [exports(b.output(i)) for i in range(len(cases))]
    for i, (x, w, img, plan, level) in enumerate(inst):
        out = b.output(i)
        assert all(out.shard_info(u)[0] == level - 1 for u in range(out.info()[4]))
        assert np.abs(out.decrypt() - hl.ref_conv2d(x, w, 1)).max() < 1e-5
    # item 0 (mode 0) against the oracle
    x, w, img, plan, level = inst[0]
    lay = hl.natural_layout(prm.N, *x.shape)
    cts = [o.encrypt(o.encode(v, level, 2.0 ** 40), seed=500, index=u) for u, v in enumerate(hl.pack(x, lay))]
    oc, ol = hl.conv2d(hl.CkksBackend(o), cts, lay, w, pad=1)
    for u in range(len(oc)):
        assert (eager[0][u] == oc[u].data).all()
    for rep in range(3):
        log("graph launch %d" % rep)
        b.launch(graph=True)
        got = [exports(b.output(i)) for i in range(len(cases))]
        for i in range(len(cases)):
            for u in range(len(eager[i])):
                assert (got[i][u] == eager[i][u]).all(), (rep, i, u)
        # other eager work on the context between replays
        _ = inst[1][3].run(inst[1][2])
        b.launch(graph=False)
        for i in range(len(cases)):
            assert all((a == e).all() for a, e in zip(exports(b.output(i)), eager[i]))
    with pytest.raises(hecnn.HecError) as e:
        b.add(inst[0][3], inst[0][2])
    assert e.value.status == hecnn.HEC_EBUSY


def test_batch_replay_reads_current_inputs(ring):
    """Two batches sharing one plan, each with its own input image, record and
    replay independently: every replay gives its own input's convolution,
    the same bits as before."""
    ctx, prm, o = ring
    rng = np.random.default_rng(10)
    x1, x2 = rng.uniform(-1, 1, (4, 16, 16)), rng.uniform(-1, 1, (4, 16, 16))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    i1, i2 = ctx.image_encrypt(x1, 5, 1), ctx.image_encrypt(x2, 5, 2)
    plan = ctx.conv2d_plan(i1, w)
    ctx.gen_rotation_keys(plan.steps())
    b1, b2 = ctx.batch(), ctx.batch()
    b1.add(plan, i1)
    b2.add(plan, i2)
    b1.launch(graph=True)
    b2.launch(graph=True)
    r1, r2 = b1.output(0).decrypt(), b2.output(0).decrypt()
    assert np.abs(r1 - hl.ref_conv2d(x1, w, 1)).max() < 1e-5
    assert np.abs(r2 - hl.ref_conv2d(x2, w, 1)).max() < 1e-5
    b1.launch(graph=True)
    assert np.abs(b1.output(0).decrypt() - r1).max() == 0


def test_batch_graph_with_two_streams(ring):
    """With hoisted rotation batches on two streams (ks_overlap=1) the eager
    launch forks and joins a second stream; the recorded graph keeps to the
    one stream it captures.  Both give the same bits, also on replays."""
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = ring
    saved = hecnn.tune_get("ks_overlap")
    hecnn.tune_set("ks_overlap", 1)
    try:
        rng = np.random.default_rng(19)
        x = rng.uniform(-1, 1, (4, 16, 16))
        w = rng.normal(0, 0.1, (4, 4, 3, 3))
        img = ctx.image_encrypt(x, 8, 700)
        plan = ctx.conv2d_plan(img, w)
        plan.set_mode(0)      # 35 hoisted rotations: more than one batch (32 by default)
        ctx.gen_rotation_keys(plan.steps())
        b = ctx.batch()
        b.add(plan, img)
        b.launch(graph=False)
        eager = exports(b.output(0))
        hecnn.tune_set("ks_overlap", 0)
        single = exports(plan.run(img))
        hecnn.tune_set("ks_overlap", 1)
        assert all((a == s).all() for a, s in zip(eager, single))
        for rep in range(3):
            b.launch(graph=True)
            assert all((a == e).all() for a, e in zip(exports(b.output(0)), eager)), rep
            _ = plan.run(img)   # eager two-stream work between replays
    finally:
        hecnn.tune_set("ks_overlap", saved)
