"""The request loop (hec_server_*): two lanes with their own streams over the
resident keys and plans, admission by device memory, continuous batching.
Every result is the same, bit for bit, whether its request ran alone or in a
mix of requests of two models that overlap on the device and are batched;
each decrypts within 1e-5 of FP64; a request larger than the memory budget
is rejected, and requests are queued so that the admitted footprints never
exceed the budget."""
import numpy as np
import pytest

from checks import log
from oracle import he_layers as hl

pytestmark = pytest.mark.gpu


def exports(img):
    return [img.shard_export(u) for u in range(img.info()[4])]


@pytest.fixture(scope="module")
def setup():
    from paper_2306_09189_amd import hecnn
    ctx = hecnn.Context(11, 8, 60, 40, 3, 60, 3, 40, device=0)
    ctx.keygen(23)
    rng = np.random.default_rng(77)
    models = []
    # (shape, output channels): a one-shard image (channels duplicated) and a four-shard one
    for shape, co in (((4, 8, 8), 4), ((16, 16, 16), 8)):
        w = rng.normal(0, 0.1, (co, shape[0], 3, 3))
        like = ctx.image_encrypt(rng.uniform(-1, 1, shape), 6, 1)
        plan = ctx.conv2d_plan(like, w)
        plan.set_mode(4)
        ctx.gen_rotation_keys(plan.steps())
        conv = plan.run(like)
        ctx.gen_rotation_keys(ctx.avgpool_steps(conv))
        models.append((shape, w, plan, like))
    return ctx, models, rng


def reference(ctx, plan, img, pool_mode):
    return ctx.avgpool(plan.run(img), mode=pool_mode)


@pytest.mark.parametrize("pool_mode", [4, 2])
def test_server_alone_vs_mix(setup, pool_mode):
    """pool_mode 4: key-stationary pooling; 2: lazy ModDown pooling, which a
    batch takes over the shards of all its images in one fused launch per
    group of terms -- the same bits as each image pooled alone."""
    from paper_2306_09189_amd import hecnn
    ctx, models, rng = setup
    srv = hecnn.Server(ctx, lanes=2, max_batch=4, mem_budget=8 << 30)
    try:
        mids = [srv.add_model(plan, like, pool_mode=pool_mode) for (_, _, plan, like) in models]
        assert all(srv.footprint(m) > 0 for m in mids)
        # a pool of request images of both models
        reqs = []
        for i in range(12):
            m = 0 if i % 10 < 7 else 1
            shape, w, plan, like = models[m]
            x = rng.uniform(-1, 1, shape)
            reqs.append((m, x, ctx.image_encrypt(x, 6, 100 + i)))
        refs = [exports(reference(ctx, models[m][2], img, pool_mode)) for (m, x, img) in reqs]
        # alone: one request at a time on an idle server
        for j in (0, 7):
            m, x, img = reqs[j]
            out, lat = srv.poll(srv.submit(mids[m], img))
            got = exports(out)
            assert all((a == b).all() for a, b in zip(got, refs[j]))
        # the mix: everything submitted at once, so lanes overlap and batch
        ids = [srv.submit(mids[m], img) for (m, x, img) in reqs]
        for j, rid in enumerate(ids):
            m, x, img = reqs[j]
            out, lat = srv.poll(rid)
            got = exports(out)
            assert len(got) == len(refs[j])
            assert all((a == b).all() for a, b in zip(got, refs[j])), j
            w = models[m][1]
            fp = hl.ref_avgpool2x2(hl.ref_conv2d(x, w, 1))
            assert np.abs(out.decrypt() - fp).max() < 1e-5
        st = srv.stats()
        log("server stats", st)
        assert st["completed"] == 14 and st["rejected"] == 0
        assert st["batched_requests"] == 14 and st["batches"] < 14   # some requests evaluated together
        assert st["max_concurrent"] >= 2                             # lanes overlapped
        assert st["p99_ms"] >= st["p50_ms"] > 0 and st["req_per_s"] > 0
    finally:
        srv.stop()


def test_server_memory_admission(setup):
    from paper_2306_09189_amd import hecnn
    ctx, models, rng = setup
    probe = hecnn.Server(ctx, lanes=1, max_batch=1, mem_budget=8 << 30)
    fa = probe.footprint(probe.add_model(models[0][2], models[0][3], pool_mode=4))
    fb = probe.footprint(probe.add_model(models[1][2], models[1][3], pool_mode=4))
    probe.stop()
    assert fb > fa
    # room for one small request at a time; the large one never fits
    budget = int(fa * 1.5)
    srv = hecnn.Server(ctx, lanes=2, max_batch=4, mem_budget=budget)
    try:
        ma = srv.add_model(models[0][2], models[0][3], pool_mode=4)
        mb = srv.add_model(models[1][2], models[1][3], pool_mode=4)
        imgs = [ctx.image_encrypt(rng.uniform(-1, 1, models[0][0]), 6, 200 + i) for i in range(4)]
        big = ctx.image_encrypt(rng.uniform(-1, 1, models[1][0]), 6, 300)
        ids = [srv.submit(ma, im) for im in imgs]
        rb = srv.submit(mb, big)
        for rid in ids:
            srv.poll(rid)
        with pytest.raises(hecnn.HecError) as e:
            srv.poll(rb)
        assert e.value.status == hecnn.HEC_ENOMEM
        st = srv.stats()
        log("admission stats", st)
        assert st["peak_mem"] <= budget and st["max_concurrent"] == 1
        assert st["completed"] == 4 and st["rejected"] == 1
    finally:
        srv.stop()
