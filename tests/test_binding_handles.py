"""Handle lifetime in the Python binding (CPU only, with a stand-in for the
native library): a context is destroyed only after every handle of it is
freed, also when finalizers run in arbitrary order (cyclic garbage)."""
import gc

from paper_2306_09189_amd import hecnn


class FakeLib:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def f(*a):
            self.calls.append(name)
            return 0
        return f


def fake_ctx(h):
    ctx = object.__new__(hecnn.Context)
    ctx.h, ctx._live, ctx._close_pending = h, 0, False
    return ctx


def test_close_waits_for_handles(monkeypatch):
    fl = FakeLib()
    monkeypatch.setattr(hecnn, "_lib", fl)
    ctx = fake_ctx(1)
    a, b = hecnn.Image(ctx, 11), hecnn.Block(ctx, 12)
    borrowed = hecnn.Ciphertext(ctx, 13, owned=False)
    ctx.close()
    assert fl.calls == []
    del a
    assert fl.calls == ["hec_image_free"]
    del borrowed                       # never freed natively
    b.free()
    b.free()                           # idempotent
    assert fl.calls == ["hec_image_free", "he_block_free", "hec_ctx_destroy"]
    ctx.close()
    assert fl.calls.count("hec_ctx_destroy") == 1


def test_cyclic_garbage_any_order(monkeypatch):
    fl = FakeLib()
    monkeypatch.setattr(hecnn, "_lib", fl)
    for order in range(3):
        fl.calls.clear()
        ctx = fake_ctx(2)
        objs = [hecnn.Image(ctx, 21), hecnn.ConvPlan(ctx, 22), hecnn.Plaintext(ctx, 23, 0, 1.0)]
        holder = {"o": objs[order:] + [ctx] + objs[:order]}
        holder["self"] = holder
        del ctx, objs, holder
        gc.collect()
        assert fl.calls[-1] == "hec_ctx_destroy" and len(fl.calls) == 4, fl.calls


def test_context_without_handles(monkeypatch):
    fl = FakeLib()
    monkeypatch.setattr(hecnn, "_lib", fl)
    ctx = fake_ctx(3)
    ctx.close()
    assert fl.calls == ["hec_ctx_destroy"] and ctx.h is None
