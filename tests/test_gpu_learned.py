"""GPU checks of the learned schedule cost model: the MLP kernels against the
float64 oracle (forward in FP32 and BF16, loss gradient, Adam step), training
that learns, and learned schedule choice: the count never changes and the
chosen schedule is not slower than the analytic model's on held-out patterns
and graphs."""

import os
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from oracle import patterns as P
from paper_1911_12877_amd import gz, learn, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gz.library()
    yield


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _case(seed, n=300, D=gz.FEATURES, H=128):
    rng = np.random.Generator(np.random.PCG64(seed))
    Pm = learn.init_params(D, H, seed)
    Pm[H * D:] = rng.normal(0, 0.3, Pm.size - H * D).astype(np.float32)
    X = rng.normal(0, 1, (n, D)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    return Pm, X, t, D, H


def test_mlp_forward_fp32_and_bf16():
    Pm, X, t, D, H = _case(1)
    y = gz.mlp_forward(_t(Pm), _t(X), H).cpu().numpy()
    want, _ = omlp.forward(Pm, X, D, H)
    # FP32 accumulation of D = 108 and H = 128 products of O(1) terms
    assert np.allclose(y, want, rtol=1e-5, atol=1e-4)
    yb = gz.mlp_forward(_t(Pm), _t(X), H, bf16=True).cpu().numpy()
    wantb, _ = omlp.forward(Pm, X, D, H, bf16_mode=True)
    # same BF16 operands, FP32 sums in another order
    assert np.allclose(yb, wantb, rtol=1e-4, atol=1e-3)
    # BF16 against FP32: 8-bit mantissas, errors of a few 2^-8 relative
    assert np.max(np.abs(yb - want)) < 0.05 * max(1.0, np.max(np.abs(want)))


def test_mlp_loss_gradient():
    Pm, X, t, D, H = _case(2)
    loss, g = gz.mlp_loss_grad(_t(Pm), _t(X), _t(t), H)
    wl, wg = omlp.loss_grad(Pm, X, t, D, H)
    assert abs(loss - wl) <= 1e-4 * max(1.0, wl)
    g = g.cpu().numpy()
    scale = np.max(np.abs(wg))
    assert np.max(np.abs(g - wg)) <= 1e-4 * scale


def test_mlp_adam_step():
    import torch
    Pm, X, t, D, H = _case(3)
    rng = np.random.Generator(np.random.PCG64(4))
    G = rng.normal(0, 1, Pm.size).astype(np.float32)
    m = rng.normal(0, 0.1, Pm.size).astype(np.float32)
    v = np.abs(rng.normal(0, 0.1, Pm.size)).astype(np.float32)
    Pd, Gd, md, vd = _t(Pm), _t(G), _t(m), _t(v)
    gz.mlp_adam(Pd, Gd, md, vd, D, H, 1e-2, 5)
    wp, wm, wv = omlp.adam(Pm.astype(np.float64), G, m, v, 1e-2, 5)
    assert np.allclose(Pd.cpu().numpy(), wp, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), wm, rtol=1e-5, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), wv, rtol=1e-5, atol=1e-7)


def test_training_learns_a_smooth_target():
    rng = np.random.Generator(np.random.PCG64(5))
    D = gz.FEATURES
    X = rng.normal(0, 1, (512, D)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * np.abs(X[:, 3])).astype(np.float32)
    Pm, losses = learn.train(X, t - t.mean(), H=64, steps=800, lr=3e-3)
    assert losses[-1] < 0.25 * losses[0]


def _model_or_skip():
    if not os.path.exists(learn.MODEL_PATH):
        pytest.skip("no trained cost model bundled")
    return learn.install()


def test_learned_choice_keeps_counts():
    _model_or_skip()
    e = synth.chung_lu_edges(3000, 2.3, 10.0, 881, cap=True)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    for nm in ["house", "diamond", "tailed_triangle", "k5e", "c5", "c6chord03"]:
        a = np.array(P.named(nm), np.uint8)
        s = gz.compile_pattern_graph(G, a, True, gz.SCHED_LEARNED)
        assert s.info()["order"] in [o for o, _ in gz.enumerate_schedules(a, True)]
        assert gz.count(G, s) == oracle.count(O, P.named(nm), True)


def test_learned_not_slower_than_analytic_on_held_out():
    """Held-out patterns (never in the training corpus) on graphs not used
    for training: total kernel time of the learned choices against the
    analytic model's choices, counts identical."""
    _model_or_skip()
    cases = []
    for gname, e in (("rmat10", synth.rmat_edges(10, 16, seed=8801)),
                     ("cl4000", synth.chung_lu_edges(4000, 2.3, 10.0, 8802, cap=True))):
        G = gz.load_edges(*e)
        for nm, a in learn.held_out_patterns().items():
            sa = gz.compile_pattern(a, True)
            sl = gz.compile_pattern_graph(G, a, True, gz.SCHED_LEARNED)
            print(f"timing {gname} {nm}", file=sys.stderr, flush=True)
            ca, ta = learn.time_schedule(G, sa, reps=3)
            cl, tl = learn.time_schedule(G, sl, reps=3)
            assert ca == cl
            cases.append((gname, nm, ta, tl))
            print(f"{gname} {nm}: analytic {sa.info()['order']} {ta:.2f} ms, learned "
                  f"{sl.info()['order']} {tl:.2f} ms", file=sys.stderr, flush=True)
    ta = sum(c[2] for c in cases)
    tl = sum(c[3] for c in cases)
    assert tl <= 1.05 * ta, (ta, tl)
    # and case by case, within timing noise (10% and half a millisecond)
    for gname, nm, a, l in cases:
        assert l <= 1.10 * a + 0.5, (gname, nm, a, l)
