"""Learned warm start on the GPU against the FP64 oracle.

  - the 12 features of every contact match the oracle's (same state, same cache);
  - network forward: FP32 kernel within 1e-5, BF16 MFMA kernel within ~1e-2 of
    the oracle's FP64 forward (same seeded weights);
  - FP32 gradients of the training kernels within 1e-4 (relative, per tensor)
    of the oracle's FP64 gradients on the same minibatch;
  - a LEARNED step (FP32 inference, and BF16 inference on the matrix cores
    against the oracle's network at that precision) takes the same start
    decision as the oracle and matches its velocities to the usual one-step bar.
"""
import ctypes as C

import numpy as np
import pytest

import pyoracle as O
from helpers import settled_column, vel_tol, with_

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")


class DevBuf:
    """A device buffer from the HIP runtime (float32)."""

    _hip = None

    def __init__(self, host):
        if DevBuf._hip is None:
            DevBuf._hip = C.CDLL("libamdhip64.so.7")
        self.host = np.ascontiguousarray(host, dtype=np.float32)
        self.nbytes = max(self.host.nbytes, 4)
        p = C.c_void_p()
        assert DevBuf._hip.hipMalloc(C.byref(p), C.c_size_t(self.nbytes)) == 0
        self.ptr = p.value
        assert DevBuf._hip.hipMemcpy(C.c_void_p(self.ptr), self.host.ctypes.data_as(C.c_void_p),
                                     C.c_size_t(self.host.nbytes), 1) == 0

    def get(self):
        out = np.empty_like(self.host)
        DevBuf._hip.hipDeviceSynchronize()
        assert DevBuf._hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(self.ptr),
                                     C.c_size_t(self.host.nbytes), 2) == 0
        return out

    def free(self):
        DevBuf._hip.hipFree(C.c_void_p(self.ptr))


def random_weights(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    w = dict(W1=rng.normal(0, 0.35, (64, 12)) * scale, b1=rng.normal(0, 0.1, 64), W2=rng.normal(0, 0.15, (64, 64)),
             b2=rng.normal(0, 0.1, 64), W3=rng.normal(0, 0.1, (3, 64)), b3=np.array([0.3, 0.0, 0.0]),
             in_scale=rng.uniform(0.5, 1.5, 12))
    return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in w.items()}


def flat(w):
    return np.concatenate([w[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3", "in_scale")]).astype(np.float32)


def test_features_match_oracle_first_and_second_step():
    spec = with_(settled_column(seed=11, n=500, footprint=0.7), warm_start="prev", max_sweeps=80)
    g = T.scene_from_specs(spec)
    g.set_learn_capture(True)
    o = O.OracleScene(spec)
    for step in range(2):
        fo, fro, so = o.features()
        g.step(1)
        fg, _ = g.get_learn_samples(0)
        o.step()
        assert fg.shape == fo.shape and len(fo) > 500
        scale = np.maximum(np.max(np.abs(fo), axis=0), 1e-3)
        err = np.max(np.abs(fg - fo), axis=0) / scale
        # exact on the first step (identical state); FP32-vs-FP64 state after it
        bound = 2e-5 if step == 0 else 5e-3
        assert np.all(err[[0, 6, 7, 8, 9, 10, 11]] <= 2e-5), (step, err)
        assert np.all(err <= bound), (step, err)


def test_network_forward_fp32_bf16_against_oracle():
    w = random_weights(3)
    rng = np.random.default_rng(4)
    feat = rng.normal(0, 1.0, (1000, 12)).astype(np.float32)
    ref = O.mlp_forward(w, feat.astype(np.float64))
    W = DevBuf(flat(w))
    F = DevBuf(feat)
    out32, out16 = DevBuf(np.zeros((1000, 3))), DevBuf(np.zeros((1000, 3)))
    T.mlp_forward(W.ptr, F.ptr, 1000, out32.ptr, bf16=False)
    T.mlp_forward(W.ptr, F.ptr, 1000, out16.ptr, bf16=True)
    y32, y16 = out32.get(), out16.get()
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(y32 - ref)) <= 1e-5 * scale
    e16 = np.max(np.abs(y16 - ref)) / scale
    assert e16 <= 3e-2, e16
    assert np.mean(np.abs(y16 - ref)) / scale <= 5e-3
    for b in (W, F, out32, out16):
        b.free()


def _bf16(a):
    """Round FP32 values to BF16 (nearest, ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [1000, 70001])
def test_bf16_forward_matches_its_rounding_model(n):
    # the same rounding as the MFMA path (inputs x scale, the weight matrices
    # and both hidden layers in BF16, FP32 sums and biases) evaluated in FP64:
    # only summation order, exp and the reciprocal differ, so a misplaced
    # operand element or a wrong tile shows as an O(1) error
    w = random_weights(5)
    rng = np.random.default_rng(6)
    feat = rng.normal(0, 1.0, (n, 12)).astype(np.float32)
    Wf = flat(w)
    F, W, out = DevBuf(feat), DevBuf(Wf), DevBuf(np.zeros((n, 3)))
    T.mlp_forward(W.ptr, F.ptr, n, out.ptr, bf16=True)
    y = out.get()
    sc = np.asarray(w["in_scale"], dtype=np.float32)
    x = _bf16(feat * sc)
    z1 = x @ _bf16(w["W1"]).T + np.asarray(w["b1"], dtype=np.float64)
    h1 = _bf16((z1 / (1.0 + np.exp(-z1))).astype(np.float32))
    z2 = h1 @ _bf16(w["W2"]).T + np.asarray(w["b2"], dtype=np.float64)
    h2 = _bf16((z2 / (1.0 + np.exp(-z2))).astype(np.float32))
    ref = h2 @ _bf16(w["W3"]).T + np.asarray(w["b3"], dtype=np.float64)
    scale = np.max(np.abs(ref))
    err = np.abs(y - ref) / scale
    assert np.max(err) <= 2e-3, np.max(err)
    assert np.mean(err) <= 1e-4, np.mean(err)
    for b in (F, W, out):
        b.free()


def test_training_gradients_match_oracle():
    w = random_weights(5)
    rng = np.random.default_rng(6)
    B = 200  # several training blocks and a ragged tail
    feat = rng.normal(0, 1.0, (B, 12)).astype(np.float32)
    lab = rng.normal(0, 1.0, (B, 3)).astype(np.float32)
    loss_ref, g_ref = O.mlp_loss_grad(w, feat.astype(np.float64), lab.astype(np.float64))
    W, F, L = DevBuf(flat(w)), DevBuf(feat), DevBuf(lab)
    G = DevBuf(np.zeros(T.MLP_TRAINABLE))
    LS = DevBuf(np.zeros(1))
    ns = T.mlp_grad_scratch_floats(B)
    S = DevBuf(np.zeros(ns))
    T.mlp_loss_grad(W.ptr, F.ptr, L.ptr, B, G.ptr, LS.ptr, S.ptr, ns)
    g = G.get()
    assert LS.get()[0] == pytest.approx(loss_ref, rel=1e-5)
    o = 0
    for k, shp in (("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (3, 64)), ("b3", (3,))):
        sz = int(np.prod(shp))
        gg = g[o:o + sz].reshape(shp)
        o += sz
        rel = np.linalg.norm(gg - g_ref[k]) / max(np.linalg.norm(g_ref[k]), 1e-30)
        assert rel <= 1e-4, (k, rel)
    # one Adam step moves every weight against its gradient by at most lr
    M, V = DevBuf(np.zeros(T.MLP_TRAINABLE)), DevBuf(np.zeros(T.MLP_TRAINABLE))
    w0 = W.get()
    T.mlp_adam_step(W.ptr, G.ptr, M.ptr, V.ptr, 1e-3, 1)
    w1 = W.get()
    d = w1[:T.MLP_TRAINABLE] - w0[:T.MLP_TRAINABLE]
    big = np.abs(g) > 1e-6
    assert np.all(np.sign(d[big]) == -np.sign(g[big]))
    assert np.max(np.abs(d)) <= 1e-3 + 4 * np.spacing(np.float32(np.max(np.abs(w0))))
    assert np.array_equal(w1[T.MLP_TRAINABLE:], w0[T.MLP_TRAINABLE:])
    for b in (W, F, L, G, LS, S, M, V):
        b.free()


@pytest.mark.parametrize("seed,scale", [(7, 1.0), (8, 0.0)])
def test_learned_step_matches_oracle(seed, scale):
    w = random_weights(seed, scale)
    spec = with_(settled_column(seed=12, n=400, footprint=0.6), warm_start="learned", max_sweeps=60)
    g = T.scene_from_specs(spec)
    g.set_mlp_weights(flat(w))
    g.set_learned_precision(False)
    o = O.OracleScene(spec, mlp=w)
    for k in range(2):
        st = g.step(1)[0]
        oo = o.step()
        keys, _ = g.get_contacts(0)
        assert np.array_equal(keys, oo["keys"])
        assert st["fallback_used"] == oo["fallback_used"], (k, st, oo["r1"])
        assert st["sweeps"] == oo["sweeps"]
        p = g.get_particles(0)
        assert np.max(np.abs(p["v"] - o.v)) <= vel_tol(o.v) * (1 + 4 * k)


@pytest.mark.parametrize("seed,scale,kept", [(7, 1.0, None), (8, 0.0, None), (7, 0.2, True)])
def test_bf16_learned_step_matches_the_oracles_bf16_network(seed, scale, kept):
    # BF16 inference on the matrix cores against the oracle's network at the
    # same precision (bfloat16 inputs, weight matrices and hidden layers, wide
    # sums): the same start decision and velocities to the one-step bar.  In
    # the kept case the first step has no previous impulses (the fallback is
    # the cold start, whose first residual is 1) and the network predicts a
    # compressive normal impulse, so the learned start is kept on both sides.
    w = random_weights(seed, scale)
    if kept:
        w["b3"] = np.array([1.0, 0.0, 0.0])
    spec = with_(settled_column(seed=12, n=400, footprint=0.6), warm_start="learned", max_sweeps=60)
    g = T.scene_from_specs(spec)
    g.set_mlp_weights(flat(w))
    g.set_learned_precision(True)
    o = O.OracleScene(spec, mlp=dict(w, bf16=True))
    for k in range(1 if kept else 2):
        st = g.step(1)[0]
        oo = o.step()
        keys, _ = g.get_contacts(0)
        assert np.array_equal(keys, oo["keys"])
        assert st["fallback_used"] == oo["fallback_used"], (k, st, oo["r1_trial"])
        if kept:
            assert oo["fallback_used"] == 0 and oo["learned_used"] == 1
        assert st["sweeps"] == oo["sweeps"]
        p = g.get_particles(0)
        assert np.max(np.abs(p["v"] - o.v)) <= vel_tol(o.v) * (1 + 4 * k)


def test_nonfinite_network_falls_back():
    w = random_weights(9)
    w["b3"] = np.array([np.float32(1e38)] * 3, dtype=np.float64)
    w["W3"] = np.full((3, 64), 1e38)
    spec = with_(settled_column(seed=13, n=300, footprint=0.5), warm_start="learned", max_sweeps=30)
    g = T.scene_from_specs(spec)
    g.set_mlp_weights(flat(w))
    st = g.step(1)[0]
    assert st["fallback_used"] == 1
    assert np.all(np.isfinite(g.get_particles(0)["v"]))


def test_samples_need_a_step_that_wrote_features():
    # a step writes the learned start's inputs only when it runs the network
    # or capture is on; without them get_learn_samples is refused
    spec = with_(settled_column(seed=12, n=300, footprint=0.6), warm_start="prev", max_sweeps=20)
    g = T.scene_from_specs(spec)
    g.step(1)
    with pytest.raises(T.TerrainError) as ei:
        g.get_learn_samples(0)
    assert ei.value.code == T.TR_E_STATE
    g.set_learn_capture(True)
    g.step(1)
    f, lab = g.get_learn_samples(0)
    assert len(f) > 0 and f.shape[1] == 12 and lab.shape[1] == 3
    g.set_learn_capture(False)
    g.step(1)
    with pytest.raises(T.TerrainError):
        g.get_learn_samples(0)
