"""The training gradient without allocation (mlp_loss_grad_noalloc, the
library's fixed per-GPU scratch) against mlp_loss_grad with a caller
workspace: the same kernels, so gradient and loss agree bit for bit.  Two
calls in a row, the second with a smaller, ragged batch; limits rejected on
the host before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")


def _pair(W, B, seed):
    from paper_2011_00459_amd.devmem import DeviceArray
    rng = np.random.default_rng(seed)
    F = DeviceArray.from_host(rng.normal(0, 1, (B, 12)).astype(np.float32))
    Y = DeviceArray.from_host(rng.normal(0, 1, (B, 3)).astype(np.float32))
    ns = T.mlp_grad_scratch_floats(B)
    S, G1, L1 = DeviceArray(ns), DeviceArray(T.MLP_TRAINABLE), DeviceArray(1)
    G2, L2 = DeviceArray(T.MLP_TRAINABLE), DeviceArray(1)
    T.mlp_loss_grad(W.ptr, F.ptr, Y.ptr, B, G1.ptr, L1.ptr, S.ptr, ns)
    T.mlp_loss_grad_noalloc(W.ptr, F.ptr, Y.ptr, B, G2.ptr, L2.ptr)
    out = G1.get(), L1.get(), G2.get(), L2.get()
    for a in (F, Y, S, G1, L1, G2, L2):
        a.free()
    return out


def test_noalloc_gradient_equals_the_workspace_gradient():
    from paper_2011_00459_amd import learn as LN
    from paper_2011_00459_amd.devmem import DeviceArray
    W = DeviceArray.from_host(LN.flatten(LN.init_weights(3)))
    for B, seed in ((T.MLP_NOALLOC_MAX_BATCH, 1), (1000 + 17, 2)):
        g1, l1, g2, l2 = _pair(W, B, seed)
        assert np.all(np.isfinite(g1)) and np.any(g1 != 0)
        assert np.array_equal(g1, g2), (B, np.max(np.abs(g1 - g2)))
        assert np.array_equal(l1, l2), (B, l1, l2)


def test_noalloc_gradient_rejects_sizes_beyond_its_scratch():
    from paper_2011_00459_amd.devmem import DeviceArray
    W = DeviceArray(T.MLP_PARAMS)
    F, Y, G, L = DeviceArray((4, 12)), DeviceArray((4, 3)), DeviceArray(T.MLP_TRAINABLE), DeviceArray(1)
    for B, code in ((T.MLP_NOALLOC_MAX_BATCH + 1, T.TR_E_CAPACITY), (0, T.TR_E_INVAL)):
        with pytest.raises(T.TerrainError) as ei:
            T.mlp_loss_grad_noalloc(W.ptr, F.ptr, Y.ptr, B, G.ptr, L.ptr)
        assert ei.value.code == code
