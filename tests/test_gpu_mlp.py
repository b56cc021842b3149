"""Warm-start network kernels (BF16 MFMA GEMM, GELU, MSE, AdamW) through the
C ABI, against numpy and the FP64 CPU reference MLP."""
import numpy as np
import pytest

from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("M,N,K,ta,tb", [(70, 45, 37, False, False), (64, 64, 16, True, False),
                                          (130, 20, 100, False, True), (5, 300, 3, True, True)])
def test_gemm_bf16_layout_and_values(M, N, K, ta, tb):
    import torch
    from paper_2308_15407_amd import fdlb as F
    rng = np.random.default_rng(M + N + K)
    A = rng.normal(size=(M, K)).astype(np.float32)
    B = rng.normal(size=(K, N)).astype(np.float32)
    # storage order: A stored as [M][K] or transposed [K][M]; same for B
    As = A.T.copy() if ta else A
    Bs = B.T.copy() if tb else B
    sam, sak = (1, M) if ta else (K, 1)
    sbk, sbn = (1, K) if tb else (N, 1)
    dA = torch.from_numpy(bf16_bits(As).view(np.int16)).cuda()
    dB = torch.from_numpy(bf16_bits(Bs).view(np.int16)).cuda()
    dC = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    F.fdlb_mlp_gemm_bf16(dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, sam, sak, sbk, sbn, N,
                         torch.cuda.current_stream().cuda_stream)
    ref = bf16_round(A) @ bf16_round(B)
    got = dC.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) < 1e-5 * (1 + np.max(np.abs(ref)))


def test_gradient_matches_cpu_reference():
    from paper_2308_15407_amd.mlp import WarmStartNet, layer_shapes
    net = WarmStartNet(n_in=10, width=64, depth=3, n_out=40, max_batch=64, seed=3)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(50, 10)).astype(np.float32)
    t = rng.normal(size=(50, 40)).astype(np.float32)
    loss, g = net.loss_grad(x, t)
    p = net.get_params().astype(np.float64)
    shapes = layer_shapes(10, 64, 3, 40)
    # the GPU multiplies BF16-rounded weights and inputs
    pr = p.copy()
    off = 0
    for fin, fout in shapes:
        pr[off:off + fin * fout] = bf16_round(p[off:off + fin * fout]); off += fin * fout + fout
    Lr, gr = R.loss_grad(pr, shapes, bf16_round(x), t)
    print("loss gpu %.6f ref %.6f; grad rel err %.3e" % (loss, Lr, np.linalg.norm(g - gr) / np.linalg.norm(gr)))
    assert abs(loss - Lr) < 2e-2 * abs(Lr)
    assert np.linalg.norm(g - gr) < 3e-2 * np.linalg.norm(gr)
    off = 0
    for fin, fout in shapes:   # every layer's gradient points the same way
        n = fin * fout + fout
        a, b = g[off:off + n], gr[off:off + n]
        assert np.dot(a, b) > 0.995 * np.linalg.norm(a) * np.linalg.norm(b)
        off += n


def test_training_reduces_loss():
    from paper_2308_15407_amd.mlp import WarmStartNet
    net = WarmStartNet(n_in=10, width=128, depth=4, n_out=64, max_batch=256, seed=5)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(256, 10)).astype(np.float32)
    s = np.linspace(0, 1, 64)
    t = (np.sin(np.pi * np.outer(x[:, 0], s)) + x[:, 1:2] * s[None, :] ** 2).astype(np.float32)
    first = net.train_step(x, t, 1e-3, want_loss=True)
    for _ in range(300):
        net.train_step(x, t, 1e-3)
    last = net.train_step(x, t, 1e-3, want_loss=True)
    print("loss %.4e -> %.4e" % (first, last))
    assert last < 0.05 * first
