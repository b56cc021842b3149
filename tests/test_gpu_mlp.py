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


# strides that are not multiples of 8 take the scalar loads; (200, 136, 72) and
# (64, 128, 40) read A and B with 16-byte loads along k, (96, 256, 264) along
# m and n, with ragged tile and depth edges; the two largest take the 128 x 128
# tiles (at least 256 of them)
@pytest.mark.parametrize("M,N,K,ta,tb", [(70, 45, 37, False, False), (64, 64, 16, True, False),
                                          (130, 20, 100, False, True), (5, 300, 3, True, True),
                                          (200, 136, 72, False, False), (96, 256, 264, True, False),
                                          (64, 128, 40, False, True), (96, 256, 264, True, True),
                                          (2100, 2060, 72, False, False), (2048, 2100, 40, True, True)])
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


@pytest.mark.parametrize("width,depth,n_out,batch", [(256, 4, 640, 256), (64, 3, 40, 50)])
def test_gradient_matches_cpu_reference_elementwise(width, depth, n_out, batch):
    """Every weight and bias gradient element against the FP64 reference that
    rounds the same operands to BF16 as the GPU (input, weights, hidden
    activations, back-propagated errors; oracle/mlp_ref.loss_grad_bf16).  The
    first case is the warm-start network itself (10 -> 4 x 256 GELU -> 640).
    What is left is FP32 accumulation order and the BF16 roundings it flips
    (an FP32 emulation of the same network on the CPU differs from the FP64
    one by at most 1.1e-3 of a tensor's largest element, with median relative
    error 3e-4 and 99th percentile 2e-2); a dropped term, a wrong scale or a
    transposed operand moves whole tensors."""
    from paper_2308_15407_amd.mlp import WarmStartNet, layer_shapes
    net = WarmStartNet(n_in=10, width=width, depth=depth, n_out=n_out, max_batch=batch, seed=3)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(batch, 10)).astype(np.float32)
    t = rng.normal(size=(batch, n_out)).astype(np.float32)
    loss, g = net.loss_grad(x, t)
    p = net.get_params().astype(np.float64)
    shapes = layer_shapes(10, width, depth, n_out)
    Lr, gr = R.loss_grad_bf16(p, shapes, x.astype(np.float64), t.astype(np.float64))
    print("loss gpu %.7f ref %.7f" % (loss, Lr), flush=True)
    assert abs(loss - Lr) < 1e-4 * abs(Lr)
    off = 0
    for layer, (fin, fout) in enumerate(shapes):
        for name, n in (("W", fin * fout), ("b", fout)):
            a_, b_ = g[off:off + n].astype(np.float64), gr[off:off + n]
            off += n
            scale = np.max(np.abs(b_))
            err = np.abs(a_ - b_)
            rel = err / (np.abs(b_) + 1e-3 * scale)
            print("layer %d %s (%d): max |dg| %.1e of max |g|, relative: median %.1e, 99th percentile %.1e" %
                  (layer, name, n, err.max() / scale, np.median(rel), np.percentile(rel, 99)), flush=True)
            assert scale > 0
            assert err.max() < 5e-3 * scale, (layer, name)
            assert np.median(rel) < 1e-3, (layer, name)
            assert np.percentile(rel, 99) < 5e-2, (layer, name)
    assert off == g.size


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
