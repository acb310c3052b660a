"""GPU tests of the warm-start network: the BF16 matrix-core GEMM against the
oracle's FP64 product within the FP32-accumulation bound, the network's
gradient against the oracle's backpropagation, and training."""
import numpy as np
import pytest

from oracle import mlp as OM

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def bits_dev(x):
    """BF16 values (float64 array) -> device int16 tensor of their bit patterns."""
    u = (np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(u.view(np.int16).copy()).cuda()


def from_bits(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


SHAPES = [(77, 131, 48), (64, 1000, 512), (37, 2051, 80), (128, 64, 16), (1, 5, 3),
          (256, 300, 520), (130, 257, 44)]


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("tb", [0, 1])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{m}x{n}x{k}" for m, n, k in SHAPES])
def test_gemm_matches_oracle(pd, ta, tb, shape):
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N * 3 + K + 10 * ta + 20 * tb)
    A = OM.bf16(rng.standard_normal((M, K)))
    B = OM.bf16(rng.standard_normal((K, N)))
    a_st = A.T.copy() if ta else A        # stored layout the kernel reads
    b_st = B.T.copy() if tb else B
    bias = rng.standard_normal(N).astype(np.float32)
    relu = (M + N) % 2 == 0
    c32 = torch.empty((M, N), dtype=torch.float32, device="cuda")
    c16 = torch.empty((M, N), dtype=torch.int16, device="cuda")
    pd.gemm_bf16(bits_dev(a_st), bits_dev(b_st), M, N, K, ta=ta, tb=tb,
                 bias_dev=torch.from_numpy(bias).cuda(), relu=relu, c32_dev=c32, c16_dev=c16)
    torch.cuda.synchronize()
    ref, bound = OM.gemm(a_st, b_st, ta, tb, bias=bias.astype(np.float64), relu=relu)
    got = c32.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bound + 1e-30), np.abs(got - ref).max()
    assert np.array_equal(from_bits(c16), OM.bf16(got))


@pytest.mark.parametrize("n_out", [300, 5000])
def test_network_gradient_matches_oracle(pd, n_out):
    """The GPU gradient against the oracle's backpropagation with the same BF16
    rounding points.  Both sides may round an intermediate to neighbouring BF16
    values where FP32 and FP64 sums straddle a rounding boundary, so each
    parameter block is held to one BF16 unit (2^-8) in relative 2-norm.  With
    5000 outputs the product dH2 = dO W3 (k = the outputs) takes the split-K
    path: partial products of 1024-wide k chunks added in chunk order."""
    rng = np.random.default_rng(3)
    n_in, hid, B = 64, 128, 32
    npar = hid * n_in + hid + hid * hid + hid + n_out * hid + n_out
    p = np.concatenate([rng.standard_normal(hid * n_in) * np.sqrt(2 / n_in), np.zeros(hid) + 0.1,
                        rng.standard_normal(hid * hid) * np.sqrt(2 / hid), np.zeros(hid) + 0.1,
                        rng.standard_normal(n_out * hid) * np.sqrt(1 / hid), np.zeros(n_out)])
    assert p.size == npar
    theta = rng.standard_normal((B, n_in))
    target = rng.standard_normal((B, n_out))
    net = pd.MLP(n_in, hid, n_out, p.astype(np.float32), max_batch=B)
    g, loss = net.gradient(torch.from_numpy(theta.astype(np.float32)).cuda(),
                           torch.from_numpy(target.astype(np.float32)).cuda())
    p32 = p.astype(np.float32).astype(np.float64)
    lo, go = OM.loss_and_grad(p32, theta.astype(np.float32).astype(np.float64),
                              target.astype(np.float32).astype(np.float64), n_in, hid, n_out)
    assert loss == pytest.approx(lo, rel=1e-5)
    sizes = [hid * n_in, hid, hid * hid, hid, n_out * hid, n_out]
    o = 0
    for name, s in zip(["W1", "b1", "W2", "b2", "W3", "b3"], sizes):
        rel = np.linalg.norm(g[o:o + s] - go[o:o + s]) / np.linalg.norm(go[o:o + s])
        assert rel <= 2.0 ** -8, (name, rel)
        o += s
    net.close()


def test_training_fits_a_teacher(pd):
    """Adam steps on the GPU fit the outputs of a random teacher network of the
    same shape: the loss falls below a quarter of its starting value."""
    rng = np.random.default_rng(4)
    n_in, hid, n_out, B = 16, 64, 40, 128
    def init(scale):
        return np.concatenate([rng.standard_normal(hid * n_in) * np.sqrt(2 / n_in), np.zeros(hid),
                               rng.standard_normal(hid * hid) * np.sqrt(2 / hid), np.zeros(hid),
                               rng.standard_normal(n_out * hid) * scale * np.sqrt(1 / hid),
                               np.zeros(n_out)])
    teacher = init(1.0)
    theta = rng.standard_normal((B, n_in))
    target = OM.forward(teacher, theta, n_in, hid, n_out, quantize=False)["o"]
    net = pd.MLP(n_in, hid, n_out, init(0.1).astype(np.float32), max_batch=B)
    th = torch.from_numpy(theta.astype(np.float32)).cuda()
    tg = torch.from_numpy(target.astype(np.float32)).cuda()
    first = net.train_step(th, tg, 3e-3)
    for _ in range(400):
        last = net.train_step(th, tg, 3e-3)
    assert last < 0.25 * first, (first, last)
    out = torch.empty((B, n_out), dtype=torch.float32, device="cuda")
    net.forward(th, out)
    torch.cuda.synchronize()
    ref = OM.forward(net.params(), theta.astype(np.float32), n_in, hid, n_out, quantize=True)["o"]
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-3 * max(1.0, np.abs(ref).max())
    net.close()


@pytest.mark.parametrize("n_in,hid,B", [(64, 256, 40), (16, 128, 1), (32, 512, 96)])
def test_fused_hidden_layers_equal_separate_gemms(pd, n_in, hid, B):
    """The forward pass runs both hidden layers in one launch when the shapes
    allow it; it must give the same bits as the three separate GEMM launches
    (BF16 theta, layer 1 with bias and ReLU, layer 2, output layer), which the
    GEMM test above holds to the oracle."""
    rng = np.random.default_rng(n_in + hid + B)
    n_out = 72
    sizes = [hid * n_in, hid, hid * hid, hid, n_out * hid, n_out]
    p = np.concatenate([rng.standard_normal(k) * 0.2 for k in sizes]).astype(np.float32)
    net = pd.MLP(n_in, hid, n_out, p, max_batch=128)
    theta = rng.standard_normal((B, n_in)).astype(np.float32)
    out = torch.empty((B, n_out), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(theta).cuda(), out)
    offs = np.cumsum([0] + sizes)
    part = [p[offs[i]:offs[i + 1]] for i in range(6)]
    w1, b1, w2, b2, w3, b3 = (part[0], part[1], part[2], part[3], part[4], part[5])
    dev32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    xb = bits_dev(OM.bf16(theta.astype(np.float64)))
    h1 = torch.empty((B, hid), dtype=torch.float32, device="cuda")
    h1b = torch.empty((B, hid), dtype=torch.int16, device="cuda")
    pd.gemm_bf16(xb, bits_dev(OM.bf16(w1.astype(np.float64))), B, hid, n_in, ta=0, tb=1,
                 bias_dev=dev32(b1), relu=True, c32_dev=h1, c16_dev=h1b)
    h2 = torch.empty((B, hid), dtype=torch.float32, device="cuda")
    h2b = torch.empty((B, hid), dtype=torch.int16, device="cuda")
    pd.gemm_bf16(h1b, bits_dev(OM.bf16(w2.astype(np.float64))), B, hid, hid, ta=0, tb=1,
                 bias_dev=dev32(b2), relu=True, c32_dev=h2, c16_dev=h2b)
    ref = torch.empty((B, n_out), dtype=torch.float32, device="cuda")
    pd.gemm_bf16(h2b, bits_dev(OM.bf16(w3.astype(np.float64))), B, n_out, hid, ta=0, tb=1,
                 bias_dev=dev32(b3), relu=False, c32_dev=ref)
    torch.cuda.synchronize()
    net.close()
    assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
