"""Pins of the network oracle (CPU): its gradient against central differences
of its own loss, BF16 rounding against the format's definition, and the GEMM
bound against exactly representable cases."""
import numpy as np
import pytest

from oracle import mlp as M


def test_bf16_rounding_definition():
    # exactly representable values are kept; halfway cases go to the even neighbour
    x = np.array([1.0, -2.5, 3.0 * 2 ** -20, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9,
                  1.0 + 2 ** -8 + 2 ** -20], dtype=np.float64)
    want = np.array([1.0, -2.5, 3.0 * 2 ** -20, 1.0, 1.0 + 2 ** -6, 1.0, 1.0 + 2 ** -7])
    got = M.bf16(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> even (1); 1 + 3 2^-8 -> 1 + 2^-6 (even)
    assert np.array_equal(got[:2], want[:2]) and got[2] == want[2]
    assert got[3] == 1.0 and got[4] == 1.0 + 2 ** -6
    # 1 + 2^-9 is below halfway; 1 + 2^-8 + 2^-20 is just above it
    assert got[5] == 1.0 and got[6] == 1.0 + 2 ** -7
    # every result has at most 8 significant bits
    r = np.random.default_rng(0).standard_normal(1000)
    b = M.bf16(r)
    m, e = np.frexp(b)
    assert np.all(np.abs(m * 2 ** 8 - np.round(m * 2 ** 8)) == 0)
    assert np.all(np.abs(b - r) <= 2.0 ** -8 * np.abs(r))


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    n_in, hid, n_out, B = 5, 7, 4, 3
    npar = hid * n_in + hid + hid * hid + hid + n_out * hid + n_out
    p = rng.standard_normal(npar) * 0.5
    theta = rng.standard_normal((B, n_in))
    target = rng.standard_normal((B, n_out))
    loss, g = M.loss_and_grad(p, theta, target, n_in, hid, n_out, quantize=False)
    h = 1e-6
    fd = np.empty(npar)
    for i in range(npar):
        e = np.zeros(npar)
        e[i] = h
        lp, _ = M.loss_and_grad(p + e, theta, target, n_in, hid, n_out, quantize=False)
        lm, _ = M.loss_and_grad(p - e, theta, target, n_in, hid, n_out, quantize=False)
        fd[i] = (lp - lm) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_linear_limit_has_closed_form():
    """With one hidden unit kept positive and identity-like weights the network
    is affine, and the gradient of the squared error has the textbook form."""
    n_in, hid, n_out, B = 2, 2, 1, 4
    W1 = np.eye(2)
    b1 = np.array([10.0, 10.0])          # keeps h1 > 0 on these inputs
    W2 = np.eye(2)
    b2 = np.zeros(2)
    W3 = np.array([[1.0, -1.0]])
    b3 = np.array([0.5])
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    theta = np.array([[1.0, 2.0], [0.5, -1.0], [2.0, 2.0], [-1.0, 0.0]])
    target = np.zeros((B, 1))
    loss, g = M.loss_and_grad(p, theta, target, n_in, hid, n_out, quantize=False)
    o = theta[:, 0] - theta[:, 1] + 0.5
    assert loss == pytest.approx((o ** 2).sum() / (2 * B))
    gb3 = o.sum() / B
    assert g[-1] == pytest.approx(gb3)


def test_gemm_oracle_bound_is_zero_for_exact_cases():
    a = M.bf16(np.array([[1.0, 2.0], [3.0, 4.0]]))
    b = M.bf16(np.array([[0.5, -1.0], [2.0, 0.25]]))
    c, bound = M.gemm(a, b)
    assert np.array_equal(c, np.array([[4.5, -0.5], [9.5, -2.0]]))
    c2, _ = M.gemm(a.T.copy(), b, ta=1)
    assert np.array_equal(c, c2)
    c3, _ = M.gemm(a, b.T.copy(), tb=1)
    assert np.array_equal(c, c3)
