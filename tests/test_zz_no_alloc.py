"""pdcs_project_noalloc (the projection entry point that allocates no device
memory) against pdcs_project on the same inputs.

Both build the same tile plan and run the same kernels, so the results must be
identical bit for bit; the test also holds both to the oracle's projection
(1e-12 of the block scale, the bar of the other projection tests).  Two calls
in a row, the second with a smaller input, check that the fixed scratch
carries nothing over from the first call (barrier counters of grid-level SOC
blocks, partial sums, rotated offsets)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ZERO, FREE, NONNEG, SOC, EXP, EXP_DUAL, RSOC = range(7)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def say(*a):
    print(*a, flush=True)


def cone_list(rng, n_small, n_exp, big_dims, rsoc):
    """Mixed cone list: elementwise runs, lane-group SOC blocks, workgroup and
    grid-level SOC blocks, exponential cones and (optionally) rotated SOC."""
    types, dims = [], []
    for i in range(n_small):
        k = int(rng.integers(1, 5))
        types += [NONNEG, SOC, FREE, ZERO][k - 1:k]
        dims.append(int(rng.integers(2, 300)) if types[-1] == SOC else int(rng.integers(1, 3000)))
    for k in big_dims:
        types.append(SOC)
        dims.append(k)
    for _ in range(n_exp):
        types.append(EXP if rng.random() < 0.5 else EXP_DUAL)
        dims.append(3)
    if rsoc:
        for _ in range(40):
            types.append(RSOC)
            dims.append(int(rng.integers(3, 70)))
    order = rng.permutation(len(types))
    types = [types[i] for i in order]
    dims = [dims[i] for i in order]
    v = np.concatenate([rng.standard_normal(k) * 10 ** rng.uniform(-1.5, 1.5) for k in dims])
    return types, dims, v


def block_scale(dims, v):
    out = np.empty_like(v)
    o = 0
    for k in dims:
        out[o:o + k] = max(1.0, np.linalg.norm(v[o:o + k]))
        o += k
    return out


CASES = [
    # (seed, small blocks, exp cones, grid/workgroup SOC dims, rotated, scaled)
    (11, 3000, 2000, [8192, 70001, 300000, 5000], True, False),
    (12, 400, 300, [9000, 1000], False, True),
]


@pytest.mark.parametrize("dual", [False, True])
def test_noalloc_matches_project_two_calls(pd, orc, dual):
    for seed, n_small, n_exp, big, rsoc, scaled in CASES:
        rng = np.random.default_rng(seed + 100 * dual)
        types, dims, v = cone_list(rng, n_small, n_exp, big, rsoc)
        d = 10 ** rng.uniform(-1, 1, v.size) if scaled else None
        say("noalloc vs project", seed, "dual" if dual else "primal", len(types), v.size)
        a = dev(v)
        b = dev(v)
        pd.project(types, dims, a, None if d is None else dev(d), dual=dual)
        pd.project_noalloc(types, dims, b, None if d is None else dev(d), dual=dual)
        torch.cuda.synchronize()
        ga, gb = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(ga, gb), np.max(np.abs(ga - gb))
        ref = orc.proj_blocks(types, dims, v, d, dual=dual)
        err = np.max(np.abs(gb - ref) / block_scale(dims, ref))
        assert err <= 1e-12, err


def test_noalloc_rejects_oversized_plan(pd):
    # 2e6 SOC blocks of dim 3 need about 29 MB of plan scratch, above the 16 MiB array
    types = np.full(2_000_000, SOC, np.int32)
    dims = np.full(2_000_000, 3, np.int64)
    v = torch.zeros(6_000_000, dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PdcsError, match="scratch"):
        pd.project_noalloc(types, dims, v)
    # the projection of a small list still works after the rejection
    w = dev(np.array([-1.0, 3.0, 4.0, 2.0]))
    pd.project_noalloc([SOC, NONNEG], [3, 1], w)
    torch.cuda.synchronize()
    assert np.allclose(w.cpu().numpy(), [2.0, 1.2, 1.6, 2.0], rtol=0, atol=1e-15)
