"""The allocation-free surrogate forward (static per-GPU scratch) against
ms_surrogate_forward, which allocates its own workspace: the same kernels
on the same inputs, so the outputs must agree bit for bit. Two calls in a
row, the second with fewer poses, so stale scratch contents from the first
call would show; and a batch beyond the scratch size is refused with
nothing written."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"


def _net(model, hidden, seed):
    gm = ms.Model(model)
    s = ms.Surrogate(gm, hidden=hidden, seed=seed)
    rng = np.random.default_rng(seed)
    # a non-trivial output standardisation, so the de-standardising
    # epilogue is exercised too
    s.set_norm(rng.normal(0.0, 0.1, s.n_out), rng.uniform(0.01, 0.2, s.n_out))
    return gm, s


def _poses(model, s, n, seed):
    q = torch.zeros(n, model["nq"], device=DEV)
    s.sample(q, seed)
    torch.cuda.synchronize()
    return q


def _both(model, s, q):
    n, nm = q.shape[0], model["n_mus"]
    L0 = torch.full((n, nm), float("nan"), device=DEV)
    r0 = torch.full((n, nm, 3), float("nan"), device=DEV)
    L1, r1 = L0.clone(), r0.clone()
    s.forward(q, L0, r0)
    s.forward_noalloc(q, L1, r1)
    torch.cuda.synchronize()
    return (L0.cpu().numpy(), r0.cpu().numpy()), (L1.cpu().numpy(), r1.cpu().numpy())


@pytest.mark.parametrize("kind", ["chain", "human"])
def test_noalloc_forward_equals_forward_on_two_calls(kind):
    if kind == "chain":
        m = synth.chain_model(1)
        gm, s = _net(m, 64, 5)
    else:
        m = synth.human_model(2)
        gm, s = _net(m, 512, 41)
    nmax = s.noalloc_max()
    if kind == "human":
        assert nmax == 7598      # 16 MiB / (80*2 + 512*2 + 512*2 bytes per pose)
    n1 = min(nmax, 2048)
    n2 = max(1, n1 // 3 + 5)     # a smaller second call, not a multiple of the GEMM tile
    for n, seed in ((n1, 101), (n2, 202)):
        q = _poses(m, s, n, seed)
        (L0, r0), (L1, r1) = _both(m, s, q)
        assert np.isfinite(L0).all() and np.isfinite(r0).all()
        assert np.array_equal(L0, L1), (kind, n, float(np.abs(L0 - L1).max()))
        assert np.array_equal(r0, r1), (kind, n, float(np.abs(r0 - r1).max()))
    del gm


def test_noalloc_forward_rejects_a_batch_beyond_its_scratch():
    m = synth.human_model(2)
    gm, s = _net(m, 512, 41)
    n = s.noalloc_max() + 1
    q = _poses(m, s, n, 7)
    L = torch.full((n, m["n_mus"]), 3.0, device=DEV)
    r = torch.full((n, m["n_mus"], 3), 3.0, device=DEV)
    with pytest.raises(ms.MsError) as e:
        s.forward_noalloc(q, L, r)
    assert e.value.code == -5    # MS_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((L == 3.0).all()) and bool((r == 3.0).all())
    del gm
