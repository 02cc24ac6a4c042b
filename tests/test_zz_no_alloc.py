"""hp_apply_h_noalloc: the H apply for callers that cannot allocate device memory, with its
intermediate buffers in the library's fixed per-GPU workspace, against hp_apply_h (the
same kernels on the context's buffers): bit-identical on two calls in a row, the second on
a smaller input (the workspace keeps the first call's contents), and sizes beyond the
workspace rejected before any GPU work."""
import numpy as np
import pytest

from conftest import ground_state

pytestmark = pytest.mark.gpu


def _hp():
    from paper_2203_15684_amd import hp
    return hp


def _apply_noalloc(ctx, entry, x):
    import torch
    hp = _hp()
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    yd = torch.full_like(xd, complex(np.nan, np.nan))
    torch.cuda.synchronize()
    hp.hp_apply_h_noalloc(ctx, entry, xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("name", ["duo_k221", "olivine28_gamma"])
def test_noalloc_apply_matches_apply_h(name):
    hp = _hp()
    if name.startswith("olivine"):
        from synth import cache
        gs = cache.get(name)
    else:
        gs = ground_state(name)
    ctx = hp.hp_ground_state_load(gs)
    rng = np.random.default_rng(5)
    calls = [(len(gs.kpts) - 1, 9), (0, 3)]  # the second call is smaller and on another entry
    for entry, n in calls:
        npw = gs.kpts[entry].npw
        x = rng.standard_normal((n, npw)) + 1j * rng.standard_normal((n, npw))
        print(f"[noalloc] {name} entry {entry} n {n}", flush=True)
        y = _apply_noalloc(ctx, entry, x)
        assert np.array_equal(y, hp.hp_apply_h(ctx, entry, x)), (entry, n)
    ctx.close()


def test_noalloc_rejects_oversize_and_host_arrays():
    import torch
    hp = _hp()
    gs = ground_state("duo_k221")
    ctx = hp.hp_ground_state_load(gs)
    npw = gs.kpts[0].npw
    x = torch.zeros((4096, npw), dtype=torch.complex128, device="cuda")
    with pytest.raises(hp.HpError) as e:
        hp.hp_apply_h_noalloc(ctx, 0, x, x.clone())   # beyond the fixed workspace
    assert e.value.status == hp.HP_ERR_ARG and "workspace" in str(e.value)
    with pytest.raises(ValueError):
        hp.hp_apply_h_noalloc(ctx, 0, x[:2].cpu(), x[:2].cpu())
    ctx.close()
