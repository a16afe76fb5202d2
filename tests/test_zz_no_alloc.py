"""The allocation-free denoiser entry point, pdf_denoise_stats_noalloc,
against pdf_denoise_stats through the C ABI: two calls in a row, the first on
a canyon mesh of about 45 k nodes (two chunks of the fixed scratch) and the
second on a smaller one (about 10 k nodes, one partial chunk, over what the
first call left in the scratch).  Both entry points run the same per-node
arithmetic, so the results must agree exactly, as must the counts of rejected
corrections."""
import numpy as np
import pytest

from synth import configs as CF

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _denoiser(L, target_elems, seed, hidden=64):
    from paper_1006_0720_amd.runner import workload_context

    w = CF.canyon(target_elems=target_elems, ppe=10, seed=seed)
    print(f"[no-alloc] {w.name} nodes={w.mesh.n_nodes} hidden={hidden}", flush=True)
    ctx = workload_context(w)
    ctx.advance(2, w.dt)
    dn = L.Denoiser(ctx, hidden=hidden, seed=seed)
    f = dn.features().cpu().numpy()
    st = ctx.stats()
    q = [0, 1, 4, 5, 6, 8, 11, 3]
    scale = 0.05 * np.sqrt((st[q] ** 2).mean(axis=1))
    dn.set_norm(f.mean(0), f.std(0) + 1e-3, scale)
    return w, ctx, dn


def test_noalloc_matches_denoise_stats_two_calls(L):
    import torch

    for target, seed in ((90_000, 1), (20_000, 2)):
        w, ctx, dn = _denoiser(L, target, seed)
        nn = w.mesh.n_nodes
        ref, nf_ref = dn.denoise(tau=3.0, device=True)
        out = torch.full((25, nn), float("nan"), dtype=torch.float64, device=ctx.device)
        nf = torch.full((1,), -1, dtype=torch.int64, device=ctx.device)
        dn.denoise_noalloc(out, nf, tau=3.0)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"{target}: {(out != ref).sum().item()} values differ"
        assert int(nf.item()) == nf_ref
        assert 0 < nf_ref < 8 * nn  # some corrections taken, some rejected
        # without a counter
        out2 = torch.zeros_like(out)
        dn.denoise_noalloc(out2, None, tau=3.0)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
        dn.close()
        ctx.close()


def test_noalloc_rejects_unsupported_width_and_arguments(L):
    import torch

    w, ctx, dn = _denoiser(L, 20_000, 3, hidden=256)  # activations would not fit the scratch
    out = torch.zeros((25, w.mesh.n_nodes), dtype=torch.float64, device=ctx.device)
    with pytest.raises(L.PdfError) as ei:
        dn.denoise_noalloc(out, None)
    assert ei.value.status == 1 and "48..128" in str(ei.value)
    dn.close()
    w, ctx2, dn = _denoiser(L, 20_000, 3)
    with pytest.raises(L.PdfError) as ei:
        dn.denoise_noalloc(out, None, tau=-1.0)
    assert ei.value.status == 1
    dn.close()
    ctx.close()
    ctx2.close()
