"""sw_score_dev_noalloc: the score pass with the library's fixed scratch as workspace.

Compared through the C ABI with sw_score_dev (caller workspace) and with the
oracle, on two calls in a row, the second on a smaller pair, so the second call
runs on scratch that still holds the first call's contents.  A pair whose
workspace exceeds the scratch is refused before any device work.
"""
import pytest

from paper_1304_5966_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1304_5966_amd import swmi
    c = swmi.Context(0)
    yield c
    c.close()


def _dev(p):
    import torch
    return torch.from_numpy(p.a).cuda(), torch.from_numpy(p.b).cuda()


def test_noalloc_equals_workspace_entry_point_twice(ctx, orc):
    from paper_1304_5966_amd import swmi
    big = synth.homologous_pair(4101, 9000, 7000, 0.08)
    small = synth.homologous_pair(4102, 1700, 1500, 0.12)
    for p, opts in ((big, {}), (small, {}), (big, dict(prune=swmi.PRUNE_BEST)),
                    (small, dict(rows_per_lane=4, waves_per_cu=12))):
        print(f"[case] noalloc {p.a.size} x {p.b.size} {opts}", flush=True)
        d_a, d_b = _dev(p)
        ref = ctx.score_dev(d_a, d_b, **opts)
        got = ctx.score_dev_noalloc(d_a, d_b, **opts)
        assert got.key() == ref.key()
        assert got.cells_computed == ref.cells_computed or opts.get("prune")
        assert got.key() == orc.sw_score(p.a.tobytes(), p.b.tobytes())


def test_noalloc_empty_and_too_large(ctx):
    import torch
    from paper_1304_5966_amd import swmi
    e = torch.empty(0, dtype=torch.uint8, device="cuda")
    x = torch.full((100,), ord("A"), dtype=torch.uint8, device="cuda")
    assert ctx.score_dev_noalloc(e, x).key() == (0, -1, -1)
    # a pair whose workspace is larger than the scratch: refused on the host
    la, lb = 400_000, 400_000
    assert ctx.workspace_size(la, lb) > swmi.NOALLOC_SCRATCH_BYTES
    big_a = torch.full((la,), ord("C"), dtype=torch.uint8, device="cuda")
    big_b = torch.full((lb,), ord("G"), dtype=torch.uint8, device="cuda")
    with pytest.raises(swmi.SwError) as ei:
        ctx.score_dev_noalloc(big_a, big_b)
    assert ei.value.status == swmi.SW_ENOMEM
    # and the scratch still works afterwards
    p = synth.homologous_pair(4103, 800, 900, 0.1)
    d_a, d_b = _dev(p)
    assert ctx.score_dev_noalloc(d_a, d_b).key() == ctx.score_dev(d_a, d_b).key()
