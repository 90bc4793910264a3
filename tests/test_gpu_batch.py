"""GPU batch (many pairs in one persistent launch) against the CPU oracle."""
import numpy as np
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


def _case(msg):
    print(f"[case] {msg}", flush=True)


def test_batch_mixed(ctx, orc):
    rng = np.random.default_rng(31)
    pairs = []
    for t in range(300):
        la = int(rng.choice([0, 1, 5, 63, 64, 65, 200, 513, 1500, 3000]))
        lb = int(rng.choice([0, 1, 7, 64, 100, 511, 700, 2100]))
        p = synth.homologous_pair(t, la, lb, 0.1) if (t % 2 and la and lb) else synth.random_pair(t, la, lb)
        pairs.append((p.a.tobytes(), p.b.tobytes()))
    for prune in (0, 1):
        for R in (4, 8):
            _case(f"batch mixed prune={prune} R={R}")
            got = ctx.batch(pairs, prune=prune, rows_per_lane=R)
            for (a, b), g in zip(pairs, got):
                assert g.key() == orc.sw_score(a, b), (len(a), len(b))


def test_batch_config3_sample(ctx, orc):
    idx = list(range(0, 400, 1)) + list(range(19_600, 20_000, 7))
    pairs = [synth.config3_pair(i) for i in idx]
    _case(f"batch config3 sample of {len(pairs)}")
    got = ctx.batch([(p.a, p.b) for p in pairs])
    for p, g in zip(pairs, got):
        assert g.key() == orc.sw_score(p.a.tobytes(), p.b.tobytes()), p.tag


def test_batch_device_entry(ctx, orc):
    import torch
    pairs = [synth.config3_pair(i) for i in range(60)]
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs])))
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs])))
    d_a = torch.from_numpy(a).cuda()
    d_b = torch.from_numpy(b).cuda()
    _case("batch_dev")
    got = ctx.batch_dev(d_a, oa, d_b, ob)
    for p, g in zip(pairs, got):
        assert g.key() == orc.sw_score(p.a.tobytes(), p.b.tobytes())


def test_batch_errors(ctx):
    from paper_1304_5966_amd import swmi
    _case("batch bad letter")
    with pytest.raises(swmi.SwError):
        ctx.batch([(b"ACGT", b"ACGT"), (b"ACXT", b"AC")])
    assert ctx.batch([]) == []
