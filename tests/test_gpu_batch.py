"""Ragged batching (beagle_eval_batched), its graph cache and the tile-width
tuner, on the GPU."""
import numpy as np
import pytest

import gates
from oracle import fitness as ofit
from paper_2603_12292_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = {ofit.MSE: "mse", ofit.CORR: "corr"}


def _api():
    from paper_2603_12292_amd import api
    return api


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.int64)


def _problem(ps, data):
    api = _api()
    return (api.DevicePrograms.from_programset(ps), torch.from_numpy(data.X).cuda(),
            torch.from_numpy(data.y).cuda())


def _small_problems(seed=11, kind=ofit.MSE):
    """Problems of different D, M (ragged tails, one chunk and many) and N,
    one with malformed programs."""
    shapes = [(1, 2, 40), (2, 100, 64), (3, 1000, 200), (9, 5000, 128), (5, 70_001, 300), (4, 2049, 33),
              (7, 20_000, 256), (8, 4096, 100)]
    out = []
    for q, (D, M, N) in enumerate(shapes):
        if kind == ofit.CORR and M < 2:
            continue
        ps = wl.random_population(seed * 100 + q, N, 3, 80, D)
        if q == 3:  # malformed programs: a bad variable and an underflow
            toks = ps.tokens.copy()
            toks[ps.tok_offset[0]] = wl.tok(wl.VAR, D + 1)
            toks[ps.tok_offset[1]] = wl.tok(wl.ADD)
            ps = wl.ProgramSet(toks, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset, ps.const_count)
        data = wl.make_dataset(seed * 100 + q, M, D, target_len=8) if M >= 50 else \
            wl.Dataset(np.random.default_rng(q).uniform(1, 5, (M, D)).astype(np.float32),
                       np.random.default_rng(q + 1).uniform(1, 5, M).astype(np.float32), [], [])
        out.append((ps, data))
    return out


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_tile_width_changes_no_bit(kind):
    """Class-0 programs give the same fitness bits with 8 and with 4 cases per lane."""
    api = _api()
    ctx = api.Context(0)
    for ps, data in _small_problems(5, kind):
        if data.D > 8:
            continue
        progs, X, y = _problem(ps, data)
        ctx.set_tuning("wide")
        a = api.evaluate(progs, X, y, KINDS[kind], ctx=ctx).cpu().numpy()
        ctx.set_tuning("narrow")
        b = api.evaluate(progs, X, y, KINDS[kind], ctx=ctx).cpu().numpy()
        assert np.array_equal(_bits(a), _bits(b)), (data.D, data.M)
    ctx.close()


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_batched_equals_single(kind):
    api = _api()
    ctx = api.Context(0)
    probs = _small_problems(7, kind)
    dev = [_problem(ps, d) for ps, d in probs]
    single = [api.evaluate(p, X, y, KINDS[kind], with_status=True, ctx=ctx) for p, X, y in dev]
    # an empty population in the middle is skipped
    ps0, d0 = probs[2]
    batch = dev[:3] + [_problem(ps0.subset([]), d0)] + dev[3:]
    fits, sts = api.evaluate_batched(batch, KINDS[kind], with_status=True, ctx=ctx)
    torch.cuda.synchronize()
    assert fits[3].numel() == 0
    del fits[3], sts[3]
    for q, ((f1, s1), f2, s2) in enumerate(zip(single, fits, sts)):
        assert np.array_equal(s1.cpu().numpy(), s2.cpu().numpy()), q
        assert np.array_equal(_bits(f1.cpu().numpy()), _bits(f2.cpu().numpy())), q
    bad = [i for i, (ps, d) in enumerate(probs) if d.D == 9][0]
    assert (sts[bad].cpu().numpy()[:2] != 0).all()
    ctx.close()


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_batched_oracle_parity(kind):
    """Sampled programs of every problem against the oracle's gates."""
    api = _api()
    probs = _small_problems(9, kind)
    dev = [_problem(ps, d) for ps, d in probs]
    fits = [f.cpu().numpy() for f in api.evaluate_batched(dev, KINDS[kind])]
    compared = ill = checked = finite = 0
    for q, ((ps, data), gpu) in enumerate(zip(probs, fits)):
        sub = list(range(0, ps.n, max(1, ps.n // 12)))
        r = gates.references(ps, data.X, data.y, kind, subset=sub, processes=4)
        # a dozen programs per problem is too few to bound the shares per
        # problem; they are bounded over the whole batch below
        s = gates.check(gpu[sub], r, kind, data.y, max_ill_frac=1.0, max_unchecked_frac=1.0, label=f"batch q={q}",
                        min_value=0)
        gates.output_gate(ps, data.X, data.y, kind, gpu[sub], s, idx=sub, label=f"batch q={q}")
        compared += s.n_value
        ill += s.n_ill
        checked += s.n_checked
        finite += s.n_finite
    print(f"value-gated {compared}, ill-conditioned {ill}, under a value gate {checked} of {finite} finite")
    assert compared > 50 and checked >= 0.8 * finite
    # programs up to 80 tokens often hold exp of large arguments, whose
    # relative condition number is |x|: with MSE (which keeps the magnitude
    # of yhat) about half of them move by more than 1e-6 under fp32 rounding
    assert ill <= (0.6 if kind == ofit.MSE else 0.35) * (compared + ill)


def test_graph_is_captured_once_and_replayed():
    """Same table -> one capture, every replay equal to the eager results, the
    replay reads the current contents of the caller's buffers."""
    api = _api()
    ctx = api.Context(0)
    probs = _small_problems(13)
    dev = [_problem(ps, d) for ps, d in probs]
    out = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _, _ in dev]
    eager = [api.evaluate(p, X, y, "mse", ctx=ctx).cpu().numpy() for p, X, y in dev]
    c0, r0 = ctx.graph_stats()
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        api.evaluate_batched(dev, "mse", ctx=ctx, out=out)
        scratch.mul_(1.0001).add_(0.5)   # eager work between replays
        s = scratch.sum()
        torch.cuda.synchronize()
        for q in range(len(dev)):
            assert np.array_equal(_bits(out[q].cpu().numpy()), _bits(eager[q])), (rep, q)
        assert torch.isfinite(s)
    c1, r1 = ctx.graph_stats()
    assert c1 - c0 == 1 and r1 - r0 == 4
    # new data in the same buffers: the replayed graph sees it
    p, X, y = dev[4]
    X.mul_(0.5)
    api.evaluate_batched(dev, "mse", ctx=ctx, out=out)
    ref = api.evaluate(p, X, y, "mse", ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(out[4].cpu().numpy()), _bits(ref.cpu().numpy()))
    assert not np.array_equal(_bits(out[4].cpu().numpy()), _bits(eager[4]))
    c2, _ = ctx.graph_stats()
    assert c2 == c1
    # other output buffers: another table, another capture
    api.evaluate_batched(dev, "mse", ctx=ctx)
    c3, _ = ctx.graph_stats()
    assert c3 == c2 + 1
    ctx.close()


def test_batched_argument_errors():
    api = _api()
    probs = _small_problems(3)
    dev = [_problem(ps, d) for ps, d in probs[:3]]
    with pytest.raises(api.BeagleError) as e:
        api.evaluate_batched(dev, 7)
    assert e.value.code == -1
    bad = list(dev)
    p, X, y = bad[1]
    bad[1] = (p, X[:1].contiguous(), y[:1].contiguous())
    with pytest.raises(api.BeagleError) as e:
        api.evaluate_batched(bad, "corr")
    assert "problem 1" in str(e.value)
    assert api.evaluate_batched([], "mse") == []


def test_autotune_cache_file(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BEAGLE_AUTOTUNE_CACHE", str(path))
    api = _api()
    ctx = api.Context(0)
    ps, data = _small_problems(17)[4]
    p, X, y = _problem(ps, data)
    a = api.evaluate(p, X, y, "corr", ctx=ctx).cpu().numpy()
    ctx.close()
    lines = [ln.split() for ln in path.read_text().splitlines() if not ln.startswith("#")]
    assert len(lines) == 1 and len(lines[0]) == 5
    kind, D, mlog, llog, kv = map(int, lines[0])
    assert (kind, D, mlog) == (1, data.D, round(np.log2(data.M))) and kv in (0, 1)
    ctx2 = api.Context(0)   # reads the file: no new measurement, same bits
    b = api.evaluate(p, X, y, "corr", ctx=ctx2).cpu().numpy()
    ctx2.close()
    assert np.array_equal(_bits(a), _bits(b))
    assert len([ln for ln in path.read_text().splitlines() if not ln.startswith("#")]) == 1


@pytest.mark.parametrize("kind", [ofit.MSE])
def test_ragged_workload_full_size(kind):
    """The 64-problem ragged workload (1024 programs each, L 5..96, D 1..9,
    M 10^3..10^6) in the launch configuration the benchmark times: batched
    fitness bit-identical to 64 separate evaluations, sampled oracle parity."""
    api = _api()
    ws = wl.ragged_problems()
    dev = [_problem(w.programs, w.data) for w in ws]
    fits = [f.cpu().numpy() for f in api.evaluate_batched(dev, KINDS[kind])]
    for q, (p, X, y) in enumerate(dev):
        one = api.evaluate(p, X, y, KINDS[kind]).cpu().numpy()
        assert np.array_equal(_bits(one), _bits(fits[q])), q
    compared = checked = finite = 0
    for q in range(0, 64, 8):
        w = ws[q]
        sub = [3, 517, 1001]
        r = gates.references(w.programs, w.data.X, w.data.y, kind, subset=sub, processes=2)
        s = gates.check(fits[q][sub], r, kind, w.data.y, max_ill_frac=1.0, max_unchecked_frac=1.0,
                        label=f"ragged q={q}", min_value=0)
        gates.output_gate(w.programs, w.data.X, w.data.y, kind, fits[q][sub], s, idx=sub, label=f"ragged q={q}")
        compared += s.n_value
        checked += s.n_checked
        finite += s.n_finite
    print(f"value-gated {compared}, under a value gate {checked} of {finite} finite")
    assert compared >= 12 and checked >= 18
