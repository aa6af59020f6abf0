"""The paper's own scores (Eq. 3 point-to-point, Eq. 2 r^4) on the GPU
against the oracle (oracle/scores.py).

Integer work is bit-exact where the outputs are: programs of + - * / only
give outputs identical to the fp32-emulating oracle (O32e), so their POINT
scores must match exactly.  With transcendental operators the outputs may
differ by a few ulps; a case score can then change only where the rounding
argument or the validity of the output is ambiguous, i.e. where the oracle's
own O64 / O32e / O32p (two seeds) evaluations disagree on that case; the
difference is bounded by those cases' score ranges."""
import math

import numpy as np
import pytest

import progtext
from oracle import interp
from oracle import scores as sc
from paper_2603_12292_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

S = 1000.0


def _scores(ps, data, kind, smax=S):
    from paper_2603_12292_amd import api
    P = api.DevicePrograms.from_programset(ps)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    out, st = api.evaluate_score(P, X, y, kind, smax, with_status=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy()


def _outputs(t, c, X):
    modes = [("o64", 0), ("o32e", 0), ("o32p", 1), ("o32p", 2)]
    return [interp.run(t, c, X, m, seed) for m, seed in modes]


def _arith_population(rng, n, D):
    progs = []
    for _ in range(n):
        toks, consts = wl.random_program(rng, int(rng.integers(1, 40)), D)
        out = []
        for t in toks:
            out += [t] if (t & 0xFF) >= 9 or (t & 0xFF) < 4 else [wl.tok(wl.VAR, 0), wl.tok(wl.ADD)]
        progs.append((out, consts))
    # outputs that overflow (invalid) on part of the domain
    progs.append((progtext.parse("x0 x0 * x0 * x0 * c0 *"), [np.float32(3e37)]))
    progs.append((progtext.parse("x1 c0 / x1 *"), [np.float32(1e-38)]))
    return wl.pack_programs(progs)


def test_point_score_bit_exact_on_arithmetic_programs():
    rng = np.random.default_rng(61)
    data = wl.invalid_target_dataset(62, 3000, 3)
    ps = _arith_population(rng, 48, 3)
    got, st = _scores(ps, data, "point")
    assert np.all(st == 0)
    for p in range(ps.n):
        t, c = ps.program(p)
        yh = interp.run(t, c, data.X, "o32e")
        assert got[p] == sc.point_score(yh, data.y, S), p


def test_r4_score_on_arithmetic_programs():
    rng = np.random.default_rng(63)
    data = wl.invalid_target_dataset(64, 3000, 3)
    ps = _arith_population(rng, 48, 3)
    got, st = _scores(ps, data, "r4")
    assert np.all(st == 0)
    for p in range(ps.n):
        t, c = ps.program(p)
        yh = interp.run(t, c, data.X, "o32e")
        n, c1, c2 = sc.pair_counts(yh, data.y)
        exact = -S * (c1 - c2)
        term = sc.r4_score(yh, data.y, S) - exact
        # counts exact; the r^4 term within binary64 summation-order error
        # of the oracle's (relative to itself)
        assert abs((got[p] - exact) - term) <= 1e-9 * abs(term) + 1e-12 * S * n + 2.0 ** -50 * abs(exact), \
            (p, got[p], exact, term)


# share of random programs (lengths 3..40) whose r^4 term is compared:
# the others have a case whose validity, or an r^4 term that, moves under
# the oracle's own fp32 modes
R4_FLOOR = 0.6

# relative output error the device functions may add (they are within 4 ulp
# of the exact values; twice that)
OUT_EPS = 2.0 ** -21


def _ambiguity(outs, y, smax):
    """Sum over cases of (max - min) of the case score over the oracle's
    evaluation modes and over the binary32 outputs moved by +-OUT_EPS
    relative: Eq. 3 rounds S min/max, so a case whose argument lies within
    the device's error of a rounding boundary has no unique score (the random
    perturbations of the O32p modes need not land on its other side)."""
    with np.errstate(all="ignore"):
        shifted = [(outs[1] * f).astype(np.float32).astype(np.float64) for f in (1.0 - OUT_EPS, 1.0 + OUT_EPS)]
    per = np.array([[sc.case_score(float(a), float(b), smax) for a, b in zip(o.tolist(), y.astype(np.float64).tolist())]
                    for o in list(outs) + shifted])
    return float(np.sum(per.max(axis=0) - per.min(axis=0)))


def _r4_gate(got, outs, y):
    """Eq. 2 on one program against the oracle's evaluation modes.  Returns
    False (not compared) when the validity of some case depends on rounding
    (the counts differ between modes) or when the r^4 term is ill
    conditioned (moves by more than 1e-6 of itself between modes); otherwise
    asserts the counts' part -S (c1 - c2) exactly and the r^4 term
    S r^4 (N - c1 - c2) within 1e-5 relative of the binary64 oracle's, plus
    the binary64 rounding of the score and of separating the two parts."""
    counts = {sc.pair_counts(o, y) for o in outs}
    if len(counts) != 1:
        return False
    n, c1, c2 = counts.pop()
    exact = -S * (c1 - c2)
    terms = [sc.r4_score(o, y, S) - exact for o in outs]
    ref = terms[0]
    at = 1e-12 * S * max(n, 1) + 2.0 ** -50 * abs(exact)
    if max(abs(t - ref) for t in terms) > 1e-6 * abs(ref) + at:
        return False
    assert abs((got - exact) - ref) <= 1e-5 * abs(ref) + at, (got, exact, ref)
    return True


def test_point_score_general_programs():
    w = wl.random_population(65, 96, 3, 40, 3)
    data = wl.invalid_target_dataset(66, 2000, 3)
    got, st = _scores(w, data, "point")
    assert np.all(st == 0)
    n_exact = 0
    for p in range(w.n):
        t, c = w.program(p)
        outs = _outputs(t, c, data.X)
        ref = sc.point_score(outs[1], data.y, S)
        amb = _ambiguity(outs, data.y, S)
        assert abs(got[p] - ref) <= amb, (p, got[p], ref, amb)
        n_exact += got[p] == ref
    assert n_exact >= 0.8 * w.n


def test_r4_score_general_programs():
    w = wl.random_population(67, 96, 3, 40, 3)
    data = wl.invalid_target_dataset(68, 2000, 3)
    got, st = _scores(w, data, "r4")
    assert np.all(st == 0)
    n_cmp = 0
    for p in range(w.n):
        t, c = w.program(p)
        n_cmp += _r4_gate(got[p], _outputs(t, c, data.X), data.y)
    print(f"r^4 term compared on {n_cmp} of {w.n} programs")
    assert n_cmp >= R4_FLOOR * w.n


def test_scores_degenerate_and_arguments():
    from paper_2603_12292_amd import api
    data = wl.invalid_target_dataset(69, 500, 2)
    texts = ["c0", "x0 x0 -", "x1 c0 *"]
    ps = wl.pack_programs([(progtext.parse(t), [np.float32(2.0)]) for t in texts])
    pt, _ = _scores(ps, data, "point", 10.0)
    r4, _ = _scores(ps, data, "r4", 10.0)
    for p in range(ps.n):
        t, c = ps.program(p)
        yh = interp.run(t, c, data.X, "o32e")
        assert pt[p] == sc.point_score(yh, data.y, 10.0)
        assert r4[p] == pytest.approx(sc.r4_score(yh, data.y, 10.0), rel=1e-9, abs=1e-9)
    # every target invalid: r := 0, every valid output a one-invalid pair
    bad = wl.Dataset(data.X, np.full(500, np.nan, dtype=np.float32), [], [])
    r4b, _ = _scores(ps, bad, "r4", 10.0)
    assert np.all(r4b == -10.0 * 500)
    # an invalid program gets NaN; invalid arguments are rejected
    ps2 = wl.pack_programs([(progtext.parse("x0 +"), [])])
    out, st = _scores(ps2, data, "point")
    assert st[0] != 0 and math.isnan(out[0])
    P = api.DevicePrograms.from_programset(ps)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    with pytest.raises(api.BeagleError):
        api.evaluate_score(P, X, y, "point", -1.0)
    with pytest.raises(api.BeagleError):
        api.evaluate_score(P, X, y, "mse", 10.0)
    with pytest.raises(api.BeagleError):
        api.evaluate(P, X, y, "r4")


def test_scores_full_size_sampled():
    """At the plain-mid shape (N = 4096, M = 10^5), with the invalid-target
    data of that shape: 12 sampled programs against the oracle."""
    w = wl.config_mid()
    data = wl.invalid_target_dataset(70, 100_000, 5)
    got_p, st = _scores(w.programs, data, "point")
    got_r, _ = _scores(w.programs, data, "r4")
    assert np.all(st == 0)
    rng = np.random.default_rng(71)
    n_cmp = 0
    for p in rng.choice(w.programs.n, 12, replace=False):
        t, c = w.programs.program(int(p))
        outs = _outputs(t, c, data.X)
        ref = sc.point_score(outs[1], data.y, S)
        assert abs(got_p[p] - ref) <= _ambiguity(outs, data.y, S), (p, got_p[p], ref)
        n_cmp += _r4_gate(got_r[p], outs, data.y)
    assert n_cmp >= 6


# the paper's further operators (unprotected: NaN outside the domains of
# asin and acos, Inf at 1/0) produce exactly the invalid values the scores
# are built around
ALL_UNARY = wl.UNARY_OPS + wl.EXTENDED_OPS


def test_point_score_extended_operators():
    w = wl.random_population(165, 96, 3, 40, 3, unary=ALL_UNARY)
    data = wl.invalid_target_dataset(166, 2000, 3)
    got, st = _scores(w, data, "point")
    assert np.all(st == 0)
    n_exact = 0
    for p in range(w.n):
        t, c = w.program(p)
        outs = _outputs(t, c, data.X)
        ref = sc.point_score(outs[1], data.y, S)
        amb = _ambiguity(outs, data.y, S)
        assert abs(got[p] - ref) <= amb, (p, got[p], ref, amb)
        n_exact += got[p] == ref
    # 78 of the 96 programs have no ambiguous case at all
    assert n_exact >= 0.7 * w.n


def test_r4_score_extended_operators():
    w = wl.random_population(167, 96, 3, 40, 3, unary=ALL_UNARY)
    data = wl.invalid_target_dataset(168, 2000, 3)
    got, st = _scores(w, data, "r4")
    assert np.all(st == 0)
    n_cmp = 0
    for p in range(w.n):
        t, c = w.program(p)
        n_cmp += _r4_gate(got[p], _outputs(t, c, data.X), data.y)
    print(f"r^4 term compared on {n_cmp} of {w.n} programs")
    assert n_cmp >= R4_FLOOR * w.n
