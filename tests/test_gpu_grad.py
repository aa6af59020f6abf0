"""Adjoint (beagle_eval_grad) against the oracle gradient and finite differences."""
import math

import numpy as np
import pytest

import gates
import progtext
from oracle import fitness as ofit
from oracle import grad as og
from oracle import interp
from paper_2603_12292_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRAD_RTOL = 1e-4
COND_RTOL = 1e-5


def _spread(t, c, data, g64, kind=ofit.MSE):
    """Largest move of each gradient component under the O32e and two O32p
    gradient modes (what an fp32 adjoint can be expected to reproduce)."""
    spread = np.zeros_like(g64)
    fn = og.mse_and_grad if kind == ofit.MSE else og.corr_and_grad
    for mode, seed in (("o32e", 0), ("o32p", 1), ("o32p", 2)):
        _, gm = fn(t, c, data.X, data.y, mode, seed)
        spread = np.maximum(spread, np.where(np.isfinite(gm), np.abs(gm - g64), np.inf))
    return spread


def _stable_components(t, c, data, g64, kind=ofit.MSE):
    """Norm-wise stability: components moving by at most COND_RTOL * max|g64|
    (a tenth of the norm-wise gate)."""
    scale = float(np.max(np.abs(g64)))
    return _spread(t, c, data, g64, kind) <= COND_RTOL * scale, scale


def _api():
    from paper_2603_12292_amd import api
    return api


def _grad(ps, data, with_status=False, kind="mse"):
    api = _api()
    P = api.DevicePrograms.from_programset(ps)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    out = api.evaluate_grad(P, X, y, kind, with_status=True)
    torch.cuda.synchronize()
    f, g, st = out[0].cpu().numpy(), out[1].cpu().numpy(), out[2].cpu().numpy()
    return f, g, st


def _well_conditioned(ps, data, idx, kind=ofit.MSE):
    r = gates.references(ps, data.X, data.y, kind, subset=idx)
    at = gates.atol(kind, data.y)
    ok = []
    for j in range(len(idx)):
        sp = max([abs(r.f32[j] - r.f64[j])] + [abs(p[j] - r.f64[j]) for p in r.pert])
        ok.append(math.isfinite(r.f64[j]) and sp <= gates.RTOL_COND * abs(r.f64[j]) + at)
    return np.array(ok)


def test_gradient_matches_oracle():
    w = wl.config_differentiation(N=160, M=3000)
    ps, data = w.programs, w.data
    f, g, st = _grad(ps, data)
    assert np.all(st == 0)
    well = _well_conditioned(ps, data, list(range(ps.n)))
    n_cmp = 0
    bad = []
    for p in range(ps.n):
        if not well[p]:
            continue
        t, c = ps.program(p)
        F, g64 = og.mse_and_grad(t, c, data.X, data.y)
        if not (math.isfinite(F) and np.all(np.isfinite(g64))):
            continue
        o, cc = int(ps.const_offset[p]), int(ps.const_count[p])
        gg = g[o:o + cc].astype(np.float64)
        stable, scale = _stable_components(t, c, data, g64)
        assert abs(f[p] - F) <= 1e-5 * abs(F) + gates.atol(ofit.MSE, data.y)
        if not np.any(stable):
            continue
        err = float(np.max(np.abs(gg - g64)[stable]))
        if err > GRAD_RTOL * scale + 1e-7:
            bad.append((p, err / max(scale, 1e-300), gg, g64))
        n_cmp += 1
    assert not bad, bad[:5]
    print(f"compared gradients of {n_cmp} of {ps.n} programs")
    assert n_cmp > 0.5 * ps.n


def test_gradient_against_finite_differences_full_size():
    """The differentiation workload at full size (N=4096, M=100000); FP64
    central differences of the oracle on a 64-program subset."""
    w = wl.config_differentiation()
    ps, data = w.programs, w.data
    f, g, st = _grad(ps, data)
    assert np.all(st == 0)
    rng = np.random.default_rng(2)
    sub = sorted(rng.choice(ps.n, size=64, replace=False).tolist())
    well = _well_conditioned(ps, data, sub)
    n = 0
    for j, p in enumerate(sub):
        if not well[j]:
            continue
        t, c = ps.program(p)
        F, g64 = og.mse_and_grad(t, c, data.X, data.y)
        if not (math.isfinite(F) and np.all(np.isfinite(g64))):
            continue
        # component-wise stability, a tenth of the component-wise FD gate
        stable = _spread(t, c, data, g64) <= 1e-4 * np.abs(g64)
        fd1, ok1 = og.central_fd(t, c, data.X, data.y, rel_step=1e-5)
        fd2, ok2 = og.central_fd(t, c, data.X, data.y, rel_step=1e-6)
        o = int(ps.const_offset[p])
        for k in np.nonzero(ok1 & ok2 & stable)[0]:
            if not (np.isfinite(fd1[k]) and np.isfinite(fd2[k])):
                continue
            if abs(fd1[k] - fd2[k]) > 1e-4 * max(abs(fd2[k]), 1e-12):
                continue  # differences not converged
            tol = 1e-3 * abs(fd2[k]) + 1e-6 * max(1.0, abs(f[p]))
            assert abs(float(g[o + k]) - fd2[k]) <= tol, (p, k, g[o + k], fd2[k])
            n += 1
    print(f"checked {n} constants against central differences")
    assert n >= 30


def test_forward_equals_plain_evaluation():
    api = _api()
    w = wl.config_differentiation(N=512, M=20000)
    f, g, st = _grad(w.programs, w.data)
    P = api.DevicePrograms.from_programset(w.programs)
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    f2 = api.evaluate(P, X, y, "mse").cpu().numpy()
    fin = np.isfinite(f2)
    assert np.array_equal(np.isnan(f), np.isnan(f2))
    assert np.all(np.abs(f[fin] - f2[fin]) <= 1e-12 * np.abs(f2[fin]) + 1e-300)


def test_long_tapes_many_constants_and_limits():
    rng = np.random.default_rng(9)
    data = wl.make_dataset(19, 2500, 3, x_range=(1.0, 3.0), target_len=8)
    progs = []
    for L in (70, 150, 255):           # LDS tape (decoded words > 64)
        t, _ = wl.random_program(rng, L, 3, allow_const=False)
        progs.append(wl.place_constants(rng, t, 5))
    for L in (30, 60):                 # more constant slots than lane accumulators
        t, _ = wl.random_program(rng, L, 3, allow_const=False)
        progs.append(wl.place_constants(rng, t, 14))
    t, _ = wl.random_program(rng, 700, 3, allow_const=False)   # > 256 decoded words
    progs.append(wl.place_constants(rng, t, 3))
    ps = wl.pack_programs(progs)
    f, g, st = _grad(ps, data)
    assert list(st[:5]) == [0] * 5
    assert st[5] == interp.ST_TOO_LONG and math.isnan(f[5])
    well = _well_conditioned(ps, data, list(range(5)))
    for p in range(5):
        t, c = ps.program(p)
        F, g64 = og.mse_and_grad(t, c, data.X, data.y)
        o, cc = int(ps.const_offset[p]), int(ps.const_count[p])
        if not (math.isfinite(F) and np.all(np.isfinite(g64))):
            continue
        if well[p]:
            assert abs(f[p] - F) <= 1e-5 * abs(F) + gates.atol(ofit.MSE, data.y)
        stable, scale = _stable_components(t, c, data, g64)
        err = np.abs(g[o:o + cc] - g64)[stable]
        assert np.all(err <= GRAD_RTOL * scale + 1e-7), (p, g[o:o + cc], g64, stable)


def test_tape_size_boundaries():
    """Unary chains "x0 c0 + u1 u2 ... uk": one tape entry per unary word, so
    k = 32, 33, 48, 49, 62 put the programs at both sides of each boundary of
    the derivative-tape kernels (at most 32, 48 and 64 entries per case)."""
    rng = np.random.default_rng(14)
    data = wl.make_dataset(23, 3000, 2, x_range=(1.0, 3.0), target_len=8)
    cycle = [wl.COS, wl.SQRT, wl.SIN, wl.EXP, wl.LOG]   # every unary operator, well conditioned
    progs = []
    for k in (32, 33, 48, 49, 62):
        start = int(rng.integers(len(cycle)))
        t = [wl.tok(wl.VAR, 0), wl.tok(wl.CONST, 0), wl.tok(wl.ADD)]
        t += [wl.tok(cycle[(start + i) % len(cycle)]) for i in range(k)]
        progs.append((t, [float(np.float32(rng.uniform(-1, 1)))]))
    ps = wl.pack_programs(progs)
    f, g, st = _grad(ps, data)
    assert np.all(st == 0)
    n_cmp = 0
    for p in range(ps.n):
        t, c = ps.program(p)
        F, g64 = og.mse_and_grad(t, c, data.X, data.y)
        assert math.isfinite(F) and np.all(np.isfinite(g64))
        assert abs(f[p] - F) <= 1e-5 * abs(F) + gates.atol(ofit.MSE, data.y)
        stable, scale = _stable_components(t, c, data, g64)
        err = np.abs(g[p:p + 1] - g64)[stable]
        assert np.all(err <= GRAD_RTOL * scale + 1e-7), (p, g[p], g64)
        n_cmp += int(np.any(stable))
    assert n_cmp == 5


def test_constant_free_subtrees():
    """Subtrees without constants store no tape entries and the reverse sweep
    steps over them: constant-free root (unused slot: zero gradient),
    constant-free left / right operands, nested and fused forms."""
    data = wl.make_dataset(29, 2000, 2, x_range=(1.0, 3.0), target_len=8)
    texts = [
        ("x0 x1 * sin x0 cos +", 1),
        ("x0 x1 * sin c0 x0 * +", 1),
        ("c0 x0 x1 / sqrt x1 exp * -", 1),
        ("x0 sin x1 cos * c0 c1 + /", 2),
        ("x0 c0 + x1 x0 * x1 sin / *", 1),
        ("x1 x0 x1 * x0 / - c0 * x0 x1 + sin x0 * log c1 * +", 2),
        ("x0 x1 - x0 * x1 x0 / + c0 /", 1),
        ("c0 x0 x1 * x1 x0 - / sin *", 1),
    ]
    progs = [(progtext.parse(t), [0.7, -1.3][:k]) for t, k in texts]
    ps = wl.pack_programs(progs)
    f, g, st = _grad(ps, data)
    assert np.all(st == 0)
    for p in range(ps.n):
        t, c = ps.program(p)
        F, g64 = og.mse_and_grad(t, c, data.X, data.y)
        o, cc = int(ps.const_offset[p]), int(ps.const_count[p])
        assert abs(f[p] - F) <= 1e-5 * abs(F) + gates.atol(ofit.MSE, data.y), texts[p]
        if p == 0:
            assert g[o] == 0.0 and g64[0] == 0.0
            continue
        stable, scale = _stable_components(t, c, data, g64)
        assert np.any(stable), texts[p]
        err = np.abs(g[o:o + cc] - g64)[stable]
        assert np.all(err <= GRAD_RTOL * scale + 1e-7), (texts[p], g[o:o + cc], g64)


def test_corr_gradient_matches_oracle():
    """The adjoint of 1 - r^2 against the oracle on well-conditioned
    programs and stable components; the fitness is beagle_eval's, bit for
    bit."""
    api = _api()
    w = wl.config_differentiation(N=160, M=3000)
    ps, data = w.programs, w.data
    f, g, st = _grad(ps, data, kind="corr")
    assert np.all(st == 0)
    P = api.DevicePrograms.from_programset(ps)
    f_eval = api.evaluate(P, torch.from_numpy(data.X).cuda(), torch.from_numpy(data.y).cuda(), "corr").cpu().numpy()
    assert np.array_equal(f, f_eval, equal_nan=True)
    well = _well_conditioned(ps, data, list(range(ps.n)), ofit.CORR)
    n_cmp = 0
    bad = []
    for p in range(ps.n):
        if not well[p]:
            continue
        t, c = ps.program(p)
        F, g64 = og.corr_and_grad(t, c, data.X, data.y)
        if not (math.isfinite(F) and np.all(np.isfinite(g64))) or F >= 1.0:
            continue
        o, cc = int(ps.const_offset[p]), int(ps.const_count[p])
        gg = g[o:o + cc].astype(np.float64)
        stable, scale = _stable_components(t, c, data, g64, ofit.CORR)
        if not np.any(stable) or scale == 0.0:
            continue
        err = float(np.max(np.abs(gg - g64)[stable]))
        if err > GRAD_RTOL * scale + 1e-7:
            bad.append((p, err / max(scale, 1e-300), gg, g64))
        n_cmp += 1
    assert not bad, bad[:5]
    print(f"compared correlation gradients of {n_cmp} of {ps.n} programs")
    assert n_cmp > 0.4 * ps.n


def test_corr_gradient_affine_invariance_and_degenerate():
    """Outer scale and shift constants get a zero gradient (up to rounding);
    a constant output gets zero; a NaN fitness (an fp32 overflow: e^80 e^80
    is +Inf, classified NaN as O32e does) NaN gradients."""
    data = wl.make_dataset(37, 4000, 2, x_range=(1.0, 3.0), target_len=8)
    texts = [("x0 sin x1 * c0 * c1 +", [1.5, -0.25]),
             ("c0 sin c1 *", [0.3, 2.0]),
             ("x0 exp exp exp x1 exp exp exp * c0 *", [1.0])]
    ps = wl.pack_programs([(progtext.parse(t), c) for t, c in texts])
    f, g, st = _grad(ps, data, kind="corr")
    F0, g0 = og.corr_and_grad(progtext.parse("x0 sin x1 *"), [], data.X, data.y)
    assert abs(f[0] - F0) <= 1e-5 * abs(F0) + 1e-9
    assert np.all(np.abs(g[0:2]) <= 1e-5), g[0:2]
    assert f[1] == 1.0 and np.all(g[2:4] == 0.0)
    assert math.isnan(f[2]) and math.isnan(g[4])


def test_autograd_function_and_adam():
    from paper_2603_12292_amd import autograd as ag
    api = _api()
    w = wl.config_differentiation(N=256, M=5000)
    P = api.DevicePrograms.from_programset(w.programs)
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    owner = ag.const_owner(P)
    consts = P.consts.clone().requires_grad_(True)
    fit = ag.EvalGrad.apply(consts, P, X, y, owner)
    go = torch.randn_like(fit)
    fit.backward(go)
    _, g = api.evaluate_grad(P, X, y)
    expect = go[owner] * g.double()
    got = consts.grad.double()
    fin = torch.isfinite(expect)
    assert torch.allclose(got[fin], expect[fin], rtol=1e-6, atol=0)
    res = ag.tune_constants(P, X, y, steps=20, lr=0.05, record=True)
    before, after = res.fitness_before.cpu().numpy(), res.fitness_after.cpu().numpy()
    ok = np.isfinite(before) & np.isfinite(after)
    ratio = after[ok] / np.maximum(before[ok], 1e-300)
    # gradient steps on each program's own constants: most programs improve
    assert np.median(ratio) < 1.0
    assert np.mean(ratio < 1.0) > 0.6
    # under the correlation fitness 1 - r^2 as well
    res = ag.tune_constants(P, X, y, steps=20, lr=0.05, kind="corr")
    before, after = res.fitness_before.cpu().numpy(), res.fitness_after.cpu().numpy()
    ok = np.isfinite(before) & np.isfinite(after) & (before < 1.0)
    assert np.mean(after[ok] <= before[ok] + 1e-12) > 0.6
    assert np.median(after[ok] - before[ok]) <= 0.0


def test_decoder_passes_agree():
    """Programs of at most 64 tokens are decoded by the first pass (narrow
    LDS scratch), longer ones by the second (wide LDS scratch up to 128
    tokens, global scratch beyond).  The same 390 programs mixing all three
    lengths, grouped by length and shuffled, give bit-identical fitness,
    status and constant gradients per program (same population size, hence
    the same case chunks; each program's result is independent of its
    position and of the list order of both passes)."""
    api = _api()
    rng = np.random.default_rng(77)
    flat = []
    for lo, hi, n in ((3, 64, 300), (65, 128, 60), (129, 300, 30)):
        for _ in range(n):
            t, _ = wl.random_program(rng, int(rng.integers(lo, hi + 1)), 3, allow_const=False)
            flat.append(wl.place_constants(rng, t, int(rng.integers(0, 5))))
    order = rng.permutation(len(flat))
    grouped = wl.pack_programs(flat)
    mixed = wl.pack_programs([flat[i] for i in order])
    data = wl.make_dataset(78, 3000, 3, x_range=(1.0, 5.0), target_len=8)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    for kind in ("mse", "corr"):
        out = []
        for ps in (grouped, mixed):
            f, g, st = api.evaluate_grad(api.DevicePrograms.from_programset(ps), X, y, kind, with_status=True)
            out.append((f.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()))
        (f1, g1, s1), (fm, gm, sm) = out
        assert (s1 == 0).sum() > 350
        for k, i in enumerate(order):
            assert fm[k].view(np.uint64) == f1[i].view(np.uint64), (kind, k, i)
            assert sm[k] == s1[i]
            o, cc = int(mixed.const_offset[k]), int(mixed.const_count[k])
            o1 = int(grouped.const_offset[i])
            assert np.array_equal(gm[o:o + cc].view(np.uint32), g1[o1:o1 + cc].view(np.uint32)), (kind, k, i)


def test_overlapping_constant_ranges():
    """The gradient has the constants' layout, so for beagle_eval_grad the
    constant ranges must not overlap either: a program whose constant range
    overlaps a lower-indexed program's gets BEAGLE_PROG_BAD_LAYOUT (8), NaN
    fitness, and leaves the shared gradient slots to the first."""
    api = _api()
    data = wl.make_dataset(43, 2000, 2, x_range=(1.0, 5.0), target_len=8)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    t0 = progtext.parse("x0 c0 * c1 +")
    t1 = progtext.parse("x1 c0 * x0 +")
    toks = np.array(t0 + t1, dtype=np.uint16)
    consts = np.array([1.5, -0.5], dtype=np.float32)
    P = api.DevicePrograms.from_arrays(toks, [0, len(t0)], [len(t0), len(t1)], consts, [0, 0], [2, 1])
    f, g, st = api.evaluate_grad(P, X, y, "mse", with_status=True)
    f, g, st = f.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    assert list(st) == [0, 8] and math.isnan(f[1]) and math.isfinite(f[0])
    F, gref = og.mse_and_grad(t0, consts, data.X, data.y)
    assert np.allclose(g, gref, rtol=1e-4, atol=1e-7), (g, gref)
    # the same constants as separate ranges: both valid
    Q = api.DevicePrograms.from_arrays(toks, [0, len(t0)], [len(t0), len(t1)], np.concatenate([consts, consts[:1]]),
                                       [0, 2], [2, 1])
    _, _, st = api.evaluate_grad(Q, X, y, "mse", with_status=True)
    assert np.all(st.cpu().numpy() == 0)
