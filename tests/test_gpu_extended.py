"""The paper's further operators (x^2, 1/x, tan, asin, acos, atan, tanh) on
the GPU: operator accuracy, population fitness, gradients and generation
against the oracle."""
import math

import numpy as np
import pytest

import gates
from oracle import fitness as ofit
from oracle import gp
from oracle import grad as og
from oracle import interp
from paper_2603_12292_amd import workloads as wl
from progtext import parse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ALL_UNARY = wl.UNARY_OPS + wl.EXTENDED_OPS
NAMES = ("sq", "inv", "tan", "asin", "acos", "atan", "tanh")


def _api():
    from paper_2603_12292_amd import api
    return api


def _population(seed, N, lo, hi, D, **kw):
    ps = wl.random_population(seed, N, lo, hi, D, unary=ALL_UNARY, **kw)
    n_ext = sum(any((int(t) & 0xFF) >= 11 for t in ps.program(p)[0]) for p in range(ps.n))
    assert n_ext > N // 2
    return ps


def test_operator_accuracy():
    """Each operator alone on a wide spread of binary32 inputs and special
    values: NaN/Inf pattern identical to the binary32 rounding of the exact
    result, x^2 and 1/x bit-exact, the others within 4 ulp."""
    api = _api()
    rng = np.random.default_rng(17)
    x = np.concatenate([rng.uniform(-1.0, 1.0, 4000), rng.standard_normal(4000) * 10.0 ** rng.integers(-30, 30, 4000),
                        [0.0, -0.0, 1.0, -1.0, 1.0000001, np.inf, -np.inf, np.nan, 1e-45, 3.4e38, 1.5707964,
                         -1.5707964, 20.0, -9.0, 1e30]]).astype(np.float32)
    X = x[:, None]
    ps = wl.pack_programs([(parse(f"x0 {name}"), []) for name in NAMES])
    out = api.predict(api.DevicePrograms.from_programset(ps), torch.from_numpy(X).cuda()).cpu().numpy()
    for j, name in enumerate(NAMES):
        ref64 = interp.run(parse(f"x0 {name}"), [], X, "o64")
        with np.errstate(all="ignore"):
            ref = ref64.astype(np.float32)
        got = out[j]
        assert np.array_equal(np.isnan(got), np.isnan(ref)), name
        assert np.array_equal(np.isinf(got), np.isinf(ref)) and np.array_equal(got[np.isinf(got)], ref[np.isinf(ref)]), name
        fin = np.isfinite(ref)
        if name in ("sq", "inv"):
            assert np.array_equal(got[fin].view(np.uint32), ref[fin].view(np.uint32)), name
            continue
        # ulp of the reference (the spacing at its magnitude, subnormal floor)
        ulp = np.spacing(np.abs(ref[fin])).astype(np.float64)
        err = np.abs(got[fin].astype(np.float64) - ref64[fin])
        worst = float(np.max(err / np.maximum(ulp, 2.0 ** -149)))
        print(f"{name}: max error {worst:.2f} ulp")
        assert worst <= 4.0, (name, worst)


def _class_stable(f32e, others, i):
    c = ofit.classify(f32e[i])
    return all(ofit.classify(o[i]) == c for o in others)


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_population_fitness(kind):
    """Random programs over all twelve unary operators (N=1000, L in 3..40,
    D=3, M=5000, inputs in (-1.2, 1.2) so that asin and acos meet both sides
    of their domain): classification as the binary32 oracle wherever that is
    stable across the oracle's modes, values within the usual gate."""
    api = _api()
    ps = _population(1101 + kind, 1000, 3, 40, 3, const_range=(-1.5, 1.5))
    data = wl.make_dataset(1102, 5000, 3, x_range=(-1.2, 1.2), target_len=8)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    f, st = api.evaluate(api.DevicePrograms.from_programset(ps), X, y, "mse" if kind == ofit.MSE else "corr",
                         with_status=True)
    gpu = f.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    r = gates.references(ps, data.X, data.y, kind)
    unstable = [i for i in range(ps.n) if not _class_stable(r.f32, [r.f64] + r.pert, i)]
    keep = [i for i in range(ps.n) if i not in set(unstable)]
    n_nan = sum(math.isnan(r.f32[i]) for i in keep)
    print(f"{len(unstable)} programs of unstable class, {n_nan} NaN fitness")
    assert len(unstable) < 0.05 * ps.n
    assert n_nan > 20  # asin / acos / 1/x produce invalid values
    s = gates.check(gpu[keep], r.take(keep), kind, data.y, max_ill_frac=0.35, max_unchecked_frac=0.1,
                    label=f"extended kind={kind}")
    # about two programs in three are NaN (asin, acos, 1/x) or unstable
    print(s, "output gate:", gates.output_gate(ps, data.X, data.y, kind, gpu[keep], s, idx=keep, label="ext"))
    assert s.n_value > 0.18 * ps.n and s.n_checked >= 0.9 * s.n_finite


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_gradient(kind):
    """Constant gradients of programs with the further operators (value-tape
    adjoint) against the oracle, on components stable under its fp32 modes."""
    api = _api()
    rng = np.random.default_rng(1201 + kind)
    progs = []
    while len(progs) < 400:
        t, _ = wl.random_program(rng, int(rng.integers(4, 30)), 3, allow_const=False, unary=ALL_UNARY)
        if not any((x & 0xFF) >= 11 for x in t):
            continue
        progs.append(wl.place_constants(rng, t, int(rng.integers(1, 5)), const_lo=-1.0, const_hi=1.0))
    ps = wl.pack_programs(progs)
    data = wl.make_dataset(1202, 3000, 3, x_range=(-0.9, 0.9), target_len=8)
    P = api.DevicePrograms.from_programset(ps)
    f, g, st = api.evaluate_grad(P, torch.from_numpy(data.X).cuda(), torch.from_numpy(data.y).cuda(),
                                 "mse" if kind == ofit.MSE else "corr", with_status=True)
    f, g, st = f.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    fn = og.mse_and_grad if kind == ofit.MSE else og.corr_and_grad
    n_cmp, bad = 0, []
    for p in range(ps.n):
        t, c = ps.program(p)
        F, g64 = fn(t, c, data.X, data.y)
        if not (math.isfinite(F) and np.all(np.isfinite(g64))) or (kind == ofit.CORR and not 0.0 < F < 1.0):
            continue
        spread = np.zeros_like(g64)
        for mode, seed in (("o32e", 0), ("o32p", 1), ("o32p", 2)):
            _, gm = fn(t, c, data.X, data.y, mode, seed)
            spread = np.maximum(spread, np.where(np.isfinite(gm), np.abs(gm - g64), np.inf))
        scale = float(np.max(np.abs(g64)))
        stable = spread <= 1e-5 * scale
        if not np.any(stable) or scale == 0.0:
            continue
        o, cc = int(ps.const_offset[p]), int(ps.const_count[p])
        err = float(np.max(np.abs(g[o:o + cc].astype(np.float64) - g64)[stable]))
        if err > 1e-4 * scale + 1e-7:
            bad.append((p, err / scale))
        n_cmp += 1
    assert not bad, bad[:5]
    # about half the programs (MSE) and a tenth (1 - r^2) have a finite
    # fitness and gradient components stable under the fp32 modes
    print(f"compared gradients of {n_cmp} programs")
    assert n_cmp > (150 if kind == ofit.MSE else 30)


def test_init_and_generation_bit_exact():
    """Operator set 1 (the paper's sixteen): initialisation, the tournament
    step and the microcosm step bit-exact against the oracle."""
    api = _api()
    kw = dict(op_set=1, p_crossover=0.5, p_mutation=0.5)
    op, ap = gp.GenParams(**kw), api.GenParams(**kw)
    D, seed = 3, 0x5EED_0F_16
    s = api.init_population(1500, D, ap, seed, problem=2)
    torch.cuda.synchronize()
    ref = gp.to_fixed(gp.init_population(1500, D, op, seed, problem=2), op.max_len, op.max_consts)
    tok = s.tokens.cpu().numpy().view(np.uint16)
    assert np.array_equal(s.len.cpu().numpy(), ref[1]) and np.array_equal(tok, ref[0])
    assert np.array_equal(s.consts.cpu().numpy().view(np.uint32), ref[2].view(np.uint32))
    assert ((tok & 0xFF) >= 11).any()
    ptok = [list(ref[0][i, :ref[1][i]]) for i in range(1500)]
    pcst = [list(ref[2][i, :ref[3][i]]) for i in range(1500)]
    rng = np.random.default_rng(3)
    fit = rng.standard_normal(1500)
    par = s.programs()
    fdev = torch.from_numpy(fit).cuda()
    kids = api.generation(par, fdev, ap, D, seed, 4)
    r = gp.to_fixed(gp.generation(ptok, pcst, fit, D, op, seed, 4), op.max_len, op.max_consts)
    assert np.array_equal(kids.len.cpu().numpy(), r[1])
    assert np.array_equal(kids.tokens.cpu().numpy().view(np.uint16), r[0])
    kids = api.generation_microcosm(par, fdev, ap, D, seed, 5, 1000)
    r = gp.to_fixed(gp.generation_microcosm(ptok, pcst, fit, D, op, seed, 5, 1000), op.max_len, op.max_consts)
    assert np.array_equal(kids.len.cpu().numpy(), r[1])
    assert np.array_equal(kids.tokens.cpu().numpy().view(np.uint16), r[0])
    assert np.array_equal(kids.consts.cpu().numpy().view(np.uint32), r[2].view(np.uint32))


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_resident_class1_small_case_set(kind):
    """The paper's regime with its full operator table: 6000 programs using
    the further operators (register-need class 1 at least) on 512 cases take
    the resident-inputs kernels; the same programs in slices of 2000 (below
    the resident threshold: the block kernels) give the same classification
    and values within summation-order rounding, and a sample passes the
    oracle gate."""
    api = _api()
    name = "mse" if kind == ofit.MSE else "corr"
    ps = _population(1301 + kind, 6000, 3, 30, 3, const_range=(-1.5, 1.5))
    data = wl.make_dataset(1302, 512, 3, x_range=(-1.2, 1.2), target_len=8)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    whole, st = api.evaluate(api.DevicePrograms.from_programset(ps), X, y, name, with_status=True)
    whole = whole.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    parts = [api.evaluate(api.DevicePrograms.from_programset(ps.subset(list(range(p0, p0 + 2000)))), X, y, name)
             .cpu().numpy() for p0 in range(0, 6000, 2000)]
    part = np.concatenate(parts)
    assert [ofit.classify(v) for v in whole] == [ofit.classify(v) for v in part]
    ok = np.isfinite(part)
    assert ok.sum() > 1000
    scale = np.maximum(np.abs(part[ok]), 1e-300)
    assert np.all(np.abs(whole[ok] - part[ok]) <= 1e-9 * scale + 1e-12)
    sub = list(range(0, 6000, 37))
    r = gates.references(ps, data.X, data.y, kind, subset=sub)
    keep = [j for j in range(len(sub)) if _class_stable(r.f32, [r.f64] + r.pert, j)]
    s = gates.check(whole[sub][keep], r.take(keep), kind, data.y, max_ill_frac=0.4, max_unchecked_frac=0.1,
                    label=f"resident class 1 {name}")
    print(s, "output gate:", gates.output_gate(ps, data.X, data.y, kind, whole[sub][keep], s,
                                               idx=[sub[j] for j in keep], label="ext resident"))
    assert s.n_value > 20 and s.n_checked >= 0.9 * s.n_finite
