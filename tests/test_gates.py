"""The parity gates themselves (tests/gates.py), on the CPU: values the
oracle's own fp32 emulation gives pass them; planted mistakes of the kinds a
kernel could make (a wrong value on a well-conditioned program, a wrong
value beyond the first-order bound on an ill-conditioned one, a wrong
class) fail them.  Also: the stored every-program values of the benchmark
workload belong to the inputs the generator draws today."""
import math

import numpy as np
import pytest

import gates
import golden_mid
from oracle import fitness as ofit
from paper_2603_12292_amd import workloads as wl


@pytest.fixture(scope="module")
def tiny_refs():
    w = wl.config_tiny()
    return w, {k: gates.references(w.programs, w.data.X, w.data.y, k, processes=4) for k in (ofit.MSE, ofit.CORR)}


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_fp32_emulation_passes(tiny_refs, kind):
    w, refs = tiny_refs
    s = gates.check(refs[kind].f32, refs[kind], kind, w.data.y, max_ill_frac=0.25)
    assert s.n_value > 200 and s.n_checked >= s.n_finite - 8


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_planted_mistakes_fail(tiny_refs, kind):
    w, refs = tiny_refs
    r = refs[kind]
    at = gates.atol(kind, w.data.y)
    base = r.f32.copy()
    spread = np.max(np.abs(np.array([r.f32] + r.pert) - r.f64), axis=0)
    fin = np.isfinite(r.f64) & np.isfinite(r.f32)
    well = [i for i in np.flatnonzero(fin) if spread[i] <= gates.RTOL_COND * abs(r.f64[i]) + at
            and abs(r.f64[i]) > 1e3 * at]
    ill = [i for i in np.flatnonzero(fin) if i not in set(well) and math.isfinite(r.bound[i])
           and r.bound[i] > 0 and spread[i] > gates.RTOL_COND * abs(r.f64[i]) + at]
    assert well and ill
    # 1e-4 relative on a well-conditioned program: the value gate
    bad = base.copy()
    bad[well[0]] *= 1.0 + 1e-4
    with pytest.raises(AssertionError, match="value|envelope"):
        gates.check(bad, r, kind, w.data.y, max_ill_frac=1.0, max_unchecked_frac=1.0)
    # beyond the bound on an ill-conditioned one: the envelope
    bad = base.copy()
    i = ill[0]
    bad[i] = r.f32[i] + 1.5 * r.bound[i] + 1e-6 * abs(r.f32[i]) + 10 * at
    with pytest.raises(AssertionError, match="envelope"):
        gates.check(bad, r, kind, w.data.y, max_ill_frac=1.0, max_unchecked_frac=1.0)
    # within the bound it passes
    ok = base.copy()
    ok[i] = r.f32[i] + 0.999 * r.bound[i]
    gates.check(ok, r, kind, w.data.y, max_ill_frac=1.0, max_unchecked_frac=1.0)
    # a NaN where the fp32 emulation is finite: the classification gate
    bad = base.copy()
    bad[well[1]] = math.nan
    with pytest.raises(AssertionError, match="classification"):
        gates.check(bad, r, kind, w.data.y, max_ill_frac=1.0, max_unchecked_frac=1.0)


def test_no_comparison_fails():
    """A comparison in which no program reaches the value gate fails."""
    w = wl.config_tiny()
    r = gates.references(w.programs.subset([0, 1, 2]), w.data.X, w.data.y, ofit.CORR)
    nan = np.full(3, math.nan)
    refs = gates.Refs(nan, r.status, nan, [nan, nan], nan)
    with pytest.raises(AssertionError, match="no program value-checked"):
        gates.check(nan, refs, ofit.CORR, w.data.y)


def test_golden_mid_values_match_the_generator():
    w = wl.config_mid()
    g = golden_mid.load(w)   # asserts the input hash
    for kind in (ofit.MSE, ofit.CORR):
        assert len(g[kind].f64) == w.programs.n
        assert np.all(g[kind].status == 0)
    # a spot check of the stored binary64 values against the oracle
    r = gates.references(w.programs, w.data.X, w.data.y, ofit.CORR, subset=[0, 1234, 4095])
    assert np.array_equal(r.f64, g[ofit.CORR].f64[[0, 1234, 4095]], equal_nan=True)
    assert np.array_equal(r.f32, g[ofit.CORR].f32[[0, 1234, 4095]], equal_nan=True)


def test_output_gate_and_planted_mistakes():
    """The output gate on fp32-emulated outputs passes; an output moved by
    twice its per-case bound, or a fitness that is not the fitness of the
    outputs, fails."""
    from oracle import bound as ob
    from oracle import interp
    w = wl.config_tiny()
    progs = [w.programs.program(p) for p in range(12)]
    for kind in (ofit.MSE, ofit.CORR):
        outs = [interp.run(t, c, w.data.X, "o32e") for t, c in progs]
        fits = [ofit.fitness(kind, o, w.data.y) for o in outs]
        ok, free = gates.check_outputs(progs, w.data.X, w.data.y, kind, outs, fits)
        assert ok > 10000
        # a case moved beyond its bound
        k = next(k for k, (t, c) in enumerate(progs) if np.any(ob.case_bounds(t, c, w.data.X)[2][-1] > 0))
        b = ob.case_bounds(*progs[k], w.data.X)[2][-1]
        i = int(np.argmax(b))
        bad = [o.copy() for o in outs]
        bad[k][i] += 2.0 * b[i] + 1e-3 * abs(bad[k][i])
        with pytest.raises(AssertionError, match="output"):
            gates.check_outputs(progs, w.data.X, w.data.y, kind, bad, fits)
        # a fitness that is not that of the outputs
        j = next(j for j, f in enumerate(fits) if math.isfinite(f) and f > 1e-3)
        badf = list(fits)
        badf[j] = fits[j] * (1 + 1e-6)
        with pytest.raises(AssertionError, match="output fitness"):
            gates.check_outputs(progs, w.data.X, w.data.y, kind, outs, badf)
