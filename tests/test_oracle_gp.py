"""Pins of the oracle's generation step and initialisation (CPU only)."""
import math

import numpy as np
import pytest

from oracle import gp, interp, tree
from oracle.philox import Stream, below, unit
from paper_2603_12292_amd import workloads as wl


def _annotate(tokens):
    """Tree with each node's postfix index (independent of gp.subtree_start)."""
    st = []
    for i, t in enumerate(tokens):
        a = gp.arity(int(t) & 0xFF)
        kids = [st.pop() for _ in range(a)][::-1]
        st.append((i, kids))
    return st[0]


def _sizes(node, out):
    i, kids = node
    out[i] = 1 + sum(_sizes(k, out) for k in kids)
    return out[i]


def test_subtree_start_against_tree_sizes():
    rng = np.random.default_rng(5)
    for _ in range(300):
        toks, _ = wl.random_program(rng, int(rng.integers(1, 40)), 3)
        sizes = {}
        _sizes(_annotate(toks), sizes)
        for i in range(len(toks)):
            assert gp.subtree_start(toks, i) == i - sizes[i] + 1


def _swap(nodeA, iA, nodeB, iB, toksA, toksB):
    """Tree-level subtree replacement, serialised back to postfix."""
    def find(node, i):
        if node[0] == i:
            return node
        for k in node[1]:
            r = find(k, i)
            if r is not None:
                return r
        return None

    donor = find(nodeB, iB)
    out = []

    def emit(node, src, inside_donor):
        i, kids = node
        if not inside_donor and src == "A" and i == iA:
            emit(donor, "B", True)
            return
        for k in kids:
            emit(k, src, inside_donor)
        out.append(toksA[i] if src == "A" else toksB[i])

    emit(nodeA, "A", False)
    return out


def test_crossover_splice_equals_tree_swap():
    rng = np.random.default_rng(6)
    for _ in range(40):
        A, _ = wl.random_program(rng, int(rng.integers(1, 12)), 2, allow_const=False)
        B, _ = wl.random_program(rng, int(rng.integers(1, 12)), 2, allow_const=False)
        ta, tb = _annotate(A), _annotate(B)
        for iA in range(len(A)):
            for iB in range(len(B)):
                sA, sB = gp.subtree_start(A, iA), gp.subtree_start(B, iB)
                child = A[:sA] + B[sB:iB + 1] + A[iA + 1:]
                assert child == _swap(ta, iA, tb, iB, A, B)
                assert interp.validate(child, 0, 2)[0] == interp.ST_OK
                assert len(child) == len(A) - (iA - sA + 1) + (iB - sB + 1)


def test_tournament_bruteforce():
    rng = np.random.default_rng(7)
    for trial in range(200):
        N = int(rng.integers(1, 9))
        f = rng.choice([0.5, 1.0, 2.0, np.inf, np.nan], size=N)
        ent = [int(v) for v in rng.integers(0, N, size=4)]
        w = gp.tournament(f, ent)
        finite = [e for e in ent if not math.isnan(f[e])]
        if finite:
            best = min(f[e] for e in finite)
            assert w == min(e for e in finite if f[e] == best)
        else:
            assert w == min(ent)


def _parents(n=24, D=3, seed=8):
    rng = np.random.default_rng(seed)
    progs = [wl.random_program(rng, int(rng.integers(1, 40)), D) for _ in range(n)]
    fit = rng.standard_normal(n)
    fit[::7] = np.nan
    return [p[0] for p in progs], [p[1] for p in progs], fit


def test_child_recomputed_from_raw_draws():
    """Selection and operator choice follow the fixed draw layout exactly."""
    pt, pc, fit = _parents()
    prm = gp.GenParams()
    seed, g = 0xDEADBEEF12345678, 3
    for c in range(len(pt)):
        s = Stream(seed, c, g, 0)
        t = prm.tournament
        ia = gp.tournament(fit, [below(s.draw(1 + k), len(pt)) for k in range(t)])
        ib = gp.tournament(fit, [below(s.draw(1 + t + k), len(pt)) for k in range(t)])
        ch_t, ch_c = gp.make_child(c, pt, pc, fit, 3, prm, seed, g)
        A, B = pt[ia], pt[ib]
        if unit(s.draw(0)) < np.float32(0.9):
            xa = below(s.draw(2 * t + 1), len(A))
            xb = below(s.draw(2 * t + 2), len(B))
            sa, sb = gp.subtree_start(A, xa), gp.subtree_start(B, xb)
            expect = [tk & 0xFF for tk in (A[:sa] + B[sb:xb + 1] + A[xa + 1:])]
            if len(expect) > prm.max_len:
                expect = [tk & 0xFF for tk in A]
            assert [tk & 0xFF for tk in ch_t] == expect
        else:
            assert len(ch_t) == len(A)


def test_mutation_invariants():
    pt, pc, fit = _parents(n=40, seed=9)
    prm = gp.GenParams(p_crossover=0.0, p_mutation=1.0)
    for g in range(1, 6):
        kids = gp.generation(pt, pc, fit, 3, prm, 77, g)
        for c, (t, k) in enumerate(kids):
            assert interp.validate(t, len(k), 3)[0] == interp.ST_OK
            s = Stream(77, c, g, 0)
            ia = gp.tournament(fit, [below(s.draw(1 + j), 40) for j in range(4)])
            A = pt[ia]
            assert len(t) == len(A)
            diff = [i for i in range(len(A))
                    if not ((A[i] & 0xFF) == 10 and (t[i] & 0xFF) == 10) and A[i] != t[i]]
            assert len(diff) <= 1
            for i in diff:
                assert gp.arity(A[i] & 0xFF) == gp.arity(t[i] & 0xFF)


def test_children_valid_and_bounded():
    pt, pc, fit = _parents(n=64, seed=10)
    prm = gp.GenParams(max_len=48)
    kids = gp.generation(pt, pc, fit, 3, prm, 5, 1)
    for t, k in kids:
        assert 1 <= len(t) <= 48
        assert len(k) <= prm.max_consts
        assert interp.validate(t, len(k), 3)[0] == interp.ST_OK
        slots = [tk >> 8 for tk in t if (tk & 0xFF) == 10]
        assert slots == list(range(len(slots)))     # constants renumbered in token order
    tok, ln, cst, cc = gp.to_fixed(kids, 48, 8)
    assert tok.shape == (64, 48) and np.all(tok[0, ln[0]:] == 0)


def _leaf_levels(node, level, out):
    i, kids = node
    if not kids:
        out.append(level)
    for k in kids:
        _leaf_levels(k, level + 1, out)


def test_ramped_half_and_half():
    prm = gp.GenParams()
    pop = gp.init_population(200, 4, prm, seed=99)
    n_depths = 5
    for c, (t, k) in enumerate(pop):
        assert interp.validate(t, len(k), 4)[0] == interp.ST_OK
        d = 2 + c % n_depths
        full = (c // n_depths) % 2 == 0
        levels = []
        _leaf_levels(_annotate(t), 0, levels)
        if full:
            assert set(levels) == {d}
        else:
            assert max(levels) <= d
        assert len(t) <= 2 ** (d + 1) - 1 <= prm.max_len
        assert len(k) <= prm.max_consts
        assert all(prm.const_lo <= v <= prm.const_hi for v in k)
    # deterministic
    assert gp.init_population(20, 4, prm, seed=99) == pop[:20]
    assert gp.init_population(20, 4, prm, seed=98) != pop[:20]


def test_const_value_mapping():
    assert gp.const_value(0, -5.0, 5.0) == -5.0
    u = 0x80000000
    assert gp.const_value(u, -5.0, 5.0) == 0.0
    v = gp.const_value(0xFFFFFFFF, -5.0, 5.0)
    assert v == float(np.float32(-5.0 + 10.0 * (1 - 2.0 ** -24)))


# ---- microcosm selection


def test_microcosm_fraction_matches_order_statistics():
    """tau is the k-th smallest (1-based k = ceil(keep s)) of s uniform draws,
    so for continuous fitness the surviving fraction F(tau) has expectation
    k / (s + 1) (the k-th order statistic of s uniforms)."""
    rng = np.random.default_rng(11)
    f = rng.normal(size=20000)
    for keep, s in ((0.5, 100), (0.25, 100), (1.0, 100), (0.5, 20)):
        k = min(s, max(1, math.ceil(np.float32(keep) * s)))
        fr = [len(gp.survivors(f, gp.microcosm_threshold(f, s, keep, 1000 + g, g))) / len(f) for g in range(300)]
        # standard error of the mean of a Beta(k, s - k + 1) variable over 300 draws
        var = k * (s - k + 1) / ((s + 1) ** 2 * (s + 2))
        assert abs(np.mean(fr) - k / (s + 1)) < 4 * math.sqrt(var / 300) + 2 / len(f), (keep, s, np.mean(fr))


def test_microcosm_degenerate_and_ties():
    nan = float("nan")
    f = np.full(50, nan)
    assert gp.survivors(f, gp.microcosm_threshold(f, 100, 0.5, 1, 1)) == list(range(50))
    f = np.full(50, 2.5)
    assert gp.microcosm_threshold(f, 100, 0.5, 1, 1) == 2.5
    assert gp.survivors(f, 2.5) == list(range(50))
    # NaN individuals never survive a finite threshold; a NaN threshold
    # keeps every finite individual
    f = np.array([1.0, nan, 3.0, 0.5, nan])
    assert gp.survivors(f, 1.0) == [0, 3]
    assert gp.survivors(f, nan) == [0, 2, 3]
    # the threshold is the sample's entry at the keep position: keep = 1
    # gives the worst drawn individual, a tiny keep the best
    rng = np.random.default_rng(3)
    f = rng.normal(size=400)
    from oracle.philox import Stream, below
    st = Stream(9, gp.MICRO_INDEX, 4, gp.MICRO_TAG)
    drawn = [float(f[below(st.draw(j), 400)]) for j in range(100)]
    assert gp.microcosm_threshold(f, 100, 1.0, 9, 4) == max(drawn)
    assert gp.microcosm_threshold(f, 100, 0.001, 9, 4) == min(drawn)


def test_microcosm_mutation_only_children():
    """p_crossover = 0, p_mutation = 1: every child is its drawn survivor
    with at most one token changed (same arity), for any child count."""
    rng = np.random.default_rng(21)
    D = 3
    parents = []
    for _ in range(64):
        toks, consts = wl.random_program(rng, int(rng.integers(3, 30)), D)
        parents.append((toks, consts))
    fit = rng.normal(size=64)
    params = gp.GenParams(p_crossover=0.0, p_mutation=1.0)
    ptok = [p[0] for p in parents]
    pcst = [p[1] for p in parents]
    for n_children in (17, 64, 150):
        kids = gp.generation_microcosm(ptok, pcst, fit, D, params, 5, 3, n_children)
        assert len(kids) == n_children
        tau = gp.microcosm_threshold(fit, 100, 0.5, 5, 3)
        surv = gp.survivors(fit, tau)
        for c, (kt, _) in enumerate(kids):
            from oracle.philox import Stream, below
            s = Stream(5, c, 3, 0)
            a = surv[below(s.draw(1), len(surv))]
            pt = ptok[a]
            assert len(kt) == len(pt)
            diff = [i for i in range(len(pt)) if (kt[i] & 0xFF) != (pt[i] & 0xFF) or
                    ((kt[i] & 0xFF) == gp.VAR and kt[i] != pt[i])]
            assert len(diff) <= 1
            for i in diff:
                assert gp.arity(kt[i] & 0xFF) == gp.arity(pt[i] & 0xFF)



def test_operator_set_one_draws_every_operator():
    """op_set 1 (the paper's sixteen): initialisation and mutation reach the
    seven further unary operators, uniformly among the unary ones."""
    params = gp.GenParams(op_set=1, p_crossover=0.0, p_mutation=1.0)
    pop = gp.init_population(3000, 2, params, seed=5)
    seen = {int(t) & 0xFF for toks, _ in pop for t in toks}
    assert set(range(11, 18)) <= seen and seen <= set(range(18))
    ptok = [t for t, _ in pop]
    pcst = [c for _, c in pop]
    fit = np.zeros(len(pop))
    kids = gp.generation(ptok, pcst, fit, 2, params, 5, 1)
    counts = np.zeros(18)
    for (kt, _), c in zip(kids, range(len(kids))):
        s = Stream(5, c, 1, 0)
        t = params.tournament
        a = gp.tournament(fit, [below(s.draw(1 + k), len(pop)) for k in range(t)])
        pt = ptok[a]
        mpos = below(s.draw(2 * params.tournament + 3), len(pt))
        if gp.arity(int(pt[mpos]) & 0xFF) == 1:
            counts[int(kt[mpos]) & 0xFF] += 1
    un = counts[list(gp.UNARY_EXT)]
    assert un.sum() > 600 and un.min() > 0.5 * un.sum() / 12
    # op_set 0 never produces them
    pop0 = gp.init_population(500, 2, gp.GenParams(), seed=5)
    assert all((int(t) & 0xFF) < 11 for toks, _ in pop0 for t in toks)
