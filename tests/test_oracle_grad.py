"""Pins of the oracle's MSE gradient with respect to constants (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import grad as og
from oracle import interp
from paper_2603_12292_amd import workloads as wl
from progtext import parse


def _data(M=400, D=3, seed=31):
    return wl.make_dataset(seed, M, D, x_range=(1.0, 5.0), target_len=8)


def test_closed_forms():
    d = _data()
    x = d.X[:, 0].astype(np.float64)
    y = d.y.astype(np.float64)
    M = len(y)
    c = np.float32(1.75)
    cf = float(c)
    # c0 * x0: dF/dc = 2/M sum (c x - y) x
    F, g = og.mse_and_grad(parse("c0 x0 *"), [c], d.X, d.y)
    assert g[0] == pytest.approx(2.0 / M * math.fsum(((cf * x - y) * x).tolist()), rel=1e-12)
    # x0 + c0: dF/dc = 2/M sum (x + c - y)
    F, g = og.mse_and_grad(parse("x0 c0 +"), [c], d.X, d.y)
    assert g[0] == pytest.approx(2.0 / M * math.fsum((x + cf - y).tolist()), rel=1e-12)
    # sin(c0): dF/dc = 2/M sum (sin c - y) cos c
    F, g = og.mse_and_grad(parse("c0 sin"), [c], d.X, d.y)
    assert g[0] == pytest.approx(2.0 / M * math.fsum((math.sin(cf) - y).tolist()) * math.cos(cf), rel=1e-12)
    # a slot read twice: c0 * c0 -> 2/M sum (c^2 - y) 2c
    F, g = og.mse_and_grad(parse("c0 c0 *"), [c], d.X, d.y)
    assert g[0] == pytest.approx(2.0 / M * math.fsum((cf * cf - y).tolist()) * 2 * cf, rel=1e-12)
    # unused slot -> 0
    F, g = og.mse_and_grad(parse("c0 x0 *"), [c, np.float32(3.0)], d.X, d.y)
    assert g[1] == 0.0


def _torch_graph(tokens, c, X, y, corr=False):
    """The same program built directly as a torch float64 graph (CPU); the
    MSE, or 1 - r^2 from the centred sums."""
    Xt = torch.tensor(X.astype(np.float64))
    st = []
    for t in tokens:
        op, arg = t & 0xFF, t >> 8
        if op == 9:
            st.append(Xt[:, arg])
        elif op == 10:
            st.append(c[arg].expand(X.shape[0]))
        elif op < 4:
            b = st.pop()
            a = st.pop()
            if op == 0:
                st.append(a + b)
            elif op == 1:
                st.append(a - b)
            elif op == 2:
                st.append(a * b)
            else:
                z = b == 0
                st.append(torch.where(z, torch.ones_like(a), a / torch.where(z, torch.ones_like(b), b)))
        else:
            x = st.pop()
            if op == 4:
                st.append(torch.sin(x))
            elif op == 5:
                st.append(torch.cos(x))
            elif op == 6:
                st.append(torch.exp(torch.clamp(x, -80.0, 80.0)))
            elif op == 7:
                z = x == 0
                st.append(torch.where(z, torch.zeros_like(x), torch.log(torch.abs(torch.where(z, torch.ones_like(x), x)))))
            elif op == 8:
                z = x == 0
                st.append(torch.where(z, torch.zeros_like(x), torch.sqrt(torch.abs(torch.where(z, torch.ones_like(x), x)))))
            else:
                f = {11: torch.square, 12: torch.reciprocal, 13: torch.tan, 14: torch.asin, 15: torch.acos,
                     16: torch.atan, 17: torch.tanh}[op]
                st.append(f(x))
    (yh,) = st
    yt = torch.tensor(y.astype(np.float64))
    if corr:
        u = yh - yh.mean()
        w = yt - yt.mean()
        r = (u * w).sum() / torch.sqrt((u * u).sum() * (w * w).sum())
        return 1.0 - r * r
    return torch.mean((yh - yt) ** 2)


def test_against_torch_autograd_float64():
    d = _data(M=300)
    rng = np.random.default_rng(41)
    n = 0
    for _ in range(150):
        toks, _ = wl.random_program(rng, int(rng.integers(4, 30)), 3, allow_const=False)
        toks, consts = wl.place_constants(rng, toks, int(rng.integers(1, 5)))
        F, g = og.mse_and_grad(toks, consts, d.X, d.y)
        if not math.isfinite(F) or not np.all(np.isfinite(g)):
            continue
        c = torch.tensor(np.asarray(consts, dtype=np.float32).astype(np.float64), requires_grad=True)
        Ft = _torch_graph(toks, c, d.X, d.y)
        Ft.backward()
        gt = c.grad.numpy()
        assert F == pytest.approx(Ft.item(), rel=1e-12)
        scale = max(1e-300, float(np.max(np.abs(gt))))
        assert np.all(np.abs(g - gt) <= 1e-9 * scale), (toks, g, gt)
        n += 1
    assert n > 60


def test_against_central_differences():
    """Analytic gradient vs FP64 central differences, where the differences converge.

    A slot is compared when no +-h step flips a protected branch and the
    differences at steps h and h/10 agree to 1e-4 (programs such as
    sin(e^80 * x) oscillate far faster than any step can resolve).
    """
    d = _data(M=300)
    rng = np.random.default_rng(43)
    n = 0
    for _ in range(120):
        toks, _ = wl.random_program(rng, int(rng.integers(4, 24)), 3, allow_const=False)
        toks, consts = wl.place_constants(rng, toks, int(rng.integers(1, 4)))
        F, g = og.mse_and_grad(toks, consts, d.X, d.y)
        if not math.isfinite(F) or not np.all(np.isfinite(g)):
            continue
        fd1, ok1 = og.central_fd(toks, consts, d.X, d.y, rel_step=1e-5)
        fd2, ok2 = og.central_fd(toks, consts, d.X, d.y, rel_step=1e-6)
        for j in np.nonzero(ok1 & ok2)[0]:
            if abs(fd1[j] - fd2[j]) > 1e-4 * max(abs(fd2[j]), 1e-12):
                continue
            h = 1e-6 * max(1.0, abs(float(consts[j])))
            tol = 1e-5 * max(abs(g[j]), abs(fd2[j])) + 1e-15 * abs(F) / h + 1e-12
            assert abs(g[j] - fd2[j]) <= tol, (toks, j, g[j], fd1[j], fd2[j])
            n += 1
    assert n > 40


def test_fp32_modes_are_close_for_benign_programs():
    """The fp32-emulating gradient modes differ from binary64 by rounding only."""
    d = _data(M=300)
    rng = np.random.default_rng(44)
    n = 0
    for _ in range(60):
        toks, _ = wl.random_program(rng, int(rng.integers(4, 20)), 3, allow_const=False)
        toks, consts = wl.place_constants(rng, toks, int(rng.integers(1, 4)))
        F, g = og.mse_and_grad(toks, consts, d.X, d.y)
        if not (math.isfinite(F) and np.all(np.isfinite(g))) or np.max(np.abs(g)) == 0:
            continue
        for mode, seed in (("o32e", 0), ("o32p", 1)):
            F32, g32 = og.mse_and_grad(toks, consts, d.X, d.y, mode, seed)
            if np.all(np.isfinite(g32)):
                # rounding-level agreement for most programs; never wild for all
                n += np.max(np.abs(g32 - g)) <= 1e-4 * np.max(np.abs(g))
    assert n >= 60
    # exactly representable case: c0 * x0 with small integers is exact in fp32
    X = np.array([[1.0], [2.0], [3.0]], dtype=np.float32)
    y = np.array([1.0, 5.0, 2.0], dtype=np.float32)
    F, g = og.mse_and_grad([10, 9, 2], [2.0], X, y)
    F32, g32 = og.mse_and_grad([10, 9, 2], [2.0], X, y, "o32e")
    assert F == F32 and g[0] == pytest.approx(g32[0], rel=1e-7)


# ---- correlation fitness 1 - r^2


def test_corr_affine_invariance():
    """1 - r^2 does not change under y_hat -> a y_hat + b (a > 0), so the
    constants of "P c0 * c1 +" have zero gradient; P's own constants do not."""
    d = _data(M=300)
    rng = np.random.default_rng(51)
    n = 0
    for _ in range(40):
        toks, _ = wl.random_program(rng, int(rng.integers(3, 16)), 3, allow_const=False)
        toks, consts = wl.place_constants(rng, toks, 1)
        t2 = list(toks) + parse("c1 * c2 +")
        c2 = list(consts) + [np.float32(1.7), np.float32(-0.4)]
        F, g = og.corr_and_grad(t2, c2, d.X, d.y)
        F0, g0 = og.corr_and_grad(toks, consts, d.X, d.y)
        if not (math.isfinite(F) and F < 1.0 and np.all(np.isfinite(g))):
            continue
        assert F == pytest.approx(F0, rel=1e-9, abs=1e-12)
        scale = max(abs(g0[0]), 1e-6)
        assert abs(g[1]) <= 1e-9 * scale + 1e-13 and abs(g[2]) <= 1e-9 * scale + 1e-13, (toks, g)
        # the inner constant's gradient scales by 1 (r is unchanged)
        assert g[0] == pytest.approx(g0[0], rel=1e-6, abs=1e-12)
        n += 1
    assert n > 15


def test_corr_against_torch_autograd_float64():
    d = _data(M=300)
    rng = np.random.default_rng(52)
    n = 0
    for _ in range(150):
        toks, _ = wl.random_program(rng, int(rng.integers(4, 30)), 3, allow_const=False)
        toks, consts = wl.place_constants(rng, toks, int(rng.integers(1, 5)))
        F, g = og.corr_and_grad(toks, consts, d.X, d.y)
        if not math.isfinite(F) or not np.all(np.isfinite(g)) or F >= 1.0 or F <= 0.0:
            continue
        # the seeds sum to zero only up to rounding, so a constant term of
        # huge magnitude (e^(c e^c)) leaves noise of its size in its slots'
        # (exactly zero) gradients, differently in each summation order:
        # compared on outputs of moderate magnitude
        y_hat = interp.run(toks, consts, d.X, "o64")
        if not np.max(np.abs(y_hat)) < 1e4:
            continue
        c = torch.tensor(np.asarray(consts, dtype=np.float32).astype(np.float64), requires_grad=True)
        Ft = _torch_graph(toks, c, d.X, d.y, corr=True)
        Ft.backward()
        gt = c.grad.numpy()
        assert F == pytest.approx(Ft.item(), rel=1e-9, abs=1e-12)
        scale = max(1e-300, float(np.max(np.abs(gt))))
        # absolute floor: constants that only shift or scale the output have
        # an exactly zero gradient, computed by both sides as rounding noise
        assert np.all(np.abs(g - gt) <= 1e-7 * scale + 1e-14), (toks, g, gt)
        n += 1
    assert n > 50


def test_corr_against_central_differences():
    d = _data(M=300)
    rng = np.random.default_rng(53)
    n = 0
    for _ in range(100):
        toks, _ = wl.random_program(rng, int(rng.integers(4, 20)), 3, allow_const=False)
        toks, consts = wl.place_constants(rng, toks, int(rng.integers(1, 4)))
        F, g = og.corr_and_grad(toks, consts, d.X, d.y)
        if not math.isfinite(F) or not np.all(np.isfinite(g)):
            continue
        fd1, ok1 = og.central_fd(toks, consts, d.X, d.y, rel_step=1e-5, kind=og.CORR_KIND)
        fd2, ok2 = og.central_fd(toks, consts, d.X, d.y, rel_step=1e-6, kind=og.CORR_KIND)
        for j in np.nonzero(ok1 & ok2)[0]:
            if abs(fd1[j] - fd2[j]) > 1e-4 * max(abs(fd2[j]), 1e-12):
                continue
            h = 1e-6 * max(1.0, abs(float(consts[j])))
            tol = 1e-5 * max(abs(g[j]), abs(fd2[j])) + 1e-15 / h + 1e-12
            assert abs(g[j] - fd2[j]) <= tol, (toks, j, g[j], fd1[j], fd2[j])
            n += 1
    assert n > 30


def test_corr_degenerate_cases():
    d = _data(M=200)
    # constant output: Sxx == 0, F = 1, zero gradient
    F, g = og.corr_and_grad(parse("c0 sin c1 *"), [np.float32(0.3), np.float32(2.0)], d.X, d.y)
    assert F == 1.0 and np.all(g == 0.0)
    # a NaN output in one case: F is NaN and so is every used slot's gradient
    X = d.X.copy()
    X[7, 0] = np.float32(np.inf)
    F, g = og.corr_and_grad(parse("x0 x0 - c0 *"), [np.float32(1.5)], X, d.y)
    assert math.isnan(F) and math.isnan(g[0])


_EXT = (4, 5, 6, 7, 8) + tuple(range(11, 18))


def test_tanh_derivative_where_tanh_saturates():
    """d tanh(c) / dc = sech^2 c keeps full relative accuracy at c = 20,
    where 1 - tanh^2 c has none."""
    d = _data()
    y = d.y.astype(np.float64)
    M = len(y)
    F, g = og.mse_and_grad(parse("c0 tanh"), [np.float32(20.0)], d.X, d.y)
    sech2 = 1.0 / math.cosh(20.0) ** 2
    assert g[0] == pytest.approx(2.0 / M * math.fsum((math.tanh(20.0) - y).tolist()) * sech2, rel=1e-12)


def test_extended_closed_forms():
    """The paper's further operators: dF/dc of f(c x0) against hand-derived
    derivatives (x0 in [1, 5], c small enough that asin/acos stay defined)."""
    d = _data()
    x = d.X[:, 0].astype(np.float64)
    y = d.y.astype(np.float64)
    M = len(y)
    c = np.float32(0.125)
    cf = float(c)
    u = cf * x
    cases = {"sq": (u * u, 2 * u), "inv": (1 / u, -1 / (u * u)), "tan": (np.tan(u), 1 + np.tan(u) ** 2),
             "asin": (np.arcsin(u), 1 / np.sqrt(1 - u * u)), "acos": (np.arccos(u), -1 / np.sqrt(1 - u * u)),
             "atan": (np.arctan(u), 1 / (1 + u * u)), "tanh": (np.tanh(u), 1 - np.tanh(u) ** 2)}
    for name, (val, dval) in cases.items():
        F, g = og.mse_and_grad(parse(f"c0 x0 * {name}"), [c], d.X, d.y)
        assert F == pytest.approx(math.fsum(((val - y) ** 2).tolist()) / M, rel=1e-12), name
        assert g[0] == pytest.approx(2.0 / M * math.fsum(((val - y) * dval * x).tolist()), rel=1e-10), name


@pytest.mark.parametrize("kind", [og.MSE_KIND, og.CORR_KIND])
def test_extended_against_torch_autograd_float64(kind):
    """Random programs over all twelve unary operators against torch's own
    derivatives of tan, asin, acos, atan, tanh, square and reciprocal."""
    d = _data(M=300)
    rng = np.random.default_rng(47 + kind)
    n = 0
    for _ in range(200):
        toks, _ = wl.random_program(rng, int(rng.integers(4, 24)), 3, allow_const=False, unary=_EXT)
        if not any((t & 0xFF) >= 11 for t in toks):
            continue
        toks, consts = wl.place_constants(rng, toks, int(rng.integers(1, 4)), const_lo=-1.0, const_hi=1.0)
        if not any((t & 0xFF) == 9 for t in toks):
            continue  # a constant output: 1 - r^2 is 1 by convention, gradient 0
        X64 = d.X.astype(np.float64)
        F, g = og.fitness_and_grad64(kind, toks, np.asarray(consts, dtype=np.float32).astype(np.float64), X64,
                                     d.y.astype(np.float64))
        if not math.isfinite(F) or not np.all(np.isfinite(g)):
            continue
        # as for the base operators: 1 - r^2 compared on outputs of moderate
        # magnitude, with an absolute floor for exactly-zero gradients that
        # both sides compute as rounding noise
        if kind == og.CORR_KIND and not np.max(np.abs(interp.run(toks, consts, d.X, "o64"))) < 1e4:
            continue
        c = torch.tensor(np.asarray(consts, dtype=np.float32).astype(np.float64), requires_grad=True)
        Ft = _torch_graph(toks, c, d.X, d.y, corr=kind == og.CORR_KIND)
        if not torch.isfinite(Ft):
            continue
        Ft.backward()
        gt = c.grad.numpy()
        if not np.all(np.isfinite(gt)):
            continue
        assert F == pytest.approx(Ft.item(), rel=1e-9, abs=1e-12)
        scale = max(1e-300, float(np.max(np.abs(gt))))
        # torch differentiates tanh as 1 - tanh^2, which keeps only noise of
        # about 1e-16 where tanh saturates (the oracle uses sech^2): floor
        floor = 1e-12 * max(1.0, abs(F))
        assert np.all(np.abs(g - gt) <= 1e-7 * scale + floor), (toks, g, gt)
        n += 1
    assert n > 25
