"""Pins of the oracle's MSE gradient with respect to constants (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import grad as og
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


def _torch_graph(tokens, c, X, y):
    """The same program built directly as a torch float64 graph (CPU)."""
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
            else:
                z = x == 0
                st.append(torch.where(z, torch.zeros_like(x), torch.sqrt(torch.abs(torch.where(z, torch.ones_like(x), x)))))
    (yh,) = st
    yt = torch.tensor(y.astype(np.float64))
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
