"""beagle_eval_static, the evaluation that allocates nothing (its workspace
is the library's static per-device array), against beagle_eval through the
C ABI: identical fitness and status bits on two calls in a row, the second
with a smaller population and dataset (the array keeps the first call's
contents), and a size beyond the array rejected before anything runs."""
import ctypes

import numpy as np
import pytest

from oracle import fitness as ofit
from paper_2603_12292_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _call_both(lib, api, ps, data, kind):
    P = api.DevicePrograms.from_programset(ps)
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    pst = P.struct()
    dst = api._dataset(X, y, P.device)
    ref, ref_st = api.evaluate(P, X, y, "mse" if kind == ofit.MSE else "corr", with_status=True)
    fit = torch.full((ps.n,), -7.0, dtype=torch.float64, device="cuda")
    st = torch.full((ps.n,), 99, dtype=torch.int8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.beagle_eval_static(ctypes.byref(pst), ctypes.byref(dst), kind, ctypes.c_void_p(fit.data_ptr()),
                                ctypes.c_void_p(st.data_ptr()), ctypes.c_void_p(stream))
    assert rc == 0, lib.beagle_last_error()
    torch.cuda.synchronize()
    a, b = ref.cpu().numpy(), fit.cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (kind, np.flatnonzero(a.view(np.uint64) != b.view(np.uint64))[:5])
    assert np.array_equal(ref_st.cpu().numpy(), st.cpu().numpy())
    return b


@pytest.mark.parametrize("kind", [ofit.CORR, ofit.MSE])
def test_static_matches_eval_twice_smaller_second(kind):
    from paper_2603_12292_amd import _lib, api
    lib = _lib.load()
    big = wl.random_population(501, 2048, 3, 60, 5)
    data_big = wl.make_dataset(502, 60_000, 5, x_range=(1.0, 10.0), target_len=16)
    small = wl.random_population(503, 97, 2, 20, 2)
    data_small = wl.make_dataset(504, 777, 2, x_range=(1.0, 5.0), target_len=6)
    print(f"static kind={kind}: N=2048 M=60000 D=5", flush=True)
    f1 = _call_both(lib, api, big, data_big, kind)
    print(f"static kind={kind}: N=97 M=777 D=2", flush=True)
    f2 = _call_both(lib, api, small, data_small, kind)
    assert np.isfinite(f1).sum() > 1000 and np.isfinite(f2).sum() > 40


def test_static_rejects_beyond_the_array():
    from paper_2603_12292_amd import _lib
    lib = _lib.load()
    # sizes only (fake device addresses): 16 inputs x 2^24 cases need 1 GiB of staging
    P = _lib.Programs(0x1000, 70, 0x2000, 0x3000, 0x4000, 20, 0x5000, 0x6000, 10)
    D = _lib.Dataset(0x7000, 0x8000, 1 << 24, 16)
    out = ctypes.c_void_p(0x9000)
    rc = lib.beagle_eval_static(ctypes.byref(P), ctypes.byref(D), _lib.FIT_MSE, out, None, None)
    assert rc == _lib.E_NOMEM
    assert b"static" in lib.beagle_last_error()
