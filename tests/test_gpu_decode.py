"""The two decoders of programs of at most 64 tokens -- a wave per program
with a token per lane (the default) and a thread per program -- give the
same statuses and bit-identical fitness, per-case outputs and constant
gradients.  The populations exercise every status a program can have, the
further operators, fused pairs and reversed operators, constant-free
subtrees, every adjoint list, long unary chains (the deepest trees of a
64-token program) and programs longer than 64 tokens (decoded by the thread
kernel under either choice); large populations span many waves and
workgroups.  The decoders share no code beyond the word format, so
agreement checks each against the other; the oracle parity of the decoded
programs is what the other GPU tests check."""
import numpy as np
import pytest

from paper_2603_12292_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _api():
    from paper_2603_12292_amd import api
    return api


def _contexts():
    api = _api()
    cw, ct = api.Context(0), api.Context(0)
    ct.set_decoder("thread")
    return cw, ct


def _mixed_population(seed, n, D):
    """Valid programs of 1..64 tokens over the nine and the sixteen
    operators, a few longer ones, token soup (bad opcodes, underflow, bad
    variables and constants, a final depth other than one) and empty
    programs."""
    rng = np.random.default_rng(seed)
    ext = (wl.SIN, wl.COS, wl.EXP, wl.LOG, wl.SQRT, wl.SQUARE, wl.RECIP, wl.TAN, wl.ASIN, wl.ACOS, wl.ATAN,
           wl.TANH)
    progs = []
    for i in range(n):
        r = i % 10
        if r < 6:
            progs.append(wl.random_program(rng, int(rng.integers(1, 65)), D))
        elif r == 6:
            progs.append(wl.random_program(rng, int(rng.integers(1, 65)), D, unary=ext))
        elif r == 7:
            progs.append(wl.random_program(rng, int(rng.integers(65, 100)), D))
        elif r == 8:
            L = int(rng.integers(1, 65))
            toks = (rng.integers(0, 20, L) | (rng.integers(0, D + 2, L) << 8)).astype(int).tolist()
            progs.append((toks, [0.5, -1.25, 2.0]))
        else:
            k = int(rng.integers(0, 64))
            progs.append(([wl.tok(wl.VAR, 0)] + [wl.tok(int(rng.choice([wl.SIN, wl.SQRT, wl.EXP])))] * k, []))
    progs.append(([], []))
    progs.append(([wl.tok(wl.VAR, 0), wl.tok(wl.VAR, 1)], []))                       # final depth 2
    progs.append(([wl.tok(wl.VAR, 0), wl.tok(wl.CONST, 0), wl.tok(wl.VAR, 1), wl.tok(wl.ADD)], [2.0]))
    progs.append(([wl.tok(wl.VAR, 0)] * 32 + [wl.tok(wl.SUB)] * 31, []))
    progs.append(([wl.tok(wl.CONST, 0)] * 32 + [wl.tok(wl.DIV)] * 31, [1.5]))
    return wl.pack_programs(progs)


def _short_population(seed, n, D, lmax):
    """The mixed population's kinds with every program of at most lmax
    tokens (lmax 0: lengths 1..16 half the time, 17..32 three times in ten,
    33..64 otherwise), empty programs and final depth two among them, so that
    the wave decoder takes its programs four (16 tokens), two (32) or one at
    a time, in every mixture."""
    rng = np.random.default_rng(seed)
    ext = (wl.SIN, wl.COS, wl.EXP, wl.LOG, wl.SQRT, wl.SQUARE, wl.RECIP, wl.TAN, wl.ASIN, wl.ACOS, wl.ATAN,
           wl.TANH)

    def length():
        if lmax:
            return int(rng.integers(1, lmax + 1))
        u = rng.random()
        return int(rng.integers(1, 17)) if u < 0.5 else int(rng.integers(17, 33)) if u < 0.8 else \
            int(rng.integers(33, 65))

    progs = []
    for i in range(n):
        r = i % 10
        if r < 6:
            progs.append(wl.random_program(rng, length(), D))
        elif r == 6:
            progs.append(wl.random_program(rng, length(), D, unary=ext))
        elif r == 7:
            progs.append(([], []) if i % 20 == 7 else ([wl.tok(wl.VAR, 0), wl.tok(wl.VAR, 1)], []))
        elif r == 8:
            L = length()
            toks = (rng.integers(0, 20, L) | (rng.integers(0, D + 2, L) << 8)).astype(int).tolist()
            progs.append((toks, [0.5, -1.25, 2.0]))
        else:
            k = length() - 1
            progs.append(([wl.tok(wl.VAR, 0)] + [wl.tok(int(rng.choice([wl.SIN, wl.SQRT, wl.EXP])))] * k, []))
    return wl.pack_programs(progs)


def _bits(t):
    return t.cpu().numpy().view(np.uint64 if t.dtype == torch.float64 else np.uint32)


@pytest.mark.parametrize("kind", ["mse", "corr"])
def test_decoders_agree_on_fitness_and_status(kind):
    api = _api()
    cw, ct = _contexts()
    ps = _mixed_population(31, 3000, 4)
    data = wl.make_dataset(32, 2000, 4, x_range=(-2.0, 5.0), target_len=8)
    X, y = torch.from_numpy(data.X).cuda(), torch.from_numpy(data.y).cuda()
    P = api.DevicePrograms.from_programset(ps)
    fw, sw = api.evaluate(P, X, y, kind, with_status=True, ctx=cw)
    ft, st = api.evaluate(P, X, y, kind, with_status=True, ctx=ct)
    sw, st = sw.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(sw, st)
    # every status a program of this population can have occurs
    assert set(np.unique(sw).tolist()) >= {0, 1, 2, 3, 4, 5, 6}, np.unique(sw)
    assert np.array_equal(_bits(fw), _bits(ft))
    assert np.isfinite(fw.cpu().numpy()).sum() > 1000


def test_decoders_agree_on_outputs():
    api = _api()
    cw, ct = _contexts()
    ps = _mixed_population(33, 600, 3)
    data = wl.make_dataset(34, 700, 3, x_range=(-3.0, 3.0), target_len=8)
    X = torch.from_numpy(data.X).cuda()
    P = api.DevicePrograms.from_programset(ps)
    ow, sw = api.predict(P, X, with_status=True, ctx=cw)
    ot, st = api.predict(P, X, with_status=True, ctx=ct)
    assert np.array_equal(sw.cpu().numpy(), st.cpu().numpy())
    assert np.array_equal(_bits(ow), _bits(ot))


@pytest.mark.parametrize("kind", ["mse", "corr"])
def test_decoders_agree_on_gradients(kind):
    """Programs with 1..8 constants (every adjoint list: value tapes and
    the three derivative-tape sizes) and a share with more than eight
    constant slots or deeper stacks."""
    api = _api()
    cw, ct = _contexts()
    a = wl.random_population(35, 1500, 4, 64, 4, consts_per_program=(1, 8))
    b = wl.random_population(36, 200, 20, 64, 4, consts_per_program=(9, 14))
    c = _mixed_population(37, 300, 4)
    progs = [a.program(i) for i in range(a.n)] + [b.program(i) for i in range(b.n)] + \
            [c.program(i) for i in range(c.n)]
    ps = wl.pack_programs(progs)
    data = wl.make_dataset(38, 3000, 4, x_range=(1.0, 4.0), target_len=8)
    X, y = torch.from_numpy(data.X).cuda(), torch.from_numpy(data.y).cuda()
    P = api.DevicePrograms.from_programset(ps)
    fw, gw, sw = api.evaluate_grad(P, X, y, kind, with_status=True, ctx=cw)
    ft, gt, st = api.evaluate_grad(P, X, y, kind, with_status=True, ctx=ct)
    assert np.array_equal(sw.cpu().numpy(), st.cpu().numpy())
    assert np.array_equal(_bits(fw), _bits(ft))
    assert np.array_equal(_bits(gw), _bits(gt))
    assert np.count_nonzero(gw.cpu().numpy()) > 5000


@pytest.mark.parametrize("log2n", [16, 18])
def test_decoders_agree_on_a_large_population(log2n):
    """2^16 and 2^18 programs of the benchmark's shape on 512 cases: many
    waves and workgroups, 16 and 32 programs per wave of the wave decoder,
    the list appends of every wave."""
    api = _api()
    cw, ct = _contexts()
    ps = wl.random_population(39, 1 << log2n, 5, 64, 5)
    data = wl.make_dataset(40, 512, 5, x_range=(1.0, 10.0), target_len=20)
    X, y = torch.from_numpy(data.X).cuda(), torch.from_numpy(data.y).cuda()
    P = api.DevicePrograms.from_programset(ps)
    for kind in ("mse", "corr"):
        fw, sw = api.evaluate(P, X, y, kind, with_status=True, ctx=cw)
        ft, st = api.evaluate(P, X, y, kind, with_status=True, ctx=ct)
        assert np.all(sw.cpu().numpy() == 0) and np.all(st.cpu().numpy() == 0)
        assert np.array_equal(_bits(fw), _bits(ft))


@pytest.mark.parametrize("lmax", [16, 32, 0])
def test_decoders_agree_on_short_programs(lmax):
    """36864 programs (nine per wave of the wave decoder) of at most 16 or
    32 tokens, or of mixed lengths: programs decoded four or two to a wave
    give the statuses, fitness and outputs of the thread decoder; also when
    some programs share a lower-indexed program's tokens (BAD_LAYOUT for
    the later ones, the ownership test inside a segment)."""
    api = _api()
    cw, ct = _contexts()
    ps = _short_population(41 + lmax, 36864, 4, lmax)
    data = wl.make_dataset(42, 300, 4, x_range=(-2.0, 5.0), target_len=8)
    X, y = torch.from_numpy(data.X).cuda(), torch.from_numpy(data.y).cuda()
    off = ps.tok_offset.astype(np.int64).copy()
    lens = ps.tok_len.astype(np.int32).copy()
    shared = np.arange(97, ps.n, 97)
    off[shared], lens[shared] = off[shared - 1], lens[shared - 1]
    layouts = [api.DevicePrograms.from_programset(ps),
               api.DevicePrograms.from_arrays(ps.tokens, off, lens, ps.consts, ps.const_offset, ps.const_count)]
    for P in layouts:
        for kind in ("mse", "corr"):
            fw, sw = api.evaluate(P, X, y, kind, with_status=True, ctx=cw)
            ft, st = api.evaluate(P, X, y, kind, with_status=True, ctx=ct)
            sw, st = sw.cpu().numpy(), st.cpu().numpy()
            assert np.array_equal(sw, st)
            assert np.array_equal(_bits(fw), _bits(ft))
            assert (sw == 0).sum() > ps.n // 2
        ow, sw = api.predict(P, X[:64], with_status=True, ctx=cw)
        ot, st = api.predict(P, X[:64], with_status=True, ctx=ct)
        assert np.array_equal(sw.cpu().numpy(), st.cpu().numpy())
        assert np.array_equal(_bits(ow), _bits(ot))
    assert set(np.unique(sw.cpu().numpy()).tolist()) >= {0, 1, 2, 3, 4, 5, 6, 8}
