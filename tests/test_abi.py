"""CPU checks of the C-ABI library: it loads, exports every function declared
in include/*.h, rejects bad arguments on the host before any device work,
and its host quantizer agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1101_3228_amd as qt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(qt.LIB_PATH):
        from paper_1101_3228_amd import build
        build.build()
    return qt.lib()


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
            names.update(re.findall(r"\b(qtree_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 15
    assert "qtree_mlp_train_step" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    for s in range(6):
        assert L.qtree_status_string(s)
    assert b"gfx950" in L.qtree_version()


def test_workspace_size_validation(L):
    N = np.array([1, 10, 10], np.int32)
    assert qt.workspace_size(1, 2, N) > 0
    assert qt.workspace_size(2, 2, N) > qt.workspace_size(1, 2, N) // 2
    # the counting scratch grows with the samples held per pass
    assert qt.workspace_size(1, 2, N, 10_000_000) > qt.workspace_size(1, 2, N, 100_000)
    for d, n, NN, code in ((0, 2, N, 1), (4, 2, N, 1), (1, 0, N, 1),
                           (1, 2, np.array([2, 10, 10], np.int32), 1),
                           (1, 2, np.array([1, 0, 10], np.int32), 1),
                           (1, 2, np.array([1, 20000, 10], np.int32), 5),
                           (2, 2, np.array([1, 5000, 10], np.int32), 5)):
        with pytest.raises(qt.QtreeError) as e:
            qt.workspace_size(d, n, NN)
        assert e.value.status == code


def _cmodel(d, n, arrays):
    return qt._Model(d, n, *(arrays[k].ctypes.data for k in ("A", "b", "T", "mu", "L", "x0")))


def test_plan_create_rejects_bad_inputs_before_device_work(L):
    import synth
    spec = synth.bm_model(1, 2)
    arrays = {k: np.ascontiguousarray(spec[k], np.float32) for k in ("A", "b", "T", "mu", "L",
                                                                     "x0")}
    grid, N = synth.layer_grids(spec, [1, 6, 7])
    fake_ws = ctypes.c_void_p(4096)   # never dereferenced on the error paths
    size = qt.workspace_size(1, 2, N)
    h = ctypes.c_void_p()

    def create(g, NN=N, ws=fake_ws, nbytes=size, model=None):
        m = model if model is not None else _cmodel(1, 2, arrays)
        return L.qtree_plan_create(ctypes.byref(m), g.ctypes.data, NN.ctypes.data, ws, nbytes,
                                   ctypes.byref(h))

    bad = grid.copy()
    bad[3] = np.nan
    assert create(bad) == 1
    unsorted = grid.copy()
    unsorted[2], unsorted[3] = grid[3], grid[2]
    assert create(unsorted) == 1 and b"increasing" in L.qtree_last_error()
    assert create(grid, nbytes=100) == 2                        # below the layer tables
    assert create(grid, ws=ctypes.c_void_p(4100)) == 1          # misaligned
    assert create(grid, ws=ctypes.c_void_p(0)) == 1
    a2 = dict(arrays)
    a2["T"] = arrays["T"].copy()
    a2["T"][0] = np.inf
    assert create(grid, model=_cmodel(1, 2, a2)) == 1
    assert L.qtree_transitions(None, 0, 10, 1, 0, 0, ctypes.c_void_p(4096), None) == 1
    assert L.qtree_bdp(None, None, None, 1, None, None, None) == 1
    assert L.qtree_plan_cell_search(None, None, None) == 1


def test_library_quantizer_matches_oracle_quantizer(L):
    from oracle.quantizer import gauss_quantizer, lloyd_step
    for N in (1, 2, 3, 10, 50, 100):
        lib_x = qt.gauss_quantizer(N)
        ref = gauss_quantizer(N)
        # the oracle's Lloyd map stops at a step of 1e-13 and contracts by
        # about 1 - c/N^2 per sweep, so it sits within ~N^2 1e-13 of the fixed point
        assert np.max(np.abs(lib_x - ref)) < 1e-13 * max(N, 10) ** 2, N
        assert np.max(np.abs(lloyd_step(lib_x) - lib_x)) < 1e-12
    x = qt.gauss_quantizer(2)
    assert abs(x[1] - np.sqrt(2 / np.pi)) < 1e-14


def test_library_quantizer_large_n_is_stationary(L):
    from oracle.quantizer import distortion, lloyd_step
    for N in (500, 2000):
        x = qt.gauss_quantizer(N)
        assert np.all(np.diff(x) > 0)
        assert np.max(np.abs(lloyd_step(x) - x)) < 1e-11
        # Bucklew-Wise: N^2 D_N -> sqrt(3) pi / 2 from below
        assert 0.99 * np.sqrt(3) * np.pi / 2 < N * N * distortion(x) < np.sqrt(3) * np.pi / 2


def test_mlp_validation_before_device_work(L):
    from paper_1101_3228_amd import surrogate as S
    S._setup()
    nb = ctypes.c_size_t()
    assert L.qtree_mlp_workspace_size(0, ctypes.byref(nb)) == 0
    inference = nb.value
    assert L.qtree_mlp_workspace_size(4096, ctypes.byref(nb)) == 0
    assert nb.value > inference + 256 * 4096 * 4 * 6          # the training activations
    assert L.qtree_mlp_workspace_size(-1, ctypes.byref(nb)) == 1
    assert L.qtree_mlp_workspace_size((1 << 24) + 1, ctypes.byref(nb)) == 1
    p = np.zeros(S.N_PARAMS, np.float32)
    lo = np.zeros(6, np.float32)
    hi = np.ones(6, np.float32)
    h = ctypes.c_void_p()
    fake = 1 << 20                                           # never dereferenced
    args = dict(p=p.ctypes.data, lo=lo.ctypes.data, hi=hi.ctypes.data, s=0.1, terms=2,
                base=0, mb=0, ws=fake, nb=inference)

    def create(**kw):
        a = dict(args, **kw)
        return L.qtree_mlp_create(a["p"], a["lo"], a["hi"], a["s"], a["terms"], a["base"],
                                  a["mb"], a["ws"], a["nb"], ctypes.byref(h))
    assert create(terms=3) == 1
    assert create(base=2) == 1
    assert create(base=1) == 1                               # sigma_min = 0 in this box
    assert create(s=0.0) == 1
    assert create(mb=-5) == 1
    assert create(ws=fake + 4) == 1                          # misaligned
    assert create(p=None) == 1
    bad = hi.copy()
    bad[2] = -1.0                                            # lo > hi
    assert create(hi=bad.ctypes.data) == 1
    assert create(nb=inference - 1) == 2                     # ENOMEM
    assert b"workspace" in L.qtree_last_error()
    assert L.qtree_mlp_forward(None, None, 4, None, None, None) == 1


def test_swing_and_forward_validation_before_device_work(L):
    qt.lib()
    assert L.qtree_swing(None, None, None, 0, 1, None, None, None) == 1
    sig = np.array([0.2], np.float64)
    assert L.qtree_payoff_forward(None, ctypes.c_double(1.0), ctypes.c_double(1.0),
                                  ctypes.c_double(0.0), ctypes.c_double(1.0), sig.ctypes.data,
                                  None, None, None) == 1


def test_pi_quarter_disc_validation_before_device_work(L):
    qt.lib()
    buf = ctypes.c_uint64(0)
    ptr = ctypes.addressof(buf)
    assert L.qtree_pi_quarter_disc(1, 0, 1, 2, None, None) == 1          # inside NULL
    for reps, npts in ((0, 2), (65536, 2), (1, 0), (1, 3), (1, (1 << 33) + 2)):
        assert L.qtree_pi_quarter_disc(1, 0, reps, npts, ptr, None) == 1, (reps, npts)
    assert buf.value == 0


def test_lloyd_validation_before_device_work(L):
    qt.lib()
    P = ctypes.c_void_p

    def call(d, N, Lm, g0, M=1000, steps=2, ws_bytes=1 << 20, ws=1):
        Lm = np.ascontiguousarray(np.asarray(Lm, np.float32))
        g0 = np.ascontiguousarray(np.asarray(g0, np.float32))
        return L.qtree_lloyd(d, N, Lm.ctypes.data, g0.ctypes.data, P(1), M, steps, 5, 1, None,
                             P(ws), ws_bytes, None)

    eye2 = np.eye(2)
    g2 = np.zeros((4, 2))
    assert call(0, 4, eye2, g2) == 1                          # d
    assert call(4, 4, np.eye(4), np.zeros((4, 4))) == 1
    assert call(2, 0, eye2, g2) == 1                          # N
    assert call(2, 2049, eye2, np.zeros((2049, 2))) == 5      # above the limit
    assert call(2, 4, eye2, g2, M=0) == 3                     # M
    assert call(2, 4, eye2, g2, M=1 << 31) == 3
    assert call(2, 4, eye2, g2, steps=0) == 1
    assert call(2, 4, 20 * eye2, g2) == 3                     # |X| could exceed 64
    bad = g2.copy()
    bad[1, 1] = np.nan
    assert call(2, 4, eye2, bad) == 1
    assert call(2, 4, eye2, g2 + 100.0) == 3
    assert call(1, 3, [[1.0]], [0.0, 0.0, 1.0]) == 1          # 1-D not increasing
    need = L.qtree_lloyd_workspace_size(2, 4)
    assert need > 0 and L.qtree_lloyd_workspace_size(2, 0) == 0
    assert call(2, 4, eye2, g2, ws_bytes=need - 1) == 2       # workspace
    assert L.qtree_lloyd(2, 4, None, None, None, 10, 1, 0, 1, None, None, 0, None) == 1


def test_stratified_validation_before_device_work(L):
    qt.lib()
    assert L.qtree_transitions_stratified(None, 100, 1, 1, 0, None, None, 0, None) == 1
    assert L.qtree_strat_workspace_size(None, 100, 1) == 0
    assert L.qtree_strat_samples(None, 0, 0, 100, 1, 0, 10, 1, 0, None, None, None) == 1
    assert L.qtree_strat_row(None, 0, 0, 100, 1) == -1
