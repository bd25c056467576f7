"""Host-only checks of the C ABI: the library loads, exports every function
include/shoot.h declares, and validates plans (no GPU call is made)."""
import ctypes
import os
import re

import pytest

from paper_2106_08817_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shoot.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(shoot_\w+)\s*\(", src, flags=re.M))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    declared = header_functions()
    assert declared == set(_lib.EXPORTS), declared ^ set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.shoot_version()


FAKE = 0x7F0000000000  # never dereferenced: plan creation is host-only


def pair(ndim=2, shape=(32, 40), rho=0.5, sigma=2.0, lam=0.01, image=FAKE, p0=FAKE + 4096, target=FAKE + 8192):
    p = _lib.ShootPair()
    p.ndim = ndim
    for a in range(3):
        p.shape[a] = shape[a] if a < len(shape) else 0
    p.rho, p.sigma, p.lambda_ = rho, sigma, lam
    p.image, p.p0, p.target = image, p0, target
    p.out_grad = FAKE + 12288
    p.out_cost = FAKE + 16384
    return p


def create(pairs, T=10, flags=0, budget=0):
    lib = _lib.load()
    arr = (_lib.ShootPair * len(pairs))(*pairs)
    h = ctypes.c_void_p(123)
    st = lib.shoot_plan_create(ctypes.cast(arr, ctypes.c_void_p), len(pairs), T, flags, budget, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,T,status", [
    (dict(ndim=4), 10, _lib.SHOOT_E_SHAPE),
    (dict(shape=(1, 40)), 10, _lib.SHOOT_E_SHAPE),
    (dict(sigma=0.0), 10, _lib.SHOOT_E_ARG),
    (dict(sigma=float("nan")), 10, _lib.SHOOT_E_ARG),
    (dict(sigma=11.0), 10, _lib.SHOOT_E_ARG),
    (dict(rho=-0.1), 10, _lib.SHOOT_E_ARG),
    (dict(lam=-1.0), 10, _lib.SHOOT_E_ARG),
    (dict(image=None), 10, _lib.SHOOT_E_ARG),
    (dict(p0=None), 10, _lib.SHOOT_E_ARG),
    (dict(), 0, _lib.SHOOT_E_ARG),
    (dict(ndim=3, shape=(4, 5, 40000)), 10, _lib.SHOOT_E_SHAPE),
])
def test_plan_validation(kw, T, status):
    st, h = create([pair(**kw)], T=T)
    assert st == status
    assert h.value is None
    assert len(_lib.load().shoot_last_error()) > 0


def test_mixed_ndim_and_unknown_flags_rejected():
    st, _ = create([pair(), pair(ndim=3, shape=(8, 8, 8))])
    assert st == _lib.SHOOT_E_SHAPE
    st, _ = create([pair()], flags=1 << 20)
    assert st == _lib.SHOOT_E_ARG


def test_plan_sizes_waves_and_unbound_execution():
    lib = _lib.load()
    st, h = create([pair(shape=(96, 128)), pair(shape=(240, 320), sigma=5.5)], T=20)
    assert st == _lib.SHOOT_OK
    n = ctypes.c_size_t()
    assert lib.shoot_plan_workspace_bytes(h, ctypes.byref(n)) == _lib.SHOOT_OK
    ck = n.value
    w = ctypes.c_int32()
    assert lib.shoot_plan_waves(h, ctypes.byref(w)) == _lib.SHOOT_OK and w.value == 1
    # execution before bind is refused before any device work
    assert lib.shoot_grad_p0(h, None) == _lib.SHOOT_E_STATE
    # bind refuses missing / misaligned / short workspaces before any HIP call
    assert lib.shoot_plan_bind(h, None, n.value, None) == _lib.SHOOT_E_WORKSPACE
    assert lib.shoot_plan_bind(h, FAKE + 4, n.value, None) == _lib.SHOOT_E_WORKSPACE
    assert lib.shoot_plan_bind(h, FAKE, n.value - 1, None) == _lib.SHOOT_E_WORKSPACE
    assert lib.shoot_plan_destroy(h) == _lib.SHOOT_OK
    # full store keeps all T states: more memory than sqrt(T) checkpoints
    st, h = create([pair(shape=(96, 128)), pair(shape=(240, 320), sigma=5.5)], T=20, flags=_lib.SHOOT_FULL_STORE)
    assert lib.shoot_plan_workspace_bytes(h, ctypes.byref(n)) == _lib.SHOOT_OK
    assert n.value > ck
    lib.shoot_plan_destroy(h)
    assert lib.shoot_plan_destroy(None) == _lib.SHOOT_OK


def test_budget_splits_into_waves():
    lib = _lib.load()
    pairs = [pair(shape=(128, 128)) for _ in range(6)]
    st, h = create(pairs, T=9)
    n1 = ctypes.c_size_t()
    lib.shoot_plan_workspace_bytes(h, ctypes.byref(n1))
    lib.shoot_plan_destroy(h)
    st, h = create(pairs, T=9, budget=n1.value // 2)
    assert st == _lib.SHOOT_OK
    w = ctypes.c_int32()
    lib.shoot_plan_waves(h, ctypes.byref(w))
    assert w.value >= 2
    n2 = ctypes.c_size_t()
    lib.shoot_plan_workspace_bytes(h, ctypes.byref(n2))
    assert n2.value < n1.value
    assert n2.value <= n1.value // 2  # the budget caps the whole workspace, headers included
    lib.shoot_plan_destroy(h)
    st, h = create(pairs, T=9, budget=1024)
    assert st == _lib.SHOOT_E_BUDGET


@pytest.mark.parametrize("npairs,shape,T", [(64, (32, 32), 40), (6, (128, 128), 9), (9, (40, 52), 20)])
def test_budget_caps_the_whole_workspace(npairs, shape, T):
    """Every budget between one pair's need and the whole batch's: the
    workspace (headers of every wave plus the largest field region) never
    exceeds it, down to the last byte."""
    lib = _lib.load()
    pairs = [pair(shape=shape) for _ in range(npairs)]
    st, h = create(pairs, T=T)
    full = ctypes.c_size_t()
    lib.shoot_plan_workspace_bytes(h, ctypes.byref(full))
    lib.shoot_plan_destroy(h)
    n = ctypes.c_size_t()
    for budget in (full.value - 1, full.value * 3 // 4, full.value // 2, full.value // 5, full.value // 9):
        st, h = create(pairs, T=T, budget=budget)
        if st == _lib.SHOOT_E_BUDGET:
            continue
        assert st == _lib.SHOOT_OK
        lib.shoot_plan_workspace_bytes(h, ctypes.byref(n))
        assert n.value <= budget, (budget, n.value)
        lib.shoot_plan_destroy(h)


def test_displacements_and_stream_copy_validate_on_the_host():
    lib = _lib.load()
    st, h = create([pair()], T=4)
    out = (ctypes.c_float * 4)()
    assert lib.shoot_plan_displacements(h, out, None) == _lib.SHOOT_E_STATE  # not bound
    assert lib.shoot_plan_displacements(h, None, None) == _lib.SHOOT_E_ARG
    lib.shoot_plan_destroy(h)
    st, h = create([pair()], T=4, flags=_lib.SHOOT_UNFUSED)
    assert lib.shoot_plan_displacements(h, out, None) == _lib.SHOOT_E_ARG
    lib.shoot_plan_destroy(h)
    assert lib.shoot_stream_copy(None, FAKE, 64, None) == _lib.SHOOT_E_ARG
    assert lib.shoot_stream_copy(FAKE, FAKE + 4096, 60, None) == _lib.SHOOT_E_ARG       # size not a multiple of 16
    assert lib.shoot_stream_copy(FAKE + 4, FAKE + 4096, 64, None) == _lib.SHOOT_E_ARG   # misaligned
    assert lib.shoot_stream_copy(FAKE, FAKE + 32, 64, None) == _lib.SHOOT_E_ARG         # overlapping


def test_lanes_flag_and_count():
    lib = _lib.load()
    n = ctypes.c_int32()
    pairs2 = [pair(shape=(96 + 8 * i, 64)) for i in range(6)]
    # default: 3 lanes in 2-D, at most one per pair; 2 in 3-D
    st, h = create(pairs2)
    assert st == _lib.SHOOT_OK and lib.shoot_plan_lanes(h, ctypes.byref(n)) == _lib.SHOOT_OK and n.value == 3
    lib.shoot_plan_destroy(h)
    st, h = create(pairs2[:2])
    lib.shoot_plan_lanes(h, ctypes.byref(n))
    assert n.value == 2
    lib.shoot_plan_destroy(h)
    st, h = create([pair(ndim=3, shape=(16, 16, 16)) for _ in range(5)])
    lib.shoot_plan_lanes(h, ctypes.byref(n))
    assert n.value == 2
    lib.shoot_plan_destroy(h)
    # a wave of at least 2^23 voxels runs as one lane unless the count is fixed
    big = [pair(ndim=3, shape=(128, 128, 256)) for _ in range(2)]      # 2 x 2^22 voxels
    st, h = create(big, T=4)
    lib.shoot_plan_lanes(h, ctypes.byref(n))
    assert st == _lib.SHOOT_OK and n.value == 1
    lib.shoot_plan_destroy(h)
    st, h = create(big[:1] + [pair(ndim=3, shape=(128, 128, 252))], T=4)   # just below
    lib.shoot_plan_lanes(h, ctypes.byref(n))
    assert st == _lib.SHOOT_OK and n.value == 2
    lib.shoot_plan_destroy(h)
    st, h = create(big, T=4, flags=_lib.SHOOT_LANES(2))
    lib.shoot_plan_lanes(h, ctypes.byref(n))
    assert st == _lib.SHOOT_OK and n.value == 2
    lib.shoot_plan_destroy(h)
    # fixed counts; the workspace hardly depends on them (lane alignment only)
    sizes = {}
    for k in (1, 2, 6):
        st, h = create(pairs2, flags=_lib.SHOOT_LANES(k))
        assert st == _lib.SHOOT_OK
        lib.shoot_plan_lanes(h, ctypes.byref(n))
        assert n.value == k
        b = ctypes.c_size_t()
        lib.shoot_plan_workspace_bytes(h, ctypes.byref(b))
        sizes[k] = b.value
        lib.shoot_plan_destroy(h)
    assert max(sizes.values()) < 1.01 * min(sizes.values())
    st, _ = create(pairs2, flags=_lib.SHOOT_LANES(9))
    assert st == _lib.SHOOT_E_ARG
    # unfused plans run pair by pair: one lane
    st, h = create(pairs2, flags=_lib.SHOOT_UNFUSED)
    lib.shoot_plan_lanes(h, ctypes.byref(n))
    assert n.value == 1
    lib.shoot_plan_destroy(h)
    assert lib.shoot_plan_lanes(None, ctypes.byref(n)) == _lib.SHOOT_E_ARG


def test_budget_counts_the_lanes_of_a_wave():
    """Admission sizes a wave with its lanes: smaller budgets give more waves
    and a smaller workspace."""
    lib = _lib.load()
    pairs = [pair(shape=(64 + 16 * (i % 3), 96)) for i in range(7)]
    st, h = create(pairs, T=9)
    full = ctypes.c_size_t()
    lib.shoot_plan_workspace_bytes(h, ctypes.byref(full))
    lib.shoot_plan_destroy(h)
    for frac in (0.9, 0.6, 0.35):
        budget = int(full.value * frac)
        st, h = create(pairs, T=9, budget=budget)
        assert st == _lib.SHOOT_OK
        b, w = ctypes.c_size_t(), ctypes.c_int32()
        lib.shoot_plan_workspace_bytes(h, ctypes.byref(b))
        lib.shoot_plan_waves(h, ctypes.byref(w))
        assert w.value >= 2 and b.value < full.value
        lib.shoot_plan_destroy(h)


def test_check_finite_flag_host_side():
    lib = _lib.load()
    st, h = create([pair()], flags=_lib.SHOOT_CHECK_FINITE)
    assert st == _lib.SHOOT_OK
    lib.shoot_plan_destroy(h)
    st, _ = create([pair()], flags=_lib.SHOOT_CHECK_FINITE | _lib.SHOOT_UNFUSED)
    assert st == _lib.SHOOT_E_ARG and b"SHOOT_CHECK_FINITE" in lib.shoot_last_error()


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_LIB", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()


def test_tuning_choices_host_side():
    lib = _lib.load()
    st, h = create([pair(shape=(96, 128))], T=6)
    assert st == _lib.SHOOT_OK
    arr = (ctypes.c_int32 * _lib.SHOOT_TUNE_COUNT)()
    assert lib.shoot_plan_get_tuning(h, arr) == _lib.SHOOT_OK
    assert list(arr) == [0] * _lib.SHOOT_TUNE_COUNT            # defaults
    n = _lib.SHOOT_TUNE_COUNT
    want = [1, 0, 1, 1, 0, 1][:n]
    assert lib.shoot_plan_set_tuning(h, (ctypes.c_int32 * n)(*want)) == _lib.SHOOT_OK
    assert lib.shoot_plan_get_tuning(h, arr) == _lib.SHOOT_OK and list(arr) == want
    bad = [0] * n
    bad[1] = 2
    assert lib.shoot_plan_set_tuning(h, (ctypes.c_int32 * n)(*bad)) == _lib.SHOOT_E_ARG
    assert lib.shoot_plan_get_tuning(h, arr) == _lib.SHOOT_OK and list(arr) == want   # unchanged
    assert lib.shoot_plan_set_tuning(h, None) == _lib.SHOOT_E_ARG
    assert lib.shoot_plan_get_tuning(None, arr) == _lib.SHOOT_E_ARG
    # autotune needs a bound workspace
    assert lib.shoot_autotune(h, None) == _lib.SHOOT_E_STATE
    lib.shoot_plan_destroy(h)


def test_pair_selection_host_side():
    lib = _lib.load()
    st, h = create([pair(shape=(40, 36)), pair(shape=(20, 24)), pair(shape=(33, 17))], T=5)
    assert st == _lib.SHOOT_OK
    arr = lambda *v: (ctypes.c_int32 * len(v))(*v)  # noqa: E731
    assert lib.shoot_plan_set_active(h, arr(1, 0, 1), None) == _lib.SHOOT_OK     # unbound: kept for the bind
    assert lib.shoot_plan_set_active(h, arr(1, 2, 1), None) == _lib.SHOOT_E_ARG
    assert lib.shoot_plan_set_active(h, arr(-1, 0, 1), None) == _lib.SHOOT_E_ARG
    assert lib.shoot_plan_set_active(h, None, None) == _lib.SHOOT_OK             # all active
    assert lib.shoot_plan_set_active(None, None, None) == _lib.SHOOT_E_ARG
    lib.shoot_plan_destroy(h)
    st, h = create([pair()], T=5, flags=_lib.SHOOT_UNFUSED)
    assert st == _lib.SHOOT_OK
    assert lib.shoot_plan_set_active(h, arr(1), None) == _lib.SHOOT_E_ARG          # not on the unfused path
    lib.shoot_plan_destroy(h)


def test_tune_class_and_cache_host_side():
    lib = _lib.load()
    # radii floor(3 sigma) = 6 and 9 -> 16; last extents 128 and 100 -> 2^7
    st, h = create([pair(shape=(96, 128), sigma=2.0), pair(shape=(64, 100), sigma=3.0)], T=6)
    assert st == _lib.SHOOT_OK
    buf = ctypes.create_string_buffer(128)
    assert lib.shoot_plan_tune_class(h, buf, len(buf)) == _lib.SHOOT_OK
    cls = buf.value.decode()
    m = re.fullmatch(r"d2-grad-v(\d+)-x7_7-r16-l(\d+)-f0", cls)
    assert m, cls
    # the largest wave holds one pair (lanes) or both: 2^13 <= 12288, 18688 < 2^15
    assert int(m.group(1)) in (13, 14)
    assert lib.shoot_plan_tune_class(h, buf, len(cls)) == _lib.SHOOT_E_ARG                # no room for the NUL
    assert lib.shoot_plan_tune_class(h, buf, len(cls) + 1) == _lib.SHOOT_OK
    hit = ctypes.c_int32(7)
    assert lib.shoot_autotune_cached(h, b"/tmp/x.json", ctypes.byref(hit), None) == _lib.SHOOT_E_STATE
    assert hit.value == 0
    assert lib.shoot_autotune_cached(h, None, None, None) == _lib.SHOOT_E_ARG
    lib.shoot_plan_destroy(h)
    # forward-only plans (no target) are timed on the forward shot; 3-D
    st, h = create([pair(ndim=3, shape=(20, 24, 36), sigma=1.0, target=None)], T=4)
    assert st == _lib.SHOOT_OK
    assert lib.shoot_plan_tune_class(h, buf, len(buf)) == _lib.SHOOT_OK
    assert re.fullmatch(r"d3-fwd-v\d+-x6_6-r4-l\d+-f0", buf.value.decode()), buf.value


def test_descend_requires_bind_and_validates_step():
    lib = _lib.load()
    st, h = create([pair(shape=(40, 52))], T=4)
    assert st == _lib.SHOOT_OK
    assert lib.shoot_descend(h, 0.0, 1, None) == _lib.SHOOT_E_ARG       # eta0 must be > 0
    assert lib.shoot_descend(h, float("nan"), 1, None) == _lib.SHOOT_E_ARG
    assert lib.shoot_descend(h, 1.0, 0, None) == _lib.SHOOT_E_STATE     # no reset yet
    assert lib.shoot_descend(h, 1.0, 1, None) == _lib.SHOOT_E_STATE     # not bound to a workspace
    lib.shoot_plan_destroy(h)
    st, h = create([pair(shape=(40, 52))], T=4, flags=_lib.SHOOT_UNFUSED)
    assert lib.shoot_descend(h, 1.0, 1, None) == _lib.SHOOT_E_ARG
    lib.shoot_plan_destroy(h)


def test_lbfgs_validation_host_side():
    lib = _lib.load()
    st, h = create([pair(shape=(40, 52))], T=4)
    assert st == _lib.SHOOT_OK
    o = ctypes.c_void_p()
    assert lib.shoot_lbfgs_create(h, 0, 1e-4, 8, ctypes.byref(o)) == _lib.SHOOT_E_ARG      # m
    assert lib.shoot_lbfgs_create(h, 5, 1.5, 8, ctypes.byref(o)) == _lib.SHOOT_E_ARG       # c1
    assert lib.shoot_lbfgs_create(h, 5, 1e-4, 0, ctypes.byref(o)) == _lib.SHOOT_E_ARG      # trials
    assert lib.shoot_lbfgs_create(None, 5, 1e-4, 8, ctypes.byref(o)) == _lib.SHOOT_E_ARG
    assert lib.shoot_lbfgs_create(h, 5, 1e-4, 8, ctypes.byref(o)) == _lib.SHOOT_OK
    n = ctypes.c_size_t()
    assert lib.shoot_lbfgs_workspace_bytes(o, ctypes.byref(n)) == _lib.SHOOT_OK and n.value > 0
    assert lib.shoot_lbfgs_step(o, None) == _lib.SHOOT_E_STATE                             # not bound
    assert lib.shoot_lbfgs_bind(o, FAKE + 4, n.value, None) == _lib.SHOOT_E_WORKSPACE
    assert lib.shoot_lbfgs_bind(o, FAKE, n.value - 1, None) == _lib.SHOOT_E_WORKSPACE
    assert lib.shoot_lbfgs_destroy(o) == _lib.SHOOT_OK
    lib.shoot_plan_destroy(h)
    p = pair(shape=(40, 52))
    p.out_grad = None
    st, h = create([p], T=4)
    assert lib.shoot_lbfgs_create(h, 5, 1e-4, 8, ctypes.byref(o)) == _lib.SHOOT_E_ARG      # needs out_grad
    assert b"out_grad" in lib.shoot_last_error()
    lib.shoot_plan_destroy(h)


def test_scheme_flags_validation():
    lib = _lib.load()
    E, M = _lib.SHOOT_SCHEME_EULERIAN, _lib.SHOOT_SCHEME_MIXED
    st, h = create([pair()], flags=E | M)
    assert st == _lib.SHOOT_E_ARG
    st, h = create([pair()], flags=E | _lib.SHOOT_UNFUSED)
    assert st == _lib.SHOOT_E_ARG
    for f in (E, M):
        st, h = create([pair()], flags=f)
        assert st == _lib.SHOOT_OK
        lib.shoot_plan_destroy(h)


def test_unfused_plan_rejects_deformation_output():
    p = pair()
    p.out_deformation = FAKE + 20480
    st, h = create([p], flags=_lib.SHOOT_UNFUSED)
    assert st == _lib.SHOOT_E_ARG
    st, h = create([p])
    assert st == _lib.SHOOT_OK
    _lib.load().shoot_plan_destroy(h)
