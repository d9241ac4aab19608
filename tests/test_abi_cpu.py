"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments before touching the HIP runtime."""
import ctypes as C

import numpy as np
import pytest

from paper_2009_12850_amd import _lib as M

FAKE = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation


def test_library_exports_every_header_symbol():
    L = M.lib()
    syms = M.header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s


def test_binding_covers_header():
    for s in M.header_symbols():
        assert s in M._SIGS, s


def _prof3():
    return FAKE, FAKE, FAKE


@pytest.mark.parametrize("nx,ny,nz", [(0, 4, 4), (4, 0, 4), (4, 4, 1), (4, 4, 129)])
def test_advect_pw_rejects_bad_grid(nx, ny, nz):
    L = M.lib()
    rc = L.monc_advect_pw(FAKE, FAKE, FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000),
                          C.c_void_p(0x4000), nx, ny, nz, 50.0, 50.0, *_prof3(), None)
    assert rc == M.MONC_EINVAL
    assert L.monc_last_error()


def test_grid_whose_plane_exceeds_32bit_offsets_is_rejected():
    """One x-plane of a field is addressed with 32-bit byte offsets, so a grid
    with (ny+4)*nz*8 bytes per plane past 2 GiB must be refused up front."""
    L = M.lib()
    ny = (1 << 31) // (8 * 128)  # (ny+4)*128*8 just above 2^31
    rc = L.monc_advect_pw(FAKE, FAKE, FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000),
                          C.c_void_p(0x4000), 4, ny, 128, 50.0, 50.0, *_prof3(), None)
    assert rc == M.MONC_EINVAL and b"2 GiB" in L.monc_last_error()
    ok_ny = (1 << 31) // (8 * 128) - 5  # just below
    rc = L.monc_advect_pw(FAKE, FAKE, FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000),
                          C.c_void_p(0x4000), 4, ok_ny, 128, -1.0, 50.0, *_prof3(), None)
    assert rc == M.MONC_EINVAL and b"dx, dy" in L.monc_last_error()


@pytest.mark.parametrize("dx,dy", [(0.0, 1.0), (1.0, -1.0), (float("nan"), 1.0),
                                   (float("inf"), 1.0)])
def test_advect_pw_rejects_bad_spacing(dx, dy):
    L = M.lib()
    rc = L.monc_advect_pw(FAKE, FAKE, FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000),
                          C.c_void_p(0x4000), 4, 4, 4, dx, dy, *_prof3(), None)
    assert rc == M.MONC_EINVAL


def test_advect_pw_rejects_null_and_alias():
    L = M.lib()
    rc = L.monc_advect_pw(None, FAKE, FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000),
                          C.c_void_p(0x4000), 4, 4, 4, 1.0, 1.0, *_prof3(), None)
    assert rc == M.MONC_EINVAL
    rc = L.monc_advect_pw(FAKE, C.c_void_p(0x5000), C.c_void_p(0x6000), FAKE,
                          C.c_void_p(0x3000), C.c_void_p(0x4000), 4, 4, 4, 1.0, 1.0,
                          *_prof3(), None)
    assert rc == M.MONC_EINVAL and b"alias" in L.monc_last_error()
    rc = L.monc_advect_pw(FAKE, FAKE, FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000),
                          C.c_void_p(0x4000), 4, 4, 4, 1.0, 1.0, None, FAKE, FAKE, None)
    assert rc == M.MONC_EINVAL


def _arr(ptrs):
    a = (C.c_void_p * len(ptrs))()
    for n, p in enumerate(ptrs):
        a[n] = p
    return a


def test_step_rejects_bad_arguments():
    L = M.lib()
    ins = _arr([0x1000 + 0x100 * n for n in range(5)])
    outs = _arr([0x9000 + 0x100 * n for n in range(5)])
    ok = dict(nscal=2, nx=8, ny=8, nz=8, dx=1.0, dy=1.0, dt=0.5)

    def call(**kw):
        a = dict(ok, **kw)
        return L.monc_step(kw.get("ins", ins), kw.get("outs", outs), a["nscal"], a["nx"],
                           a["ny"], a["nz"], a["dx"], a["dy"], *_prof3(), a["dt"],
                           kw.get("budgets", None), kw.get("ws", None), None)

    assert call(dt=0.0) == M.MONC_EINVAL
    assert call(dt=float("nan")) == M.MONC_EINVAL
    assert call(nscal=9) == M.MONC_EINVAL
    assert call(nscal=-1) == M.MONC_EINVAL
    assert call(outs=_arr([0x1000, 0x9100, 0x9200, 0x9300, 0x9400])) == M.MONC_EINVAL
    assert call(ins=_arr([0x1000, 0, 0x1200, 0x1300, 0x1400])) == M.MONC_EINVAL
    assert call(budgets=FAKE, ws=None) == M.MONC_EINVAL
    assert call(nz=129) == M.MONC_EINVAL


def test_advect_rejects_unknown_dtype_and_tvd_needs_scalars():
    L = M.lib()
    ins = _arr([0x1000 + 0x100 * n for n in range(5)])
    outs = _arr([0x9000 + 0x100 * n for n in range(5)])
    rc = L.monc_advect(7, ins, outs, 2, None, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5, None)
    assert rc == M.MONC_EINVAL
    q = _arr([0x1300])
    sq = _arr([0x9300])
    rc = L.monc_advect_tvd(FAKE, C.c_void_p(0x1100), C.c_void_p(0x1200), 0, q, sq, 8, 8,
                           8, 1.0, 1.0, *_prof3(), 0.5, None)
    assert rc == M.MONC_EINVAL
    rc = L.monc_cast_working(M.MONC_F64, 1, q, sq, None, 8, 8, 8, None)
    assert rc == M.MONC_EINVAL
    # the streaming cast needs 16-byte aligned buffers
    rc = L.monc_cast_working(M.MONC_F32, 1, _arr([0x1308]), sq, None, 8, 8, 8, None)
    assert rc == M.MONC_EINVAL and b"aligned" in L.monc_last_error()


def test_narrow_separate_entry_points_validate():
    L = M.lib()
    prof = _prof3()
    assert L.monc_advect_pw_f32(FAKE, FAKE, None, FAKE, FAKE, FAKE, 8, 8, 8, 50.0, 50.0, *prof,
                                None) == M.MONC_EINVAL
    assert L.monc_advect_pw_bf16(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 8, 8, 1, 50.0, 50.0,
                                 *prof, None) == M.MONC_EINVAL
    assert L.monc_advect_tvd_f32(FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000), 0,
                                 _block(1, 0x10000), _block(1, 0x20000), None, 8, 8, 8, 50.0,
                                 50.0, *prof, 0.5, None) == M.MONC_EINVAL
    assert b"nscal" in L.monc_last_error()
    assert L.monc_advect_tvd_bf16(FAKE, C.c_void_p(0x2000), C.c_void_p(0x3000), 1,
                                  _block(1, 0x10000), _block(1, 0x20000), None, 8, 8, 8, 50.0,
                                  50.0, *prof, -1.0, None) == M.MONC_EINVAL


def test_budgets_check_maps_device_flags():
    b = np.zeros(M.MONC_NBUDGET)
    b[M.B_COURANT] = 0.3
    assert M.monc_budgets_check(b) == M.MONC_OK
    b[M.B_COURANT] = 1.5
    assert M.monc_budgets_check(b) == M.MONC_ECFL
    b[M.B_COURANT] = float("nan")
    assert M.monc_budgets_check(b) == M.MONC_ECFL
    b[M.B_COURANT] = 0.3
    b[M.B_NONFINITE] = 2
    assert M.monc_budgets_check(b) == M.MONC_ENONFINITE


def test_strerror_and_workspace():
    L = M.lib()
    assert L.monc_strerror(M.MONC_ECFL) == b"Courant number above 1"
    assert L.monc_strerror(12345) == b"unknown error"
    assert M.monc_step_workspace_bytes(1024, 1024, 128, 2) > 0
    assert M.monc_step_workspace_bytes(0, 4, 4, 2) == 0


def test_ensemble_create_validates_members():
    L = M.lib()
    arr = (M.MoncMember * 1)()
    m = arr[0]
    m.nx, m.ny, m.nz = 8, 8, 8
    m.dx = m.dy = 50.0
    m.dt = 0.5
    m.rdz = m.rho = m.rhon = 0x1000
    for p in range(2):
        for f in range(5):
            m.state[p][f] = 0x2000 + 0x100 * (5 * p + f)
    plan = C.c_void_p()
    m.dt = 0.0
    assert L.monc_ensemble_create(C.cast(arr, C.c_void_p), 1, 2, None, 0,
                                  C.byref(plan)) == M.MONC_EINVAL
    m.dt = 0.5
    m.state[1][3] = 0
    assert L.monc_ensemble_create(C.cast(arr, C.c_void_p), 1, 2, None, 0,
                                  C.byref(plan)) == M.MONC_EINVAL
    m.state[1][3] = 0x2000
    assert L.monc_ensemble_create(C.cast(arr, C.c_void_p), 1, 2, None, 0,
                                  C.byref(plan)) == M.MONC_EINVAL  # aliases state[0][0]
    assert L.monc_ensemble_create(C.cast(arr, C.c_void_p), 0, 2, None, 0,
                                  C.byref(plan)) == M.MONC_EINVAL
    assert L.monc_ensemble_create(C.cast(arr, C.c_void_p), 1, 4, None, 0,
                                  C.byref(plan)) == M.MONC_EUNSUPPORTED
    assert L.monc_ensemble_run(None, 5, None) == M.MONC_EINVAL
    assert L.monc_ensemble_set_budgets(None, C.c_void_p(0x7000), 3) == M.MONC_EINVAL


@pytest.mark.parametrize("dtype,work", [(M.MONC_F64, 0), (M.MONC_F64, M.MONC_MAX_WORK + 1),
                                        (M.MONC_BF16, 1), (7, 1)])
def test_pw_scaled_rejects_bad_work_and_dtype(dtype, work):
    L = M.lib()
    rc = L.monc_advect_pw_scaled(dtype, FAKE, C.c_void_p(0x5000), C.c_void_p(0x6000),
                                 C.c_void_p(0x2000), C.c_void_p(0x3000), C.c_void_p(0x4000),
                                 4, 4, 4, 50.0, 50.0, *_prof3(), work, None)
    assert rc == M.MONC_EINVAL and L.monc_last_error()


def _block(n, base):
    return _arr([base + 0x100 * q for q in range(n)])


def test_learned_entry_points_validate_before_launch():
    L = M.lib()
    d = C.c_double
    prof = _prof3()
    # restriction needs multiples of 4
    rc = L.monc_restrict4(1, _block(4, 0x10000), _block(4, 0x20000), 6, 8, 8, *prof, FAKE, FAKE,
                          FAKE, None)
    assert rc == M.MONC_EINVAL and b"multiples of 4" in L.monc_last_error()
    # features: orient, zero std, missing cell list with the wrong count
    norm = (d * 8)(0, 1, 0, 1, 0, 1, 0, 1)
    bad = (d * 8)(0, 1, 0, 0, 0, 1, 0, 1)
    assert L.monc_mlp_features(_block(4, 0x10000), 4, 4, 4, norm, 2, None, 64, FAKE,
                               None) == M.MONC_EINVAL
    assert L.monc_mlp_features(_block(4, 0x10000), 4, 4, 4, bad, 0, None, 64, FAKE,
                               None) == M.MONC_EINVAL
    assert L.monc_mlp_features(_block(4, 0x10000), 4, 4, 4, norm, 0, None, 63, FAKE,
                               None) == M.MONC_EINVAL
    # forward: empty batch, misaligned rows
    assert L.monc_mlp_forward(FAKE, 0, FAKE, FAKE, FAKE, None, None, None, None,
                              None) == M.MONC_EINVAL
    assert L.monc_mlp_forward(C.c_void_p(0x1008), 4, FAKE, FAKE, FAKE, None, None, None, None,
                              None) == M.MONC_EINVAL
    # Adam: t < 1 and a bad beta
    assert L.monc_mlp_adam(FAKE, FAKE, FAKE, FAKE, 0, 1e-3, 0.9, 0.999, 1e-8, FAKE,
                           None) == M.MONC_EINVAL
    assert L.monc_mlp_adam(FAKE, FAKE, FAKE, FAKE, 1, 1e-3, 1.0, 0.999, 1e-8, FAKE,
                           None) == M.MONC_EINVAL
    # corrected step: growth must be positive, scales finite, state not aliased
    scale = (d * 4)(1, 1, 1, 1)
    nanscale = (d * 4)(1, float("nan"), 1, 1)
    args = (_block(4, 0x10000), _block(4, 0x20000), FAKE, FAKE, _block(4, 0x30000), 4, 4, 4, 50.0,
            50.0)
    assert L.monc_correct_step(*args, scale, *prof, 2.0, 0.0, FAKE, FAKE,
                               None) == M.MONC_EINVAL
    assert L.monc_correct_step(*args, nanscale, *prof, 2.0, 1.01, FAKE, FAKE,
                               None) == M.MONC_EINVAL
    alias = (_block(4, 0x10000), _block(4, 0x20000), FAKE, FAKE, _block(4, 0x10000), 4, 4, 4, 50.0,
             50.0)
    assert L.monc_correct_step(*alias, scale, *prof, 2.0, 1.01, FAKE, FAKE,
                               None) == M.MONC_EINVAL
    misaligned = (_block(4, 0x10000), _block(4, 0x20000), C.c_void_p(0x1004), FAKE,
                  _block(4, 0x30000), 4, 4, 4, 50.0, 50.0)
    assert L.monc_correct_step(*misaligned, scale, *prof, 2.0, 1.01, FAKE, FAKE,
                               None) == M.MONC_EINVAL
    assert b"16-byte" in L.monc_last_error()
    assert M.monc_correct_step_workspace_bytes(8, 8, 8) > 0
    assert M.monc_mlp_backward_workspace_bytes(0) == 0
    # fused training step: empty batch, t < 1, bad beta, zero scale, zero
    # std, misaligned pack
    fields3 = (_block(4, 0x10000), _block(4, 0x20000), _block(4, 0x30000), 4, 4, 4)

    def train(nrm, b, scl, t, b1, wpack=FAKE):
        return L.monc_mlp_train_step(*fields3, nrm, FAKE, b, 2.0, scl, FAKE, FAKE, 0.01, FAKE,
                                     FAKE, FAKE, t, 1e-3, b1, 0.999, 1e-8, wpack, FAKE, FAKE,
                                     FAKE, None)

    zscale = (d * 4)(1, 1, 0, 1)
    assert train(norm, 0, scale, 1, 0.9) == M.MONC_EINVAL
    assert train(norm, 8, scale, 0, 0.9) == M.MONC_EINVAL
    assert train(norm, 8, scale, 1, 1.0) == M.MONC_EINVAL
    assert train(norm, 8, zscale, 1, 0.9) == M.MONC_EINVAL
    assert train(bad, 8, scale, 1, 0.9) == M.MONC_EINVAL
    assert train(norm, 8, scale, 1, 0.9, C.c_void_p(0x1008)) == M.MONC_EINVAL
    assert b"16-byte" in L.monc_last_error()
    assert M.monc_mlp_train_workspace_bytes(0) == 0
    assert M.monc_mlp_train_workspace_bytes(16) < M.monc_mlp_train_workspace_bytes(32)
    assert M.monc_mlp_train_workspace_bytes(100000) == M.monc_mlp_train_workspace_bytes(8192)


def test_dynamics_entries_reject_bad_arguments():
    # every case fails validation before any HIP call
    L = M.lib()
    good = M.DynParams(1e-4, 5.0, 0.0, 9.81, 300.0)
    f = [C.c_void_p(0x1000 + 0x100 * n) for n in range(6)]
    for bad in (M.DynParams(1e-4, 5.0, 0.0, 9.81, 0.0), M.DynParams(float("nan"), 0, 0, 9.81, 300),
                M.DynParams(1e-4, float("inf"), 0, 9.81, 300)):
        assert L.monc_dyn_tend(*f, 8, 8, 8, C.byref(bad), None) == M.MONC_EINVAL
    assert L.monc_dyn_tend(*f, 8, 8, 8, None, None) == M.MONC_EINVAL
    assert L.monc_dyn_tend(f[0], f[1], f[2], f[0], f[4], f[5], 8, 8, 8, C.byref(good),
                           None) == M.MONC_EINVAL  # output aliases an input
    assert L.monc_dyn_tend(*f, 8, 0, 8, C.byref(good), None) == M.MONC_EINVAL
    ins = _arr([0x1000 + 0x100 * n for n in range(4)])
    outs = _arr([0x9000 + 0x100 * n for n in range(4)])
    tend = _arr([0x5000 + 0x100 * n for n in range(4)])
    dyn = _arr([0x7000 + 0x100 * n for n in range(3)])
    call_h = lambda nscal, i=ins, o=outs, t=tend, d=dyn, p=good: L.monc_hybrid_step(
        i, o, t, d, nscal, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5, C.byref(p), None, None)
    assert call_h(0) == M.MONC_EINVAL  # needs theta
    assert call_h(1, t=outs) == M.MONC_EINVAL  # tendencies alias the output state
    assert call_h(1, p=M.DynParams(0, 0, 0, 9.81, -1.0)) == M.MONC_EINVAL
    call_s = lambda nscal, p=good: L.monc_step_dyn(ins, outs, nscal, 8, 8, 8, 1.0, 1.0,
                                                   *_prof3(), 0.5, C.byref(p), None)
    assert call_s(0) == M.MONC_EINVAL
    assert call_s(1, M.DynParams(0, 0, 0, 9.81, 0.0)) == M.MONC_EINVAL
    assert L.monc_combine_step(0, ins, tend, None, outs, 8, 8, 8, 0.5, None) == M.MONC_EINVAL
    assert L.monc_combine_step(4, ins, tend, None, ins, 8, 8, 8, 0.5, None) == M.MONC_EINVAL
    tb = _arr([0x9000, 0, 0, 0])  # tb[0] aliases out[0]
    assert L.monc_combine_step(4, ins, tend, tb, outs, 8, 8, 8, 0.5, None) == M.MONC_EINVAL
    assert L.monc_combine_step(4, ins, tend, None, outs, 8, 8, 8, 0.0, None) == M.MONC_EINVAL


def test_step_pw_scalars_rejects_bad_arguments():
    L = M.lib()
    ins = _arr([0x1000 + 0x100 * n for n in range(5)])
    outs = _arr([0x9000 + 0x100 * n for n in range(5)])
    assert L.monc_step_pw_scalars(ins, outs, 2, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.0,
                                  None) == M.MONC_EINVAL
    assert L.monc_step_pw_scalars(ins, ins, 2, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5,
                                  None) == M.MONC_EINVAL
    assert L.monc_step_pw_scalars(ins, outs, 9, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5,
                                  None) == M.MONC_EINVAL


def test_tvd_momentum_entries_reject_bad_arguments():
    L = M.lib()
    P = [C.c_void_p(0x1000 * (n + 1)) for n in range(7)]  # u v w su sv sw cmax
    ok = (4, 4, 8, 50.0, 50.0, *_prof3(), 1.0)
    assert L.monc_advect_tvd_momentum(*P[:6], *ok[:8], 0.0, P[6], None) == M.MONC_EINVAL
    assert L.monc_advect_tvd_momentum(*P[:6], 4, 4, 1, 50.0, 50.0, *_prof3(), 1.0, P[6],
                                      None) == M.MONC_EINVAL
    assert L.monc_advect_tvd_momentum(P[0], P[1], P[2], P[0], P[4], P[5], *ok, P[6],
                                      None) == M.MONC_EINVAL  # su aliases u
    assert L.monc_advect_tvd_momentum(*P[:6], *ok, P[1], None) == M.MONC_EINVAL  # cmax = v
    assert b"alias" in L.monc_last_error()
    assert L.monc_advect_tvd_momentum(*P[:5], None, *ok, None, None) == M.MONC_EINVAL
    ins = _arr([0x1000 + 0x100 * n for n in range(5)])
    outs = _arr([0x9000 + 0x100 * n for n in range(5)])
    assert L.monc_step_tvd_momentum(ins, outs, 2, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.0, None,
                                    None) == M.MONC_EINVAL
    assert L.monc_step_tvd_momentum(ins, ins, 2, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5, None,
                                    None) == M.MONC_EINVAL
    assert L.monc_step_tvd_momentum(ins, outs, 9, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5, None,
                                    None) == M.MONC_EINVAL
    assert L.monc_step_tvd_momentum(ins, outs, 2, 8, 8, 8, 1.0, 1.0, *_prof3(), 0.5,
                                    C.c_void_p(0x9100), None) == M.MONC_EINVAL  # cmax = out


def test_static_step_rejects_grids_beyond_its_scratch():
    """monc_step_static refuses, before any HIP call, a grid whose launch needs
    more budget rows than its static scratch holds, and a missing budgets
    array."""
    L = M.lib()
    ins = _arr([0x1000 + 0x100 * n for n in range(4)])
    outs = _arr([0x9000 + 0x100 * n for n in range(4)])
    # 8 planes x 36000 columns: 9000 tiles of four columns along y
    rc = L.monc_step_static(ins, outs, 1, 8, 36000, 128, 50.0, 50.0, *_prof3(), 0.5,
                            C.c_void_p(0x7000), None)
    assert rc == M.MONC_EINVAL and b"static scratch" in L.monc_last_error()
    rc = L.monc_step_static(ins, outs, 1, 8, 8, 8, 50.0, 50.0, *_prof3(), 0.5, None, None)
    assert rc == M.MONC_EINVAL and b"budgets" in L.monc_last_error()
