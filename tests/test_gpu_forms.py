"""GPU tests of the precision forms, the multi-pass scalar groups, ragged
column heights, and the 100-step run with budgets checked every step.

FP32 tendencies (from FP32 working copies, scalars stored as anomalies from a
constant) must stay within 1e-5 of the FP64 oracle (per field, relative to the
field's largest value); BF16 storage is reported against a looser bound that
follows from its 8-bit mantissa.
"""
import sys

import numpy as np
import pytest

from gpu_util import case, dev, oracle_tendencies, prof_dev, rel_err, to_dev, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL64 = 1e-13
# After n steps the GPU and oracle states may differ by one rounding of the
# new value per step (the GPU adds dt s with a fused multiply-add), carried
# along by the scheme: the bar is this factor times n units in the last place
# of the field's largest value.
STEPS512_GROWTH = 10.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    M.lib()


def narrow_tendencies(host, g, dt, dtype, phi0):
    T = torch()
    d = to_dev(host)
    tdt = T.float32 if dtype == M.MONC_F32 else T.int16
    work = [T.empty(x.shape, dtype=tdt, device=dev()) for x in d]
    offs = [0.0, 0.0, 0.0] + list(phi0)
    M.monc_cast_working(dtype, d, work, offs)
    out = [T.zeros(x.shape, dtype=T.float32, device=dev()) for x in d]
    M.monc_advect(dtype, work, out, g.dx, g.dy, prof_dev(g), dt, phi0=phi0)
    T.cuda.synchronize()
    return [o.double().cpu().numpy() for o in out]


@pytest.mark.parametrize("shape", [(32, 32, 32), (40, 36, 128), (17, 23, 96)])
def test_fp32_tendencies_within_1e5_of_oracle(shape):
    nx, ny, nz = shape
    say(f"fp32 {shape}")
    g, host = case(nx, ny, nz, 2, seed=600 + nx)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    got = narrow_tendencies(host, g, dt, M.MONC_F32, [300.0, 0.0])
    errs = [rel_err(a, b) for a, b in zip(got, ref)]
    say(f"  fp32 relative errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("dtype", [M.MONC_F32, M.MONC_BF16])
@pytest.mark.parametrize("shape", [(37, 29, 45), (17, 23, 96)])
def test_separate_narrow_entry_points_equal_the_fused_call(dtype, shape):
    """monc_advect_pw_f32/_bf16 and monc_advect_tvd_f32/_bf16 give bitwise the
    momentum and scalar outputs of monc_advect with the same dtype (whose
    parity with the oracle the tests above establish)."""
    nx, ny, nz = shape
    say(f"separate narrow entry points dtype={dtype} {shape}")
    T = torch()
    g, host = case(nx, ny, nz, 2, seed=640 + nz)
    dt, phi0 = 0.5, [300.0, 0.0]
    d = to_dev(host)
    tdt = T.float32 if dtype == M.MONC_F32 else T.int16
    work = [T.empty(x.shape, dtype=tdt, device=dev()) for x in d]
    M.monc_cast_working(dtype, d, work, [0.0, 0.0, 0.0] + phi0)
    fused = [T.full(x.shape, np.nan, dtype=T.float32, device=dev()) for x in d]
    M.monc_advect(dtype, work, fused, g.dx, g.dy, prof_dev(g), dt, phi0=phi0)
    sep = [T.full(x.shape, np.nan, dtype=T.float32, device=dev()) for x in d]
    M.monc_advect_pw_narrow(dtype, *work[:3], *sep[:3], g.dx, g.dy, prof_dev(g))
    M.monc_advect_tvd_narrow(dtype, *work[:3], work[3:], sep[3:], g.dx, g.dy, prof_dev(g), dt,
                             phi0=phi0)
    T.cuda.synchronize()
    for n, (a, b) in enumerate(zip(sep, fused)):
        ia, ib = I.interior(a.cpu().numpy()), I.interior(b.cpu().numpy())
        assert np.all(np.isfinite(ia)), n
        np.testing.assert_array_equal(ia, ib)


@pytest.mark.parametrize("shape", [(32, 32, 32), (40, 36, 128)])
def test_bf16_storage_error_is_bounded(shape):
    nx, ny, nz = shape
    say(f"bf16 {shape}")
    g, host = case(nx, ny, nz, 2, seed=610 + nx)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    got = narrow_tendencies(host, g, dt, M.MONC_BF16, [300.0, 0.0])
    errs = [rel_err(a, b) for a, b in zip(got, ref)]
    say(f"  bf16 relative errors {['%.2e' % e for e in errs]}")
    # BF16 keeps 8 significant bits: each stored value is off by up to 2^-9
    # of itself, while neighbouring cells differ by only about 1% (the noise
    # level), so the fluxes' differences can be off by tens of percent of
    # themselves.  The bound only guards against a broken path; the errors
    # are what the precision form reports.
    assert max(errs) <= 0.25, errs


@pytest.mark.parametrize("shape", [(3, 2, 5), (4, 4, 7), (5, 1, 9), (16, 12, 64), (1, 1, 2)])
def test_cast_working_is_exact_rounding(shape):
    """The marshalling cast writes round-to-nearest-even of (x - offset) in
    FP32, and BF16 as the FP32 value rounded again to nearest even, over the
    whole padded array; padded sizes with every remainder modulo 4 (the
    kernel converts four values per lane and leaves the rest to a tail)."""
    from oracle import mlp_ref as R
    nx, ny, nz = shape
    say(f"cast {shape}")
    T = torch()
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    src = [rng.standard_normal((nx + 4, ny + 4, nz)) * 10.0 ** rng.integers(-3, 3)
           for _ in range(4)]
    src[3] = 300.0 + src[3]
    src[0][0, 0, 0] = np.inf
    src[1][-1, -1, -1] = np.nan
    offs = [0.0, 1.5, -2.25, 300.0]
    d = to_dev(src)
    w32 = [T.full(x.shape, np.nan, dtype=T.float32, device=dev()) for x in d]
    w16 = [T.full(x.shape, -1, dtype=T.int16, device=dev()) for x in d]
    M.monc_cast_working(M.MONC_F32, d, w32, offs)
    M.monc_cast_working(M.MONC_BF16, d, w16, offs)
    T.cuda.synchronize()
    for n in range(4):
        exp32 = (src[n] - offs[n]).astype(np.float32)
        got32 = w32[n].cpu().numpy()
        assert np.array_equal(got32.view(np.uint32), exp32.view(np.uint32)) or \
            np.array_equal(got32, exp32, equal_nan=True), n
        exp16 = R.bf16(src[n] - offs[n])
        got16 = (w16[n].cpu().numpy().astype(np.int32) & 0xFFFF).astype(np.uint32) << 16
        got16 = got16.view(np.float32).astype(np.float64)
        assert np.array_equal(got16, exp16, equal_nan=True), n


@pytest.mark.parametrize("shape", [(32, 32, 32), (40, 36, 128), (17, 23, 96)])
def test_bf16_path_equals_oracle_of_rounded_inputs(shape):
    """The BF16 path rounds its inputs (scalars as anomalies from phi0) to
    BF16 and computes in FP32: it must match the FP64 oracle evaluated on
    exactly those rounded inputs to the FP32 bar.  (Its difference from the
    oracle on the unrounded inputs is the storage error the precision form
    reports.)"""
    from oracle import mlp_ref as R
    nx, ny, nz = shape
    say(f"bf16 vs oracle of rounded inputs {shape}")
    g, host = case(nx, ny, nz, 2, seed=615 + nx)
    dt = 0.5
    phi0 = [300.0, 0.0]
    offs = [0.0, 0.0, 0.0] + phi0
    rounded = [o + R.bf16(h - o) for h, o in zip(host, offs)]
    ref = oracle_tendencies(rounded, g, dt)
    got = narrow_tendencies(host, g, dt, M.MONC_BF16, phi0)
    errs = [rel_err(a, b) for a, b in zip(got, ref)]
    say(f"  relative errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= 1e-5, errs


def test_anomaly_offset_is_exact_in_fp64():
    """Storing theta as an anomaly and passing phi0 gives the FP64 tendency of
    the full field (affine equivariance of the flux form)."""
    g, host = case(24, 20, 32, 2, seed=620)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    T = torch()
    anom = [h.copy() for h in host]
    anom[3] = anom[3] - 300.0
    d = to_dev(anom)
    out = [T.zeros_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), dt, phi0=[300.0, 0.0])
    T.cuda.synchronize()
    assert rel_err(out[3].cpu().numpy(), ref[3]) <= 1e-12


def test_mixed_step_matches_oracle_to_fp32_accuracy():
    say("mixed step")
    g, host = case(40, 36, 64, 2, seed=630)
    dt = 0.5
    ref = O.step([h.copy() for h in host], g, dt)
    T = torch()
    d = to_dev(host)
    out = [T.full_like(x, float("nan")) for x in d]
    b = T.zeros(M.MONC_NBUDGET, dtype=T.float64, device=dev())
    ws = T.empty(M.monc_step_workspace_bytes(40, 36, 64, 2), dtype=T.uint8, device=dev())
    M.monc_step_mixed(d, out, [300.0, 0.0], g.dx, g.dy, prof_dev(g), dt, b, ws)
    T.cuda.synchronize()
    for n in range(5):
        e = rel_err(out[n].cpu().numpy() - host[n], ref[n] - host[n])
        assert e <= 1e-5, (n, e)
    bh = b.cpu().numpy()
    assert M.monc_budgets_check(bh) == M.MONC_OK
    # the state itself stays FP64: increments are added to the FP64 values
    assert out[3].dtype == T.float64


@pytest.mark.parametrize("nscal", [5, 8])
def test_many_scalars_use_several_passes(nscal):
    say(f"nscal {nscal}")
    g, host = case(21, 18, 40, nscal, seed=640 + nscal)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    T = torch()
    d = to_dev(host)
    out = [T.zeros_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), dt)
    T.cuda.synchronize()
    for n, (a, r) in enumerate(zip(out, ref)):
        assert rel_err(a.cpu().numpy(), r) <= TOL64, n
    # the step with budgets (passes of three scalars on these 40-level columns)
    stp = O.step([h.copy() for h in host], g, dt)
    out = [T.full_like(x, float("nan")) for x in d]
    b = T.zeros(M.MONC_NBUDGET, dtype=T.float64, device=dev())
    ws = T.empty(M.monc_step_workspace_bytes(21, 18, 40, nscal), dtype=T.uint8, device=dev())
    M.monc_step(d, out, g.dx, g.dy, prof_dev(g), dt, b, ws)
    T.cuda.synchronize()
    for n in range(3 + nscal):
        assert rel_err(out[n].cpu().numpy() - host[n], stp[n] - host[n]) <= TOL64, n
    ob, sc = O.budgets(*host[:3], *ref[:3], host[3:], ref[3:], g)
    gb = M.budgets_dict(b.cpu().numpy(), nscal)
    for s in range(nscal):
        assert abs(gb[f"M_s{s}"] - ob[f"M_s{s}"]) <= 1e-13 * abs(ob[f"M_s{s}"])
        assert gb[f"min_s{s}"] == ob[f"min_s{s}"]
    assert gb["nonfinite"] == 0


@pytest.mark.parametrize("shape", [(12, 10, 96), (9, 7, 65), (11, 13, 64), (6, 5, 3)])
def test_ragged_column_heights(shape):
    nx, ny, nz = shape
    say(f"ragged nz {shape}")
    g, host = case(nx, ny, nz, 2, seed=650 + nz)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    T = torch()
    d = to_dev(host)
    out = [T.zeros_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), dt)
    T.cuda.synchronize()
    for n, (a, r) in enumerate(zip(out, ref)):
        assert rel_err(a.cpu().numpy(), r) <= TOL64, n


@pytest.mark.timeout(900)
def test_steps512_budgets_every_step():
    """512 x 512 x 128, u v w th q1 q2 q3 (divergence-free flow), 100 forward
    steps at dt = 0.5 s with the budgets checked after every step: momentum
    and scalar mass conserved, the KE identity closes, the w boundary term
    matches its closed form, mass changes by exactly dt*C, q stays positive,
    no Courant violation."""
    w, g, f = I.make_workload("steps512", padded=True)
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    say("steps512: oracle budgets of the first state")
    hosts = [O.halo_fill(f.pop(n)) for n in names]
    first = [h.copy() for h in hosts]
    tend = oracle_tendencies(hosts, g, w.dt)
    ob, sc = O.budgets(*hosts[:3], *tend[:3], hosts[3:], tend[3:], g)
    scal_scale = [np.sum(np.abs(I.interior(t)) * (g.rhon / g.rdz)[None, None, :]) for t in tend[3:]]
    del tend
    T = torch()
    A = [T.from_numpy(h).to(dev()) for h in hosts]
    del hosts
    B = [T.empty_like(x) for x in A]
    prof = prof_dev(g)
    b = T.zeros(M.MONC_NBUDGET, dtype=T.float64, device=dev())
    ws = T.empty(M.monc_step_workspace_bytes(w.nx, w.ny, w.nz, w.nscal), dtype=T.uint8,
                 device=dev())
    rho = T.from_numpy(g.rho).to(dev())
    prev = None
    for step in range(w.steps):
        M.monc_step(A, B, g.dx, g.dy, prof, w.dt, b, ws)
        wt = A[2][2:-2, 2:-2]
        closed = float((rho[0] * wt[:, :, 0] ** 2 - rho[w.nz - 2] * wt[:, :, w.nz - 2] ** 2).sum() / 4)
        bh = b.cpu().numpy()
        gb = M.budgets_dict(bh, w.nscal)
        assert M.monc_budgets_check(bh) == M.MONC_OK, (step, gb["courant"], gb["nonfinite"])
        if step == 0:
            # the flow is divergence-free, so Q (and P) vanish up to round-off:
            # each side of the identity P = Q is compared on the scale of P's terms
            for name in ["C_u", "C_v", "C_w", "P_u", "Q_u", "P_v", "Q_v", "P_w", "Q_w"]:
                scale = sc["P_" + name[2]] if name[0] in "PQ" else sc[name]
                assert abs(gb[name] - ob[name]) <= 1e-12 * scale, name
        assert abs(gb["C_u"]) <= 1e-12 * sc["C_u"], step
        assert abs(gb["C_v"]) <= 1e-12 * sc["C_v"], step
        assert abs(gb["C_w"] - closed) <= 1e-12 * sc["C_w"], step
        for c in "uvw":
            assert abs(gb[f"P_{c}"] - gb[f"Q_{c}"]) <= 1e-11 * sc[f"P_{c}"], (step, c)
        for s in range(w.nscal):
            assert abs(gb[f"C_s{s}"]) <= 1e-12 * scal_scale[s], (step, s)
            if prev is not None:
                drift = gb[f"M_s{s}"] - prev[f"M_s{s}"] - w.dt * prev[f"C_s{s}"]
                assert abs(drift) <= 1e-13 * abs(gb[f"M_s{s}"]) + 1e-9, (step, s, drift)
        for s in range(1, w.nscal):
            assert gb[f"min_s{s}"] > 0.0, (step, s)
        prev = gb
        A, B = B, A
        if step % 20 == 0:
            say(f"  step {step}: courant {gb['courant']:.3f} C_u {gb['C_u']:.2e} "
                f"P_u-Q_u {gb['P_u'] - gb['Q_u']:.2e}")

    # the state after the 100 steps against 100 oracle steps, whole domain
    say("steps512: 100 oracle steps")
    cur = [x.copy() for x in first]
    nxt = [np.empty_like(x) for x in first]
    for step in range(w.steps):
        O.step(cur, g, w.dt, out=nxt)
        cur, nxt = nxt, cur
        if step % 20 == 0:
            say(f"  oracle step {step}")
    del nxt
    T.cuda.synchronize()
    for n in range(3 + w.nscal):
        got = I.interior(A[n].cpu().numpy())
        exp = I.interior(cur[n])
        start = I.interior(first[n])
        change = np.abs(exp - start).max()
        err = np.abs(got - exp).max()
        bar = STEPS512_GROWTH * w.steps * np.spacing(np.abs(exp).max())
        say(f"  field {n}: |gpu - oracle| {err:.3e}, bar {bar:.3e}, "
            f"relative to the change {err / change:.3e}")
        assert err <= bar, (n, err, bar)


def test_big1024_precision_forms_match_oracle():
    """The precision forms at the headline size and in the launch configuration
    the benchmark times (FP32 and BF16 working copies with the scalars stored
    as anomalies from their nominal values, the mixed step), over the whole
    domain against the FP64 oracle, per field max |gpu - oracle| /
    max |oracle|."""
    say("big1024 precision forms")
    w, g, f = I.make_workload("big1024")
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    T = torch()
    hosts = [O.halo_fill(I.pad(f.pop(n))) for n in names]
    d = [T.from_numpy(h).to(dev()) for h in hosts]
    prof = prof_dev(g)
    # scalars stored as anomalies from their nominal values (theta 300 K,
    # tracers 1e-3): the working copies then round the variation, not the mean
    phi0 = [300.0] + [1e-3] * (w.nscal - 1)
    offs = [0.0, 0.0, 0.0] + phi0
    outs = {}
    for name, code, tdt in (("f32", M.MONC_F32, T.float32), ("bf16", M.MONC_BF16, T.int16)):
        work = [T.empty(x.shape, dtype=tdt, device=dev()) for x in d]
        M.monc_cast_working(code, d, work, offs)
        o = [T.empty(x.shape, dtype=T.float32, device=dev()) for x in d]
        M.monc_advect(code, work, o, g.dx, g.dy, prof, w.dt, phi0=phi0)
        outs[name] = o
        del work
    mixed = [T.empty_like(x) for x in d]
    M.monc_step_mixed(d, mixed, phi0, g.dx, g.dy, prof, w.dt)
    T.cuda.synchronize()
    say("  oracle over the whole domain")
    ref = oracle_tendencies(hosts, g, w.dt)
    for n in range(len(d)):
        exp = I.interior(ref[n])
        den = np.abs(exp).max()
        e32 = np.abs(I.interior(outs["f32"][n].double().cpu().numpy()) - exp).max() / den
        e16 = np.abs(I.interior(outs["bf16"][n].double().cpu().numpy()) - exp).max() / den
        inc = I.interior(mixed[n].cpu().numpy()) - I.interior(hosts[n])
        emx = np.abs(inc - w.dt * exp).max() / (w.dt * den)
        say(f"  field {n}: fp32 {e32:.2e} bf16 {e16:.2e} mixed {emx:.2e}")
        assert e32 <= 1e-5, (n, e32)
        assert e16 <= 0.25, (n, e16)
        assert emx <= 1e-5, (n, emx)
