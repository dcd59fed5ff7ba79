"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Metric for states: err = max |x - x_ref| / max(|x_ref|, tau), tau = 1e-30, which keeps
cells whose occupation underflows FP32 meaningful (two independent FP64 routes of the
oracle agree to about 2e-16 under this metric).  Bars: FP64 path 1e-12, mixed path 1e-8.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1809_05608_amd import tm

pytestmark = pytest.mark.gpu
TAU = 1e-30
FP64_BAR = 1e-12
MIXED_BAR = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, ref):
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), TAU)))


def _ctx(wd, precision=tm.PREC_FP64):
    return tm.Context(tm.problem_of(wd, precision)), tm.DeviceFields.of(wd)


def gpu_newton(w, max_iter, rtol, precision=tm.PREC_FP64, raise_on_status=False):
    wd = w.to("cuda")
    ctx, f = _ctx(wd, precision)
    psi = wd.psi_n.clone()
    st, stats = ctx.newton_step(f, wd.psi_n, psi, max_iter, rtol, raise_on_status=raise_on_status)
    torch.cuda.synchronize()
    return st, psi.cpu().numpy(), {k: v.cpu().numpy() for k, v in stats.items()}


def oracle_newton(w, max_iter, rtol, systems=None):
    return oracle.newton_batch(w.numpy(), max_iter=max_iter, rtol=rtol, systems=systems)


RAGGED = [
    dict(S=1, R=3, I=1, N=1),      # single zone, single group
    dict(S=2, R=3, I=37, N=13),    # padded groups (16), odd systems per block
    dict(S=1, R=5, I=19, N=20),
    dict(S=1, R=2, I=9, N=32),     # maximum group count
    dict(S=3, R=1, I=2, N=5),
]


# ------------------------------------------------------------------ residual and blocks

@pytest.mark.parametrize("shape", [dict(S=1, R=16, I=64, N=12)] + RAGGED)
def test_residual_and_blocks_match_oracle(shape):
    say("case residual/blocks", shape)
    w = synth.make_custom(**shape)
    rng = np.random.default_rng(11)
    psi = (w.psi_n.numpy() * rng.uniform(0.7, 1.3, w.psi_n.shape)).clip(0, 1)
    wd = w.to("cuda")
    ctx, f = _ctx(wd)
    psi_d = torch.as_tensor(psi, device="cuda")
    G = torch.empty_like(psi_d)
    B = torch.empty(tuple(psi_d.shape) + (w.N + 2,), dtype=torch.float64, device="cuda")
    ctx.assemble(f, wd.psi_n, psi_d, G, B)
    torch.cuda.synchronize()
    G, B = G.cpu().numpy(), B.cpu().numpy()
    wn = w.numpy()
    syss = oracle.systems_from_workload(wn)
    for s in range(w.S):
        for r in range(w.R):
            Go = oracle.residual(syss[s][r], wn["psi_n"][s, r], psi[s, r])
            np.testing.assert_allclose(G[s, r], Go, rtol=1e-11, atol=1e-13)
            A, bm, bp = oracle.jacobian_blocks(syss[s][r], psi[s, r])
            scale = np.max(np.abs(A), axis=2, keepdims=True)
            np.testing.assert_allclose(B[s, r, :, :, :w.N], A, rtol=0, atol=1e-12 * scale.max())
            np.testing.assert_allclose(B[s, r, :, :, w.N], bm, rtol=1e-11, atol=1e-14 * scale.max())
            np.testing.assert_allclose(B[s, r, :, :, w.N + 1], bp, rtol=1e-11, atol=1e-14 * scale.max())


# Temperature scaled far below and above the synthetic profile (eq. d8's detailed-balance factor
# exp(-|eps_k - eps_k'|/T)): cold zones make the factors of distant groups underflow to 0, hot zones
# bring every factor near 1.  The residual's NES sums (products of neighbour factors, summed from the far
# end) must match the oracle, which takes each factor directly; there the NES amplitude is raised 1e5-fold
# so that the NES source dominates the residual (about 1e4 times the rest).  The Newton steps run at 10
# times the synthetic amplitude (NES about as large as the rest), where diagonal pivoting holds (no
# fallback), so the float32 NES block of the mixed update (one exp2 per entry, weights split by side)
# does the solves.
@pytest.mark.parametrize("t_scale", [0.02, 50.0])
def test_nes_at_extreme_temperatures_matches_oracle(t_scale):
    say("case NES extreme temperature", t_scale)
    base = synth.make_custom(S=2, R=4, I=24, N=20)
    w = dataclasses.replace(base, temp=(base.temp * t_scale).contiguous(), nes_amp=(base.nes_amp * 1e5).contiguous())
    rng = np.random.default_rng(5)
    psi = (w.psi_n.numpy() * rng.uniform(0.7, 1.3, w.psi_n.shape)).clip(0, 1)
    wd = w.to("cuda")
    ctx, f = _ctx(wd)
    psi_d = torch.as_tensor(psi, device="cuda")
    G = torch.empty_like(psi_d)
    ctx.assemble(f, wd.psi_n, psi_d, G, None)
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    wn = w.numpy()
    syss = oracle.systems_from_workload(wn)
    for s in range(w.S):
        for r in range(w.R):
            Go = oracle.residual(syss[s][r], wn["psi_n"][s, r], psi[s, r])
            np.testing.assert_allclose(G[s, r], Go, rtol=1e-11, atol=1e-13)
    w = dataclasses.replace(base, temp=(base.temp * t_scale).contiguous(), nes_amp=(base.nes_amp * 10.0).contiguous())
    ref, _ = oracle_newton(w, 30, 1e-12)
    for precision, bar in [(tm.PREC_FP64, FP64_BAR), (tm.PREC_MIXED, MIXED_BAR)]:
        st, psi_m, stats = gpu_newton(w, 30, 1e-12, precision=precision)
        assert st == 0, tm.STATUS_NAMES[st]
        assert not np.any(stats["flags"] & tm.FLAG_PIVOT_FALLBACK)
        assert rel_err(psi_m, ref) < bar


def test_kernel_timing_brackets_the_factor_launch():
    """The measurement aid: with timing on, a solve records two events around its factor launch; off (or
    before any timed call) the query is an invalid argument."""
    say("case kernel timing")
    w = synth.make_custom(S=2, R=8, I=40, N=12)
    wd = w.to("cuda")
    for precision in (tm.PREC_FP64, tm.PREC_MIXED):
        ctx, f = _ctx(wd, precision)
        rhs = torch.ones_like(wd.psi_n)
        x = torch.empty_like(rhs)
        with pytest.raises(tm.TMError, match="INVALID_ARG"):
            ctx.kernel_time_ms()
        ctx.set_kernel_timing(True)
        with pytest.raises(tm.TMError, match="INVALID_ARG"):
            ctx.kernel_time_ms()
        ctx.factor_solve(f, wd.psi_n, rhs, x)
        ms = ctx.kernel_time_ms()
        assert 0.0 < ms < 1e4
        ctx.set_kernel_timing(False)
        with pytest.raises(tm.TMError, match="INVALID_ARG"):
            ctx.kernel_time_ms()
        ctx.close()


# ------------------------------------------------------------------ linear solves

@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("precision", [tm.PREC_FP64, tm.PREC_MIXED])
@pytest.mark.parametrize("shape", [dict(S=1, R=16, I=64, N=12)] + RAGGED)
def test_factor_solve_matches_oracle(shape, precision, transpose):
    say("case factor_solve", shape, "prec", precision, "T", transpose)
    w = synth.make_custom(**shape)
    rng = np.random.default_rng(12)
    psi = w.psi_n.numpy() * 1.05
    rhs = rng.standard_normal(psi.shape)
    wd = w.to("cuda")
    ctx, f = _ctx(wd, precision)
    x = torch.empty(psi.shape, dtype=torch.float64, device="cuda")
    ctx.factor_solve(f, torch.as_tensor(psi, device="cuda"), torch.as_tensor(rhs, device="cuda"), x, transpose)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    wn = w.numpy()
    syss = oracle.systems_from_workload(wn)
    bar = 1e-11 if precision == tm.PREC_FP64 else 3e-4
    for s in range(w.S):
        for r in range(w.R):
            A, bm, bp = oracle.jacobian_blocks(syss[s][r], psi[s, r])
            xo = oracle.block_thomas_solve(A, bm, bp, rhs[s, r], transpose=transpose)
            err = np.max(np.abs(x[s, r] - xo)) / np.max(np.abs(xo))
            assert err < bar, (s, r, err)


# ------------------------------------------------------------------ Newton step

def test_newton_cfg0_three_iterations_fp64():
    """16 rays x 64 zones x 12 groups, exactly 3 Newton updates."""
    say("case newton cfg0")
    w = synth.make(0)
    st, psi, stats = gpu_newton(w, 3, 0.0)
    assert st == 0, tm.STATUS_NAMES[st]
    ref, info = oracle_newton(w, 3, 0.0)
    assert rel_err(psi, ref) < FP64_BAR
    assert np.all(stats["iters"] == 3) and np.all(stats["flags"] == 0)
    wn = w.numpy()
    syss = oracle.systems_from_workload(wn)
    for r in range(w.R):
        so = oracle.step_stats(syss[0][r], wn["psi_n"][0, r], ref[0, r])
        np.testing.assert_allclose(stats["n_tot"][r], so["n_tot"], rtol=1e-12)
        np.testing.assert_allclose(stats["e_tot"][r], so["e_tot"], rtol=1e-12)
        np.testing.assert_allclose(stats["lum_n"][r], so["lum_n"], rtol=1e-11)
        np.testing.assert_allclose(stats["budget_n"][r], so["budget"], rtol=1e-6, atol=1e-9 * abs(so["n_tot"]))
        np.testing.assert_allclose(stats["res0_inf"][r], info[(0, r)].res0, rtol=1e-12)


@pytest.mark.parametrize("shape", RAGGED)
def test_newton_ragged_shapes_fp64(shape):
    say("case newton ragged", shape)
    w = synth.make_custom(**shape)
    st, psi, stats = gpu_newton(w, 4, 0.0)
    assert st == 0
    ref, _ = oracle_newton(w, 4, 0.0)
    assert rel_err(psi, ref) < FP64_BAR


def test_newton_to_tolerance_cfg1_sampled_rays():
    """Four species on sampled rays of the 180-ray configuration, Newton to 1e-10 relative residual:
    the same per-system iteration counts and states as the oracle."""
    say("case newton cfg1 rays")
    w = synth.make(1, rays=[0, 97, 179])
    st, psi, stats = gpu_newton(w, 30, 1e-10)
    assert st == 0, tm.STATUS_NAMES[st]
    ref, info = oracle_newton(w, 30, 1e-10)
    assert rel_err(psi, ref) < FP64_BAR
    for (s, r), res in info.items():
        assert stats["iters"][s * w.R + r] == res.iters


@pytest.mark.parametrize("terms,limiter,outer_bc", [(1, 1, 0), (1, 0, 1), (2, 1, 1), (4 | 1, 1, 0), (7, 0, 0)])
def test_newton_term_subsets(terms, limiter, outer_bc):
    say("case terms", terms, limiter, outer_bc)
    w = dataclasses.replace(synth.make_custom(S=2, R=3, I=24, N=10), terms=terms, limiter=limiter, outer_bc=outer_bc)
    st, psi, _ = gpu_newton(w, 3, 0.0)
    ref, _ = oracle_newton(w, 3, 0.0)
    assert rel_err(psi, ref) < FP64_BAR


def test_mixed_precision_refines_to_fp64_answer():
    """Mixed path (FP32 factorisation, FP64 residual/update) on rays of the spiked
    4096-ray configuration including opacity-spike rays: within 1e-8 of the FP64 oracle."""
    ids, _, _ = synth.workload._spikes(2, 4096, 540)
    rays = [int(ids[0]), int(ids[1]), 5]
    say("case mixed cfg2 rays", rays)
    w = synth.make(2, rays=rays)
    st, psi, stats = gpu_newton(w, 30, 1e-12, precision=tm.PREC_MIXED)
    assert st == 0, tm.STATUS_NAMES[st]
    ref, info = oracle_newton(w, 30, 1e-12)
    assert rel_err(psi, ref) < MIXED_BAR
    # every system reached max(1e-12 * res0, rounding level of G)
    assert not np.any(stats["flags"] & tm.FLAG_NOT_CONVERGED)
    assert np.all(stats["res_inf"] <= 1e-10 * stats["res0_inf"])


# Standalone-solve bar of each float32 factor kernel against the oracle's FP64 block-Thomas solve: float32
# elimination (about 1e-6 times the growth of these blocks), and for the variant whose NES diagonal sums are
# single bf16 products (8-bit significands, 2^-9 relative per term) a bar of 2^-9 times the same factor.
SOLVE_BAR = {"mfma": 3e-4, "valu": 3e-4, "lane": 3e-4, "window": 3e-4, "bf16x3": 3e-4, "bf16": 2e-2}


def _fine_grid(N):
    # energy-group edges 2..20 MeV: adjacent groups 12% apart, closer than the 25% the windowed NES form needs
    return 2.0 * 10.0 ** (torch.arange(N + 1, dtype=torch.float64) / N)


@pytest.mark.parametrize("kernel", ["mfma", "valu", "lane", "window", "bf16x3", "bf16"])
@pytest.mark.parametrize("shape", [dict(S=2, R=9, I=31, N=20), dict(S=1, R=17, I=12, N=13), dict(S=3, R=2, I=5, N=3),
                                   dict(S=1, R=33, I=7, N=8), dict(S=1, R=5, I=9, N=20, fine=True)])
def test_float32_factor_kernels_agree_with_oracle(monkeypatch, shape, kernel):
    """The float32 diagonal-pivot factor kernels (one system per quad with the rank-1 updates on the matrix
    cores or on the vector units; the NES block from one exp2 per entry or from the energy-window
    scalings, its diagonal sums on the vector units or as bf16 matrix-core contractions; one row per
    lane): standalone solves within the kernel's bar of the oracle's block-Thomas solve, and the mixed
    Newton step refined to 1e-12 within the mixed bar of the FP64 oracle; system counts that leave
    partial quads and wave groups; a fine energy grid on which the windowed NES form hands over to the
    exp2 form."""
    monkeypatch.setenv("TM_FACTOR_KERNEL", kernel)
    say("case f32 kernel", kernel, shape)
    shape = dict(shape)
    fine = shape.pop("fine", False)
    w = synth.make_custom(**shape, **(dict(e_edge=_fine_grid(shape["N"])) if fine else {}))
    rng = np.random.default_rng(7)
    psi = w.psi_n.numpy() * 1.03
    rhs = rng.standard_normal(psi.shape)
    wd = w.to("cuda")
    ctx, f = _ctx(wd, tm.PREC_MIXED)
    x = torch.empty(psi.shape, dtype=torch.float64, device="cuda")
    ctx.factor_solve(f, torch.as_tensor(psi, device="cuda"), torch.as_tensor(rhs, device="cuda"), x, False)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    syss = oracle.systems_from_workload(w.numpy())
    for s in range(w.S):
        for r in range(w.R):
            A, bm, bp = oracle.jacobian_blocks(syss[s][r], psi[s, r])
            xo = oracle.block_thomas_solve(A, bm, bp, rhs[s, r])
            assert np.max(np.abs(x[s, r] - xo)) / np.max(np.abs(xo)) < SOLVE_BAR[kernel], (s, r)
    pd = wd.psi_n.clone()
    st, stats = ctx.newton_step(f, wd.psi_n, pd, 30, 1e-12, raise_on_status=False)
    torch.cuda.synchronize()
    assert st == 0, tm.STATUS_NAMES[st]
    ref, _ = oracle_newton(w, 30, 1e-12)
    assert rel_err(pd.cpu().numpy(), ref) < MIXED_BAR


# ------------------------------------------------------------------ adjoint

def _adjoint_workload():
    w = synth.make_custom(S=1, R=3, I=12, N=6)
    return dataclasses.replace(w, kappa_a=w.kappa_a * 30, eta=w.eta * 30, kappa_s=w.kappa_s * 30,
                               nes_amp=w.nes_amp * 300)


def test_adjoint_matches_oracle():
    say("case adjoint")
    w = _adjoint_workload()
    ref, _ = oracle_newton(w, 40, 1e-14)
    wn = w.numpy()
    syss = oracle.systems_from_workload(wn)
    wd = w.to("cuda")
    ctx, f = _ctx(wd)
    psi = torch.as_tensor(ref, device="cuda")
    seed = np.zeros_like(ref)
    for r in range(w.R):
        seed[0, r] = oracle.luminosity_seed(syss[0][r], ref[0, r].shape)
    seed_d = torch.empty_like(psi)
    ctx.luminosity_seed(f, seed_d)
    torch.cuda.synchronize()
    np.testing.assert_allclose(seed_d.cpu().numpy(), seed, rtol=1e-14, atol=0)
    mu = torch.empty_like(psi)
    g = {n: torch.empty_like(psi) for n in ("kappa_a", "eta", "kappa_s")}
    gamp = torch.empty(w.S, w.R, w.I, dtype=torch.float64, device="cuda")
    ctx.adjoint_step(f, wd.psi_n, psi, seed_d, mu, g["kappa_a"], g["eta"], g["kappa_s"], gamp)
    torch.cuda.synchronize()
    for r in range(w.R):
        mo = oracle.adjoint(syss[0][r], ref[0, r], seed[0, r])
        go = oracle.param_vjp(syss[0][r], ref[0, r], mo)
        sc = np.max(np.abs(mo))
        np.testing.assert_allclose(mu[0, r].cpu().numpy(), mo, rtol=1e-10, atol=1e-12 * sc)
        for n in g:
            gs = np.max(np.abs(go[n]))
            np.testing.assert_allclose(g[n][0, r].cpu().numpy(), go[n], rtol=1e-9, atol=1e-11 * gs)
        # g_amp_i = c sum_k mu_ik S_ik nearly cancels where mu_k ~ W_k (number conservation makes
        # sum_k W_k S_k = 0), so its rounding floor scales with sum_k |mu_ik S_ik|, not with |g|
        S1 = oracle.transport.nes_source(syss[0][r], ref[0, r], unit_amplitude=True)
        floor = w.c_dt * np.sum(np.abs(mo * S1), axis=1)
        err = np.abs(gamp[0, r].cpu().numpy() - go["nes_amp"])
        assert np.all(err <= 1e-12 * floor + 1e-9 * np.abs(go["nes_amp"])), (err, floor)


def test_transport_step_autograd_matches_oracle_gradient():
    say("case autograd")
    w = _adjoint_workload()
    wd = w.to("cuda")
    ctx, f = _ctx(wd)
    ka = wd.kappa_a.clone().requires_grad_(True)
    et = wd.eta.clone().requires_grad_(True)
    pn = wd.psi_n.clone().requires_grad_(True)
    psi = tm.TransportStep.apply(ka, et, wd.kappa_s, pn, ctx, f, 40, 1e-14)
    seed = torch.empty_like(psi)
    ctx.luminosity_seed(f, seed)                               # dL/dpsi, outer zone only
    L = (psi * seed).sum()
    L.backward()
    wn = w.numpy()
    syss = oracle.systems_from_workload(wn)
    ref, _ = oracle_newton(w, 40, 1e-14)
    for r in range(w.R):
        seed = oracle.luminosity_seed(syss[0][r], ref[0, r].shape)
        mo = oracle.adjoint(syss[0][r], ref[0, r], seed)
        go = oracle.param_vjp(syss[0][r], ref[0, r], mo)
        for name, t in (("kappa_a", ka), ("eta", et), ("psi_n", pn)):
            np.testing.assert_allclose(t.grad[0, r].cpu().numpy(), go[name], rtol=1e-8,
                                       atol=1e-10 * np.max(np.abs(go[name])))


# ------------------------------------------------------------------ failure handling (forced from the host)

def test_nonfinite_input_is_reported():
    say("case nonfinite")
    w = synth.make_custom(S=1, R=4, I=8, N=6)
    ka = w.kappa_a.clone()
    ka[0, 2, 3, 1] = float("nan")
    w = dataclasses.replace(w, kappa_a=ka)
    st, _, stats = gpu_newton(w, 3, 1e-10)
    assert st == 5                                  # TM_ERR_NONFINITE
    assert stats["flags"][2] & tm.FLAG_NONFINITE
    assert not np.any(stats["flags"][[0, 1, 3]] & tm.FLAG_NONFINITE)


def test_iteration_cap_is_reported():
    say("case not converged")
    w = synth.make_custom(S=1, R=2, I=8, N=6)
    st, _, stats = gpu_newton(w, 1, 1e-30)
    assert st == 4                                  # TM_ERR_NOT_CONVERGED
    assert np.all(stats["flags"] & tm.FLAG_NOT_CONVERGED) and np.all(stats["iters"] == 1)


@pytest.mark.parametrize("precision", [tm.PREC_FP64, tm.PREC_MIXED])
def test_singular_block_is_reported(precision):
    """A block with an exactly zero column, made from host inputs: emission/absorption only, c dt = 1,
    kappa_a = -1 and eta = 0 in one cell, so that diagonal entry 1 + c dt (kappa_a + eta) is exactly 0 in
    both precisions and no row below it can serve as a pivot.  The solve and the adjoint return
    TM_ERR_SINGULAR (after the partial-pivoting re-run); the other system's solution stays exact."""
    say("case singular block", precision)
    w = synth.make_custom(S=1, R=2, I=3, N=4, c_dt=1.0, terms=tm.TERM_EMABS, outer_bc=0)
    ka = torch.full_like(w.kappa_a, 0.25)
    et = torch.zeros_like(w.eta)
    ka[0, 1, 2, 3] = -1.0
    w = dataclasses.replace(w, kappa_a=ka, eta=et, kappa_s=torch.full_like(w.kappa_s, 2.0))
    wd = w.to("cuda")
    ctx, f = _ctx(wd, precision)
    rhs = torch.ones_like(wd.psi_n)
    x = torch.empty_like(rhs)
    with pytest.raises(tm.TMError) as e:
        ctx.factor_solve(f, wd.psi_n, rhs, x, False)
    assert e.value.status == 3                      # TM_ERR_SINGULAR
    xs = x.cpu().numpy()
    np.testing.assert_allclose(xs[0, 0], 1.0 / 1.25, rtol=1e-7)   # diagonal blocks 1 + c dt kappa_a
    assert not np.all(np.isfinite(xs[0, 1]))
    if precision == tm.PREC_FP64:
        mu = torch.empty_like(rhs)
        with pytest.raises(tm.TMError) as e:
            ctx.adjoint_step(f, wd.psi_n, wd.psi_n, rhs, mu)
        assert e.value.status == 3


def test_binding_rejects_bad_tensors():
    say("case binding checks")
    w = synth.make_custom(S=1, R=2, I=8, N=6).to("cuda")
    ctx, f = _ctx(w)
    with pytest.raises(ValueError):
        ctx.newton_step(f, w.psi_n, w.psi_n.float(), 1, 0.0)
    with pytest.raises(ValueError):
        ctx.newton_step(f, w.psi_n, w.psi_n[:, :1].clone(), 1, 0.0)


# ------------------------------------------------------------------ pivoting policies

@pytest.mark.parametrize("env", [dict(TM_PIVOT="always"), dict(TM_GROWTH_LIMIT="0"), dict(TM_PIVOT="auto")])
@pytest.mark.parametrize("precision", [tm.PREC_FP64, tm.PREC_MIXED])
def test_pivoting_policies_agree(monkeypatch, env, precision):
    """Diagonal pivots (default), forced partial pivoting, and a growth guard of 0 (every
    system takes the partial-pivoting re-run) all give the oracle's solve and Newton step."""
    say("case pivot policy", env, precision)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    w = synth.make_custom(S=2, R=5, I=30, N=20)
    wd = w.to("cuda")
    ctx, f = _ctx(wd, precision)
    rng = np.random.default_rng(13)
    psi = w.psi_n.numpy() * 1.02
    rhs = rng.standard_normal(psi.shape)
    x = torch.empty(psi.shape, dtype=torch.float64, device="cuda")
    ctx.factor_solve(f, torch.as_tensor(psi, device="cuda"), torch.as_tensor(rhs, device="cuda"), x, False)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    syss = oracle.systems_from_workload(w.numpy())
    bar = 1e-11 if precision == tm.PREC_FP64 else 3e-4
    for s in range(w.S):
        for r in range(w.R):
            A, bm, bp = oracle.jacobian_blocks(syss[s][r], psi[s, r])
            xo = oracle.block_thomas_solve(A, bm, bp, rhs[s, r])
            assert np.max(np.abs(x[s, r] - xo)) / np.max(np.abs(xo)) < bar
    pd = wd.psi_n.clone()
    st, stats = ctx.newton_step(f, wd.psi_n, pd, 30, 1e-12, raise_on_status=False)
    torch.cuda.synchronize()
    assert st == 0
    ref, _ = oracle_newton(w, 30, 1e-12)
    assert rel_err(pd.cpu().numpy(), ref) < (FP64_BAR if precision == tm.PREC_FP64 else MIXED_BAR)
    fallback = stats["flags"].cpu().numpy() & tm.FLAG_PIVOT_FALLBACK
    if env.get("TM_GROWTH_LIMIT") == "0":
        assert np.all(fallback)
    else:
        assert not np.any(fallback)


# ------------------------------------------------------------------ float32 range

def test_mixed_precision_converges_below_float32_range():
    """Occupations near 1e-200 (single zone and group): the float32 solve works on the residual
    scaled by a power of two per system, so the mixed Newton step still reaches the oracle's answer."""
    say("case mixed tiny occupations")
    w = synth.make_custom(S=2, R=3, I=1, N=1)
    assert float(np.max(w.psi_n.numpy())) < 1e-150
    st, psi, stats = gpu_newton(w, 30, 1e-12, precision=tm.PREC_MIXED)
    assert st == 0, tm.STATUS_NAMES[st]
    ref, _ = oracle_newton(w, 30, 1e-12)
    assert rel_err(psi, ref) < MIXED_BAR


# ------------------------------------------------------------------ caller workspace

@pytest.mark.parametrize("precision", [tm.PREC_FP64, tm.PREC_MIXED])
def test_caller_workspace_batches_equal_one_launch(precision):
    """A caller workspace sized for 7 systems factors the 22 systems in batches of 7, 7, 7 and 1
    (partial wave groups included): solves, transposed solves and the Newton step are bitwise those
    of the self-allocated single launch."""
    say("case caller workspace", precision)
    w = synth.make_custom(S=2, R=11, I=23, N=20)
    wd = w.to("cuda")
    rng = np.random.default_rng(41)
    psi = torch.as_tensor(w.psi_n.numpy() * 1.02, device="cuda")
    rhs = torch.as_tensor(rng.standard_normal(tuple(psi.shape)), device="cuda")
    out = []
    for batch in (0, 7):
        ctx, f = _ctx(wd, precision)
        if batch:
            ctx.set_workspace(ctx.workspace_bytes(batch))
        x = torch.empty_like(psi)
        xt = torch.empty_like(psi)
        ctx.factor_solve(f, psi, rhs, x, False)
        ctx.factor_solve(f, psi, rhs, xt, True)
        pd = wd.psi_n.clone()
        st, stats = ctx.newton_step(f, wd.psi_n, pd, 30, 1e-12, raise_on_status=False)
        torch.cuda.synchronize()
        assert st == 0
        out.append((x.cpu().numpy(), xt.cpu().numpy(), pd.cpu().numpy(), stats["iters"].cpu().numpy()))
        ctx.close()
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
