/*
 * tm.h - C ABI of libtm, an MI355X (gfx950) implementation of the implicit,
 * ray-by-ray multi-group flux-limited diffusion (MGFLD) neutrino-transport step
 * of the CHIMERA paper (Bruenn et al., arXiv 1809.05608).
 *
 * The operation: for every independent (species, ray) "system" of I radial zones
 * and N energy groups, advance the zeroth angular moment psi from time level n to
 * n+1 by backward Euler (eq. a58 with the flux of eq. a59 and limiter eq. a20,
 * lapse a = 1, Gamma = 1).  The residual per cell is
 *
 *   G_{i,k} = psi - psi^n + c dt [ (A_{i+1/2} H_{i+1/2} - A_{i-1/2} H_{i-1/2}) / V_i
 *                                  - eta (1 - psi) + kappa_a psi - S_{i,k} ]
 *
 * with emission/absorption with Pauli blocking (the source of eq. a54), and the
 * zeroth moment of inelastic NES-like scattering S (Phi_0 terms of eq. d8 in the
 * zone-centred discretisation of eq. d40).  The Newton iteration of eq. a62aa
 * solves the linearised system of eq. a62ae: block tridiagonal in radius with
 * dense N x N diagonal blocks and diagonal off-diagonal blocks.
 *
 * Geometry and energy grid (stated with eq. a59 and eqs. a01/a01b): zone centre
 * R_i = (R_{i-1/2} + R_{i+1/2})/2, V_i = (R_{i+1/2}^3 - R_{i-1/2}^3)/3,
 * A_{i+1/2} = R_{i+1/2}^2 (4 pi dropped), group centre
 * eps_k^2 = (e_{k+1/2}^2 + e_{k+1/2} e_{k-1/2} + e_{k-1/2}^2)/3,
 * W_k = (e_{k+1/2}^3 - e_{k-1/2}^3)/3.  Transport mean free path
 * 1/lambda = kappa_a + eta + kappa_s (eqs. d10, d8c); edge value
 * lambda_{i+1/2} = sqrt(lambda_i lambda_{i+1}).
 * Limited flux, m = max((psi_i + psi_{i+1})/2, psi_floor), D = R_{i+1} - R_i:
 *   H_{i+1/2} = -lambda m (psi_{i+1} - psi_i) / (3 D m + lambda |psi_{i+1} - psi_i|).
 * NES kernels (eq. d3 weighted symmetry, eq. d4 detailed balance), T = temp_i:
 *   K^out_{kk'} = nes_amp_i (eps_k eps_k'/(10 MeV)^2) nes_g[k][k'] (W_k'/mean W) min(1, e^{-(eps_k'-eps_k)/T})
 *   K^in_{kk'}  = same with min(1, e^{+(eps_k'-eps_k)/T})
 *   S_{i,k} = (1 - psi_k) sum_k' K^in_{kk'} psi_k' - psi_k sum_k' K^out_{kk'} (1 - psi_k')
 *
 * Conventions for every entry point:
 *  - All array pointers are DEVICE pointers (HBM), caller-owned, float64 unless
 *    stated.  The library never frees or keeps them after the call returns.
 *  - Layouts (row-major, last index fastest):
 *      cell  [S][R][I][N]   kappa_a, eta, kappa_s, psi, psi_n, residual, rhs, x, mu, seed, gradients
 *      zone  [R][I]         temp
 *      sysz  [S][R][I]      nes_amp, g_nes_amp
 *      edge  [R][I+1]       r_edge (cm), edge 0 is the inner boundary
 *      sys   [S][R]         every tm_stats array
 *      e_edge [N+1] (MeV) and nes_g [N][N] are shared by all systems.
 *  - One context is bound to one HIP stream given at creation; work is ordered on
 *    that stream.  A context is not thread-safe.  tm_newton_step, tm_ye_newton_step,
 *    tm_factor_solve and tm_adjoint_step synchronise the stream (they read back counts of
 *    unconverged systems, of systems for the pivoting re-run, or of zero pivots); the
 *    other entry points are asynchronous.
 *  - Errors are returned, never thrown.  Invalid shapes or null required pointers
 *    return TM_ERR_INVALID_ARG before any device work; HIP failures return
 *    TM_ERR_HIP with the message available from tm_last_error.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_OK = 0,
    TM_ERR_INVALID_ARG = 1,   /* bad shape, null pointer, unsupported option          */
    TM_ERR_HIP = 2,           /* a HIP runtime call failed (see tm_last_error)         */
    TM_ERR_SINGULAR = 3,      /* an exactly zero pivot in some block factorisation     */
    TM_ERR_NOT_CONVERGED = 4, /* some system missed the Newton tolerance in max_iter   */
    TM_ERR_NONFINITE = 5,     /* NaN or Inf in some system's residual or update        */
    TM_ERR_WORKSPACE = 6      /* caller workspace too small, or allocation failed      */
} tm_status;

/* terms bitmask */
#define TM_TERM_DIFFUSION 1u  /* radial flux-limited diffusion (eqs. a58, a59, a20)    */
#define TM_TERM_EMABS     2u  /* emission/absorption with Pauli blocking (eq. a54)    */
#define TM_TERM_NES       4u  /* inelastic NES-like scattering, Phi_0 (eqs. d8, d40)  */
#define TM_TERMS_ALL      7u

#define TM_BC_ZERO_FLUX   0   /* psi^(1) = 0 at the boundary (inner: the paper's centre condition) */
#define TM_BC_FREE_STREAM 1   /* outer only: psi^(1) = psi^(0) of the last zone (limit eq. a22)     */
#define TM_BC_GEOMETRIC   2   /* outer only: constant luminosity through a ghost zone (eq. a62af, with
                                 R_nu squared): the ghost centre R_{I+1} = 2 R_{I+1/2} - R_I mirrors the
                                 last zone's centre across the outer edge and holds
                                 psi_{I+1} = psi_I (R_I^2 - R_nu^2/4) / (R_{I+1}^2 - R_nu^2/4), the ratio
                                 clipped to [0, 1]; the outer flux is the limited edge flux of eq. a59
                                 between zone I and the ghost, with the last zone's mean free path.
                                 Needs tm_inputs.r_nu.                                                */

#define TM_LIMITER_NONE   0   /* F = 1 (pure diffusion, eq. a21)                       */
#define TM_LIMITER_INTRP  1   /* F = F_intrp of eq. a20                                */
#define TM_LIMITER_GEOM   2   /* F = min(F_intrp, F_geom) (eqs. a23-a26a): at an edge of radius R
                                 outside the neutrinosphere of the group, F_geom = (1 + mu_nu) m / 2
                                 over lam |psi_{i+1} - psi_i| / (3 D), mu_nu = sqrt(1 - (R_nu/R)^2)
                                 (no matter velocity, no ray bending), m the floored edge mean; 1
                                 inside.  Where F_geom is the smaller, H = (1 + mu_nu) m / 2 times
                                 -sign(psi_{i+1} - psi_i) (eq. a26b).  Needs tm_inputs.r_nu.       */

#define TM_PREC_FP64  0       /* everything in float64                                 */
#define TM_PREC_MIXED 1       /* block factorisation and solve in float32; residual,
                                 update and conservation sums in float64 (Newton acts as
                                 iterative refinement)                                  */

/* per-system flags (tm_stats.flags) */
#define TM_FLAG_NOT_CONVERGED 1
#define TM_FLAG_NONFINITE     2
#define TM_FLAG_ZERO_PIVOT    4
#define TM_FLAG_PIVOT_FALLBACK 8  /* informational: re-factored with partial pivoting after the
                                     diagonal-pivot growth guard tripped (|multiplier| > 16,
                                     zero or non-finite pivot)                               */

#define TM_MAX_GROUPS 32

typedef struct {
    int32_t  n_species;   /* S >= 1                                                    */
    int32_t  n_rays;      /* R >= 1                                                    */
    int32_t  n_zones;     /* I >= 1                                                    */
    int32_t  n_groups;    /* N, 1 <= N <= TM_MAX_GROUPS                                */
    double   c_dt;        /* c * dt in cm (> 0)                                        */
    int32_t  inner_bc;    /* must be TM_BC_ZERO_FLUX                                   */
    int32_t  outer_bc;    /* TM_BC_ZERO_FLUX, TM_BC_FREE_STREAM or TM_BC_GEOMETRIC     */
    uint32_t terms;       /* TM_TERM_* bitmask                                         */
    int32_t  limiter;     /* TM_LIMITER_*                                              */
    double   psi_floor;   /* floor of the edge mean in the limiter (> 0), e.g. 1e-300  */
    int32_t  precision;   /* TM_PREC_*                                                 */
} tm_problem;

typedef struct {
    const double *r_edge;   /* edge [R][I+1], cm, strictly increasing per ray           */
    const double *e_edge;   /* [N+1] MeV, strictly increasing, > 0                      */
    const double *kappa_a;  /* cell, cm^-1, absorption inverse mean free path            */
    const double *eta;      /* cell, cm^-1, emissivity j (emission per state per length)  */
    const double *kappa_s;  /* cell, cm^-1, isoenergetic scattering (transport opacity)   */
    const double *temp;     /* zone, MeV (> 0), used by the NES detailed balance          */
    const double *nes_amp;  /* sysz, cm^-1; may be NULL when TM_TERM_NES is off          */
    const double *nes_g;    /* [N][N] symmetric shape; may be NULL when TM_TERM_NES is off */
    const double *lapse;    /* zone [R][I], lapse a_i at zone centres (> 0); NULL: a = 1       */
    const double *lapse_edge; /* edge [R][I+1], lapse at zone edges; given with lapse or not at all */
    const double *r_nu;     /* [S][N] cm, neutrinosphere radius R_nu of each species and group;
                               required by TM_LIMITER_GEOM and TM_BC_GEOMETRIC, else may be NULL */
} tm_inputs;

/* The lapse (eq. a58 with a != 1; eq. a8a).  With `lapse` set, the residual is a_i c dt times eq. a58:
 *   G_{i,k} = psi - psi^n + c dt { a_i^3 (A_{i+1/2} H_{i+1/2} / a_{i+1/2}^2 - A_{i-1/2} H_{i-1/2} / a_{i-1/2}^2) / V_i
 *                                  + a_i [ - eta (1 - psi) + kappa_a psi - S_{i,k} ] },
 * e_edge holds energies at infinity E, the groups of zone i sit at the local energies E / a_i (at which
 * the caller gives kappa_a, eta, kappa_s), and the NES kernels are evaluated at those local energies.
 * The statistics become: number sum_i V_i / a_i^3 sum_k W_k psi, energy at infinity with the same
 * weights, outer flux c A_{I+1/2} / a_{I+1/2}^2 sum_k W_k H.  tm_assemble, tm_factor_solve and
 * tm_newton_step take a lapse (the library keeps lapse-folded copies of kappa_a, eta, kappa_s, temp and
 * nes_amp: three cell arrays of workspace), and so do tm_adjoint_step (gradients with respect to the
 * caller's local-energy kappa_a, eta, kappa_s and nes_amp) and tm_luminosity_seed (the luminosity
 * c A_{I+1/2} / a_{I+1/2}^2 sum_k W_k H, whose seed is c R_{I+1/2}^2 / a_{I+1/2}^2 W_k), and
 * tm_ye_newton_step (the species rows as above with dkappa_a/dY_e and deta/dY_e at the local energies;
 * eq. a62a's rate per zone becomes c dt zeta a_i^-2 sum_k W_k (S_nue - S_nuebar), so that electrons
 * plus (V_i / a_i^3) sum_k W_k (psi_nue - psi_nuebar) are conserved, and the reported lepton number
 * takes those weights; not together with the pair processes);  tm_temperature_update returns
 * TM_ERR_INVALID_ARG when one is given. */

typedef struct {            /* every array is per system [S][R], device memory        */
    double  *res_inf;       /* max |G| at the returned psi                              */
    double  *res0_inf;      /* max |G| at the initial guess                             */
    double  *n_tot;         /* sum_i V_i sum_k W_k psi (number, constants dropped)      */
    double  *e_tot;         /* sum_i V_i sum_k W_k eps_k psi (energy)                   */
    double  *budget_n;      /* n_tot - n_tot^n + B_N - Q_N - NES_N = sum V W G (eq. a62) */
    double  *lum_n;         /* c A_{I+1/2} sum_k W_k H_{I+1/2,k} (number luminosity)      */
    int32_t *iters;         /* Newton updates applied                                   */
    int32_t *flags;         /* TM_FLAG_* bits                                           */
} tm_stats;

typedef struct tm_ctx tm_ctx;

/* Create a context for one problem shape, bound to `hip_stream` (a hipStream_t, or
 * NULL for the default stream) on the current device.  Allocates nothing on the
 * device until a call needs workspace.  *out receives the context.               */
tm_status tm_create(const tm_problem *problem, void *hip_stream, tm_ctx **out);

/* Free the context and any workspace it allocated itself.                         */
tm_status tm_destroy(tm_ctx *ctx);

/* Device bytes of workspace needed to factor `batch_systems` systems per launch
 * (0 means all S*R systems at once): (b + 15) slots of I*NT*(NT+1) values (NT = N
 * padded to a multiple of 4; float32 in TM_PREC_MIXED, else double), the 15 spare
 * slots filling a last partial wave group.  Returns 0 for an invalid problem.    */
size_t tm_workspace_bytes(const tm_problem *problem, int64_t batch_systems);

/* Hand the context caller-owned device workspace (>= tm_workspace_bytes(p, b) or
 * tm_ye_workspace_bytes(p, b) for some batch b >= 1, else TM_ERR_WORKSPACE; 256-byte
 * aligned, as device allocations are, else TM_ERR_INVALID_ARG); the context
 * then launches the factorisation in batches that fit.  A step whose own need for one
 * batch exceeds the workspace returns TM_ERR_WORKSPACE.  Without it, the context
 * allocates workspace for all systems on first use.  Pass NULL/0 to go back to
 * self-allocated workspace.                                                          */
tm_status tm_set_workspace(tm_ctx *ctx, void *device_ptr, size_t bytes);

/* Residual G(psi) (eq. a58 times c dt) into `residual` (cell).  If `blocks` is not
 * NULL it receives the exact Jacobian in block form, [S][R][I][N][N+2]: row k of
 * zone i holds the dense block A_i[k][0..N-1], then bm_{i,k}, bp_{i,k} (eq. a62ae).
 * This debug output is the only path on which a Jacobian reaches HBM.             */
tm_status tm_assemble(tm_ctx *ctx, const tm_inputs *in, const double *psi_n,
                      const double *psi, double *residual, double *blocks);

/* Solve J(psi) x = rhs (transpose = 0) or J(psi)^T x = rhs (transpose != 0) for
 * every system by block-Thomas elimination (eq. a62ae).  Each dense block is eliminated
 * with diagonal pivots (the blocks of this method are column diagonally dominant) under a
 * growth guard; a system that trips it is re-factored with partial pivoting
 * (TM_FLAG_PIVOT_FALLBACK).  The environment variable TM_PIVOT=always|never read at
 * tm_create forces partial pivoting or disables the fallback; TM_GROWTH_LIMIT sets
 * the guard (default 16).  rhs and x are cell arrays and may alias.  In TM_PREC_MIXED the
 * factorisation and solve run in float32 on the right-hand side divided by a power of two
 * near its largest magnitude in the system (so residuals below the float32 range still
 * solve); x is the float32 solution widened and scaled back.  Returns TM_ERR_SINGULAR when
 * some system meets an exactly zero pivot even with partial pivoting (its block is singular;
 * its x then holds non-finite values, the other systems are solved).                   */
tm_status tm_factor_solve(tm_ctx *ctx, const tm_inputs *in, const double *psi,
                          const double *rhs, double *x, int32_t transpose);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): tm_factor_solve with every internal buffer (grid constants,
 * per-system scalars, the factor workspace) taken from one static device array of
 * TM_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its load until the process ends.
 * Calls no hipMalloc/hipFree and no allocating library routine, clears what must start at zero with
 * kernels (no memset nodes), and never synchronises: the work is only enqueued on the context's stream.
 * The factorisation runs in batches that fit the scratch; systems that trip the diagonal-pivot guard
 * are re-factored with partial pivoting in the same enqueued sequence (TM_PIVOT=never is not honoured).
 * flags (device, [S][R] int32, may be NULL) receives the per-system TM_FLAG_ZERO_PIVOT and
 * TM_FLAG_PIVOT_FALLBACK bits; TM_ERR_SINGULAR is not returned (that would need a read-back).
 * Returns TM_ERR_WORKSPACE, before any device work, when the per-system arrays (20 bytes per system)
 * plus 16 slots of factors (I * NT * (NT+1) values each, float32 in TM_PREC_MIXED, else double)
 * exceed the scratch; TM_ERR_INVALID_ARG as tm_factor_solve, and for a lapse (not supported here).
 * Every call on one GPU shares that GPU's scratch array: calls that overlap in time on one GPU (two
 * streams, two contexts, two threads) race and give wrong results.                          */
#define TM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
tm_status tm_factor_solve_noalloc(tm_ctx *ctx, const tm_inputs *in, const double *psi,
                                  const double *rhs, double *x, int32_t transpose, int32_t *flags);

/* Backward-Euler Newton iteration (eq. a62aa) for psi^{n+1} of every system.
 * psi holds the initial guess on entry (usually a copy of psi_n) and psi^{n+1} on
 * return.  Per system, an update J delta = -G is applied while
 *   max|G(psi)| > max(rtol * max|G(psi_initial)|, g_round)
 * and fewer than max_iter updates have been made, where g_round = 32 * 2^-52 * the
 * largest sum over a cell of the magnitudes of the terms of G (the level below which
 * G itself is rounding).  rtol = 0 runs exactly max_iter updates (unless G is exactly
 * zero).  In TM_PREC_MIXED each update is an FP32 solve of the FP64 residual, so the
 * iteration is iterative refinement to the same stopping rule.  `stats` (all pointers
 * device, may be NULL as a whole) receives the per-system results at the returned
 * psi.  Returns TM_OK, or the worst of TM_ERR_NONFINITE, TM_ERR_SINGULAR,
 * TM_ERR_NOT_CONVERGED over systems (per-system detail in stats.flags).           */
tm_status tm_newton_step(tm_ctx *ctx, const tm_inputs *in, const double *psi_n,
                         double *psi, int32_t max_iter, double rtol, tm_stats *stats);

/* Adjoint of the converged step.  Solves J(psi_np1)^T mu = seed (seed = dJ/dpsi^{n+1})
 * and returns the vector-Jacobian products of the objective through the solution:
 *   g_theta = -mu^T dG/dtheta  for theta in {kappa_a, eta, kappa_s, nes_amp},
 *   mu itself is dJ/dpsi^n (dG/dpsi^n = -1).
 * Every gradient pointer may be NULL to skip it; mu must not be NULL.  Always FP64.
 * Returns TM_ERR_SINGULAR as tm_factor_solve does (mu and the gradients of such a system
 * are then non-finite).                                                            */
tm_status tm_adjoint_step(tm_ctx *ctx, const tm_inputs *in, const double *psi_n,
                          const double *psi_np1, const double *seed, double *mu,
                          double *g_kappa_a, double *g_eta, double *g_kappa_s,
                          double *g_nes_amp);

/* Seed of the adjoint for the outer-boundary number luminosity
 *   L_N = c A_{I+1/2} sum_k W_k H_{I+1/2,k}   (number through the outer surface, eq. a62)
 * written as a cell array: seed = dL_N/dpsi + add, where dL_N/dpsi = c R_{I+1/2}^2 W_k in
 * the outermost zone and zero elsewhere (zero everywhere without an outgoing flux); with a lapse
 * the area is R_{I+1/2}^2 / a_{I+1/2}^2 (lapse_edge is then read).
 * `add` (cell array) may be NULL or alias `seed`; a multi-step adjoint passes the adjoint of
 * the following step there.  Needs r_edge and e_edge only (and lapse_edge with a lapse).  With TM_BC_GEOMETRIC the outer
 * flux depends on psi_I through the limited flux to the ghost zone, so its derivative needs
 * the state: this entry point then returns TM_ERR_INVALID_ARG.                        */
tm_status tm_luminosity_seed(tm_ctx *ctx, const tm_inputs *in, const double *add, double *seed);

/* ---------------------------------------------------------------------------------
 * Y_e-coupled step (eq. a62a with the linearised system of eqs. a62ac-a62ae; matter
 * energy and temperature of eqs. a62b, a62d).
 *
 * Electron neutrinos (species 0) and antineutrinos (species 1) of a ray exchange
 * lepton number with the matter through emission and absorption, so Y_e of every zone
 * is advanced implicitly with them:
 *   G_Y,i = Y_e,i - Y_e,i^n + c dt zeta_i sum_k W_k (S_0,ik - S_1,ik),
 *   zeta_i = 4 pi m_B / ((hc)^3 rho_i),  S_q = eta_q(Y_e) (1 - psi_q) - kappa_a,q(Y_e) psi_q,
 * with m_B the atomic mass unit (1.66053906660e-24 g) and hc = 1.23984198e-10 MeV cm.
 * Over the step the absorption and emission opacities of the pair are linear in Y_e,
 * kappa_a,q(Y_e) = kappa_a,q + (Y_e - Y_e^n) dkappa_a,q/dY_e and likewise for eta; the
 * species residuals use them in their emission/absorption term, while the transport mean
 * free path (diffusion) stays at the opacities of Y_e^n.  NES does not depend on Y_e.
 * The linearised system is block tridiagonal with (2N+1)-square diagonal blocks (psi of
 * both species and Y_e of a zone) and diagonal off-diagonal blocks whose Y_e entries are
 * zero; it is eliminated by block-Thomas with partial pivoting inside each block.
 * Species 2..S-1 are independent of Y_e and are advanced by tm_newton_step on a problem
 * of their own (their arrays are the tail of the cell, sysz arrays).
 * --------------------------------------------------------------------------------- */

typedef struct {
    const double *rho;       /* zone [R][I], g cm^-3 (> 0)                                  */
    const double *ye_n;      /* zone [R][I], Y_e at time level n                             */
    const double *dka_dye;   /* [2][R][I][N] cm^-1: dkappa_a/dY_e of species 0 and 1; may be
                                NULL when TM_TERM_EMABS is off                              */
    const double *deta_dye;  /* [2][R][I][N] cm^-1: deta/dY_e; NULL as dka_dye              */
    /* Pair creation and annihilation of species 0 and 1 (eqs. d11-d22), optional: NULL
     * pair_amp turns them off.  Zeroth-moment sources (Phi_0 terms of eq. d14)
     *   S_0,k = (1 - psi_k) sum_k' Q^p_kk' (1 - pbar_k') - psi_k sum_k' Q^a_kk' chi_kk' pbar_k'
     * and the same with the species exchanged, Q^a_kk' = a_i g_kk' W_k' / Wbar (Wbar the mean
     * of W), Q^p = exp(-(eps_k + eps_k')/T_i) Q^a (eq. d12), chi = min(chi_1, chi_2) with
     * chi_1 = 1 - (3/2) eta_k eta'_k' (the ratio that defines eq. d16, for the flux factors
     * eta = psi1/psi0 given here) and chi_2 of eq. d19 from the cosines of eq. d22 at the zone
     * centre (R_nu from tm_inputs.r_nu, which is then required).  The sources join the species
     * residuals (minus c dt S), the coupled Jacobian (cross-species blocks) and the
     * temperature update's collision energy.                                            */
    const double *pair_amp;  /* zone [R][I] cm^-1, kernel amplitude a_i, or NULL           */
    const double *pair_g;    /* [N][N] symmetric kernel shape g                             */
    const double *pair_eta1; /* [2][R][I][N] flux factors psi1/psi0 of species 0 and 1      */
} tm_ye_inputs;

typedef struct {             /* every array is per ray [R], device memory                  */
    double  *res_inf;        /* max |G| over both species and Y_e at the returned state      */
    double  *res0_inf;       /* the same at the initial guess                                */
    double  *lepton;         /* total lepton number of the ray divided by 4 pi:
                                sum_i V_i [rho_i Y_e,i / m_B + (4 pi/(hc)^3) sum_k W_k
                                (psi_0 - psi_1)] at the returned state (may be NULL)         */
    int32_t *iters;          /* Newton updates applied                                      */
    int32_t *flags;          /* TM_FLAG_* bits (TM_FLAG_ZERO_PIVOT: a zero pivot met)          */
} tm_ye_stats;

/* Device bytes of workspace needed to factor `batch_rays` coupled systems per launch
 * (0 means all R): b slots of I*((2NT+1)^2 + 1) doubles (NT = N padded to a multiple of
 * 4; per zone C, y and one pad double).
 * Returns 0 for an invalid problem or N > 28.  A workspace given with
 * tm_set_workspace serves both steps; the coupled step then runs in batches of
 * floor(bytes / slot) rays.                                                          */
size_t tm_ye_workspace_bytes(const tm_problem *problem, int64_t batch_rays);

/* Backward-Euler Newton iteration for psi^{n+1} of species 0 and 1 together with
 * Y_e^{n+1}, per ray.  Needs S >= 2, N <= 28 and TM_PREC_FP64 (the coupled elimination
 * is FP64 only).  psi (cell array of the whole problem; only species 0 and 1 are read
 * and written) and ye (zone [R][I]) hold the initial guess on entry, usually psi_n and
 * ye_n, and the new state on return.  The stopping rule and line search are those of
 * tm_newton_step applied to the coupled system: max|G| is over both species and Y_e,
 * and the rounding level is the larger of the two species' levels and 32 * 2^-52 times
 * the largest per-zone sum of the magnitudes of the terms of G_Y (emission and absorption
 * counted separately) plus |Y_e| |dG_Y/dY_e|.  Synchronises the stream.  Returns as
 * tm_newton_step; `stats` may be NULL.                                                */
tm_status tm_ye_newton_step(tm_ctx *ctx, const tm_inputs *in, const tm_ye_inputs *yin,
                            const double *psi_n, double *psi, double *ye, int32_t max_iter,
                            double rtol, tm_ye_stats *stats);

/* Matter energy change and temperature after the step, per zone:
 *   de_i = -(4 pi/(hc)^3) (m_B/rho_i) sum_q w_q c dt sum_k eps_k W_k S_q,ik   (eq. a62b)
 *   T_i^{n+1} = T_i^n + (de_i - (Y_e,i - Y_e,i^n) de/dY_e) / (de/dT)            (eq. a62d)
 * de in MeV per baryon; S_q is the collision source of species q at psi (emission and
 * absorption, with the opacities at ye for species 0 and 1, and NES; isoenergetic
 * scattering exchanges no energy).  T^n is in->temp.  psi: cell array of all S species
 * after the step; ye: zone, after the step.  stat_weights: HOST array of S statistical
 * weights (e.g. 1, 1, 2, 2 when species 2 and 3 each stand for two flavours); S <= 16.
 * de_dT (MeV per baryon per MeV) and de_dye (MeV per baryon): zone arrays of the
 * matter's internal-energy derivatives.  de_out (zone) may be NULL; temp_out (zone) may
 * alias in->temp (each zone reads its own T^n before writing).  Asynchronous.       */
tm_status tm_temperature_update(tm_ctx *ctx, const tm_inputs *in, const tm_ye_inputs *yin,
                                const double *psi, const double *ye, const double *stat_weights,
                                const double *de_dT, const double *de_dye, double *de_out,
                                double *temp_out);

/* ---------------------------------------------------------------------------------
 * Energy advection (eqs. a78-a81d) and the remap after a change of the lapse (eqs. p1-p8).
 *
 * Per (species, ray, zone), over the N groups of the shared energy grid e_edge (in->e_edge):
 *  1. Lagrangian energy step (TM_EADV_LAGRANGIAN, eqs. a78-a80): every group edge E_m moves to
 *       E'_m = [1 + (a^{n+1}/a^n - 1 - dR/R) - (db/b - dR/R) eta2_m] E_m            (eq. a79)
 *     with eta2_m the scalar Eddington factor at the edge (mean of the two adjacent groups, the end
 *     edges the end group's value, 1/3 when `eddington` is NULL), and the number per unit mass is
 *     kept: psi'_k W'_k = (rho a^3)^{n+1} / (rho a^3)^n psi_k W_k                    (eq. a78).
 *     Lapse change (TM_EADV_LAPSE, eqs. p1, p2): the local grid E/a moves from E/a^n to E/a^{n+1}
 *     and psi_k W_k(E/a^n) neutrinos sit in group k.
 *  2. Remap onto the fixed grid (eq. a81; eqs. p5-p8): the number per unit energy (proportional to
 *     eps^2 psi) is given a piecewise parabolic profile on the displaced grid (eqs. h9-h24 in
 *     their planar form; two ghost groups at each end repeat the end group; each group's edge
 *     values adjusted so that its parabola has no interior extremum), and through each
 *     interior edge passes the number between the displaced and the fixed edge (eqs. h60, h61);
 *     no number passes the two outer edges.  The fluxes are scaled by
 *       xi = (E_before - sum_k N_k eps_k) / sum_k (F_{k-1/2} - F_{k+1/2}) eps_k       (eq. p8)
 *     (1 when the denominator is 0), which keeps the energy as well as the number (eq. p6).
 *  3. Over-fill limiter (eqs. a81a-a81d): from the lowest group while groups k+1 and k+2 exist, an
 *     excess psi_k - 1 > 0 is removed and added to group k+1 and removed from group k+2 so that
 *     number and energy are kept; a removal larger than psi_{k+2} is scaled down so that
 *     psi_{k+2} becomes 0 (the paper's approximate case, flagged).
 * psi (cell, in place) holds psi^n on entry and the new psi on return.  A zone whose swept region at
 * some edge is wider than the group it comes from, or whose displaced grid is not increasing, is
 * left unchanged and flagged.  Asynchronous; no workspace.
 * --------------------------------------------------------------------------------- */

#define TM_EADV_LAGRANGIAN 0
#define TM_EADV_LAPSE      1

#define TM_EADV_FLAG_DISPLACEMENT  1   /* displacement beyond a group: zone left unchanged      */
#define TM_EADV_FLAG_OVERFILL      2   /* the over-fill limiter moved neutrinos                 */
#define TM_EADV_FLAG_OVERFILL_CLAMP 4  /* ... and hit the psi_{k+2} >= 0 bound (approximate)     */

typedef struct {
    int32_t mode;               /* TM_EADV_LAGRANGIAN or TM_EADV_LAPSE                          */
    const double *rho_old;      /* zone [R][I] g cm^-3 before and after the hydro step; both or   */
    const double *rho_new;      /*   neither (NULL: no change); Lagrangian mode only              */
    const double *lapse_old;    /* zone [R][I] lapse a^n and a^{n+1} (> 0); both or neither (NULL: */
    const double *lapse_new;    /*   a = 1); required in the lapse mode                           */
    const double *dlnR;         /* zone [R][I]: dR/R and db/b of the hydro step (NULL: 0);         */
    const double *dlnb;         /*   Lagrangian mode only                                         */
    const double *eddington;    /* cell: scalar Eddington factor psi^(2)/psi^(0) (NULL: 1/3);     */
                                /*   Lagrangian mode only                                         */
} tm_eadv_inputs;

/* Apply the energy-advection update to psi (cell, in place).  Needs in->e_edge only.  xi (sysz
 * [S][R][I], may be NULL) receives the flux scale of eq. p8 (1 where nothing moved or the zone was
 * left unchanged); flags (sysz, may be NULL) the TM_EADV_FLAG_* bits of each zone.  Returns
 * TM_ERR_INVALID_ARG for a missing pointer, an unknown mode or half of an input pair.           */
tm_status tm_energy_advect(tm_ctx *ctx, const tm_inputs *in, const tm_eadv_inputs *ea, double *psi,
                           double *xi, int32_t *flags);

/* Kernel timing, a measurement aid (not an operation of the method): for benchmarks that relate the
 * diagonal-pivot factor kernel to its roofline.  With timing enabled, tm_factor_solve and tm_newton_step
 * bracket their diagonal-pivot factor launch(es) (all batches, nothing else in between) with two HIP
 * events on the context's stream.  tm_kernel_time_ms waits for the second event of the last bracketed
 * call and writes the elapsed milliseconds to *ms (host pointer); TM_ERR_INVALID_ARG when timing is off,
 * ms is NULL or no call has been bracketed since it was enabled.  Enabling creates the two events (once
 * per context; released by tm_destroy); disabling keeps them.                                          */
tm_status tm_set_kernel_timing(tm_ctx *ctx, int32_t enable);
tm_status tm_kernel_time_ms(tm_ctx *ctx, double *ms);

/* Human-readable name of a status code (static storage).                          */
const char *tm_status_string(tm_status status);

/* Last error message recorded on the context (empty string when none).            */
const char *tm_last_error(const tm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
