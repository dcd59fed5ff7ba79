// Host side of the libtm C ABI (include/tm.h): argument validation, workspace,
// launch sequencing of the Newton iteration and the adjoint, status reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tm.h"
#include "tm_kernels.hpp"

struct tm_ctx {
    tm_problem p;
    hipStream_t stream;
    int device;
    std::string err;
    // workspace (factors), either caller-owned or allocated here
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    int ws_kind = 0;            // self-allocated for: 0 the single-species factor, 1 the coupled factor
    // small internal device buffers
    tmk::Consts* consts = nullptr;
    double* res = nullptr;      // [nsys]
    double* res0 = nullptr;     // [nsys]
    int* active = nullptr;      // [nsys]
    int* iters = nullptr;       // [nsys]
    int* flags = nullptr;       // [nsys]
    int* count = nullptr;       // [1]
    double* gbuf = nullptr;     // [cells] residual for the Newton right-hand side
    int* h_count = nullptr;     // pinned host
    int* guard = nullptr;       // [nsys] growth guard of the last diagonal-pivot launch
    double* res_acc = nullptr;  // [nsys] Newton line search: accepted residual
    double* tgt = nullptr;      // [nsys] stopping target at the accepted iterate
    double* alpha = nullptr;    // [nsys] step length of the pending trial
    int* pending = nullptr;     // [nsys] trial under evaluation
    int* backtrack = nullptr;   // [nsys] trial rejected
    double* dbuf = nullptr;     // [cells] Newton update delta (for backtracking)
    int* redo = nullptr;        // [nsys] systems re-factored with partial pivoting
    // pivoting policy: 0 diagonal pivots with guarded fallback to partial pivoting (default),
    // 1 always partial pivoting, 2 diagonal pivots only (guard trips become failures)
    int pivot_policy = 0;
    int factor_kernel = tmk::kFactorQuadMfma;   // float32 diagonal-pivot solve: TM_FACTOR_KERNEL=window|bf16x3|bf16|mfma|valu|lane
    double growth_limit = 16.0;
    long long pivot_fallbacks = 0;   // systems re-factored with partial pivoting since creation
    // kernel timing (measurement aid): events around the diagonal-pivot factor launches
    hipEvent_t kt[2] = {nullptr, nullptr};
    bool timing = false;
    bool timed = false;                 // an enabled call has recorded both events
    // Y_e-coupled step, per ray [R] unless stated (allocated on first use)
    double* y_res = nullptr;
    double* y_res0 = nullptr;
    double* y_res_acc = nullptr;
    double* y_tgt = nullptr;
    double* y_alpha = nullptr;
    double* y_res_sp = nullptr;  // [2R] max|G| of the species part (written by the residual pass)
    double* y_lev = nullptr;     // [2R] rounding level of the species part
    double* y_gy = nullptr;      // [R][I] Y_e residual
    double* y_dy = nullptr;      // [R][I] Y_e update
    int* y_active = nullptr;
    int* y_iters = nullptr;
    int* y_flags = nullptr;
    int* y_pending = nullptr;
    int* y_backtrack = nullptr;
    int* y_redo = nullptr;       // rays of the tiled diagonal-pivot launch sent to partial pivoting
    // inputs with the lapse folded in (allocated on first use with a lapse)
    double* lp_ka = nullptr;
    double* lp_et = nullptr;
    double* lp_ks = nullptr;
    double* lp_temp = nullptr;   // [R][I]
    double* lp_amp = nullptr;    // [S][R][I]
};

namespace {

long long n_systems(const tm_problem& p) { return (long long)p.n_species * p.n_rays; }
long long n_cells(const tm_problem& p) { return n_systems(p) * p.n_zones * p.n_groups; }

bool valid_problem(const tm_problem* p, std::string* why) {
    auto fail = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (!p) return fail("problem is NULL");
    if (p->n_species < 1 || p->n_rays < 1 || p->n_zones < 1) return fail("S, R and I must be >= 1");
    if (p->n_groups < 1 || p->n_groups > TM_MAX_GROUPS) return fail("N must be in [1, 32]");
    if (!(p->c_dt > 0.0) || !std::isfinite(p->c_dt)) return fail("c_dt must be finite and > 0");
    if (p->inner_bc != TM_BC_ZERO_FLUX) return fail("inner_bc must be TM_BC_ZERO_FLUX");
    if (p->outer_bc != TM_BC_ZERO_FLUX && p->outer_bc != TM_BC_FREE_STREAM && p->outer_bc != TM_BC_GEOMETRIC)
        return fail("bad outer_bc");
    if (p->terms & ~TM_TERMS_ALL) return fail("unknown bit in terms");
    if (p->limiter != TM_LIMITER_NONE && p->limiter != TM_LIMITER_INTRP && p->limiter != TM_LIMITER_GEOM)
        return fail("bad limiter");
    if (!(p->psi_floor > 0.0)) return fail("psi_floor must be > 0");
    if (p->precision != TM_PREC_FP64 && p->precision != TM_PREC_MIXED) return fail("bad precision");
    if (n_systems(*p) > 0x7fffffffLL) return fail("too many systems");
    return true;
}

tmk::Shape shape_of(const tm_problem& p) {
    tmk::Shape s;
    s.S = p.n_species;
    s.R = p.n_rays;
    s.I = p.n_zones;
    s.N = p.n_groups;
    s.c_dt = p.c_dt;
    s.outer_bc = p.outer_bc;
    s.terms = p.terms;
    s.limiter = p.limiter;
    s.psi_floor = p.psi_floor;
    return s;
}

tmk::Fields fields_of(const tm_inputs& in) {
    tmk::Fields f;
    f.r_edge = in.r_edge;
    f.kappa_a = in.kappa_a;
    f.eta = in.eta;
    f.kappa_s = in.kappa_s;
    f.temp = in.temp;
    f.nes_amp = in.nes_amp;
    f.lapse = in.lapse;
    f.lapse_edge = in.lapse_edge;
    f.r_nu = in.r_nu;
    return f;
}

tm_status set_err(tm_ctx* c, tm_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

tm_status hip_check(tm_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return TM_OK;
    return set_err(c, TM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define TM_TRY(expr)                        \
    do {                                    \
        tm_status _s = (expr);              \
        if (_s != TM_OK) return _s;         \
    } while (0)

tm_status check_inputs(tm_ctx* c, const tm_inputs* in, bool need_opacity = true) {
    if (!in) return set_err(c, TM_ERR_INVALID_ARG, "inputs is NULL");
    if (!in->r_edge || !in->e_edge) return set_err(c, TM_ERR_INVALID_ARG, "r_edge and e_edge are required");
    if (need_opacity && (!in->kappa_a || !in->eta || !in->kappa_s))
        return set_err(c, TM_ERR_INVALID_ARG, "kappa_a, eta and kappa_s are required");
    if ((c->p.terms & TM_TERM_NES) && (!in->nes_amp || !in->nes_g || !in->temp))
        return set_err(c, TM_ERR_INVALID_ARG, "nes_amp, nes_g and temp are required when TM_TERM_NES is on");
    if (!in->lapse != !in->lapse_edge) return set_err(c, TM_ERR_INVALID_ARG, "lapse and lapse_edge go together");
    if ((c->p.limiter == TM_LIMITER_GEOM || c->p.outer_bc == TM_BC_GEOMETRIC) && !in->r_nu)
        return set_err(c, TM_ERR_INVALID_ARG, "r_nu is required by TM_LIMITER_GEOM and TM_BC_GEOMETRIC");
    return TM_OK;
}

tm_status no_lapse(tm_ctx* c, const tm_inputs* in, const char* what) {
    if (in && in->lapse) return set_err(c, TM_ERR_INVALID_ARG, std::string(what) + " takes no lapse (lapse must be NULL)");
    return TM_OK;
}

// Inputs with the lapse's source factor folded in (see k_lapse_fold); `out` is `*in` without a lapse.
tm_status fold_lapse(tm_ctx* c, const tm_inputs* in, tm_inputs* out) {
    *out = *in;
    if (!in->lapse) return TM_OK;
    const size_t cells = (size_t)n_cells(c->p) * sizeof(double);
    const size_t zones = (size_t)c->p.n_rays * c->p.n_zones * sizeof(double);
    const size_t sysz = (size_t)n_systems(c->p) * c->p.n_zones * sizeof(double);
    TM_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    for (double** p : {&c->lp_ka, &c->lp_et, &c->lp_ks})
        if (!*p) TM_TRY(hip_check(c, hipMalloc((void**)p, cells), "hipMalloc lapse-folded inputs"));
    if (!c->lp_temp) TM_TRY(hip_check(c, hipMalloc((void**)&c->lp_temp, zones), "hipMalloc lapse-folded inputs"));
    if (!c->lp_amp) TM_TRY(hip_check(c, hipMalloc((void**)&c->lp_amp, sysz), "hipMalloc lapse-folded inputs"));
    TM_TRY(hip_check(c, tmk::launch_lapse_fold(shape_of(c->p), in->lapse, in->kappa_a, in->eta, in->kappa_s, in->temp,
                                               in->nes_amp, c->lp_ka, c->lp_et, c->lp_ks, c->lp_temp, c->lp_amp,
                                               c->stream), "lapse folding kernel"));
    out->kappa_a = c->lp_ka;
    out->eta = c->lp_et;
    out->kappa_s = c->lp_ks;
    if (in->temp) out->temp = c->lp_temp;
    if (in->nes_amp) out->nes_amp = c->lp_amp;
    return TM_OK;
}

// Internal per-context buffers that do not depend on the factor workspace.
tm_status ensure_small(tm_ctx* c) {
    if (c->consts) return TM_OK;
    const long long ns = n_systems(c->p);
    TM_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->consts, sizeof(tmk::Consts)), "hipMalloc consts"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->res, ns * sizeof(double)), "hipMalloc res"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->res0, ns * sizeof(double)), "hipMalloc res0"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->active, ns * sizeof(int)), "hipMalloc active"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->iters, ns * sizeof(int)), "hipMalloc iters"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->flags, ns * sizeof(int)), "hipMalloc flags"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->count, sizeof(int)), "hipMalloc count"));
    TM_TRY(hip_check(c, hipHostMalloc((void**)&c->h_count, sizeof(int)), "hipHostMalloc"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->guard, ns * sizeof(int)), "hipMalloc guard"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->redo, ns * sizeof(int)), "hipMalloc redo"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->res_acc, ns * sizeof(double)), "hipMalloc res_acc"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->tgt, ns * sizeof(double)), "hipMalloc tgt"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->alpha, ns * sizeof(double)), "hipMalloc alpha"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->pending, ns * sizeof(int)), "hipMalloc pending"));
    TM_TRY(hip_check(c, hipMalloc((void**)&c->backtrack, ns * sizeof(int)), "hipMalloc backtrack"));
    return TM_OK;
}

tm_status ensure_gbuf(tm_ctx* c) {
    if (!c->gbuf)
        TM_TRY(hip_check(c, hipMalloc((void**)&c->gbuf, n_cells(c->p) * sizeof(double)), "hipMalloc residual buffer"));
    if (!c->dbuf)
        TM_TRY(hip_check(c, hipMalloc((void**)&c->dbuf, n_cells(c->p) * sizeof(double)), "hipMalloc update buffer"));
    return TM_OK;
}

// Systems per factor launch that fit the workspace; allocates all-systems workspace if none.
tm_status factor_batch(tm_ctx* c, bool fp32, long long* batch) {
    const size_t per = tmk::factor_ws_bytes_per_system(c->p.n_zones, c->p.n_groups, fp32);
    const long long ns = n_systems(c->p);
    if (c->ws && c->ws_owned && c->ws_kind != 0) {     // sized for the coupled step: size it again
        TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
        (void)hipFree(c->ws);
        c->ws = nullptr;
    }
    if (!c->ws) {
        // self-allocate: all systems if they fit in 70% of free memory, else the largest power-of-two share
        size_t freeb = 0, totalb = 0;
        TM_TRY(hip_check(c, hipMemGetInfo(&freeb, &totalb), "hipMemGetInfo"));
        long long b = ns;
        while (b > 1 && (double)(b + tmk::kWsPadSystems) * per > 0.7 * (double)freeb) b = (b + 1) / 2;
        const size_t bytes = (size_t)(b + tmk::kWsPadSystems) * per;
        hipError_t e = hipMalloc(&c->ws, bytes);
        if (e != hipSuccess) {
            c->ws = nullptr;
            return set_err(c, TM_ERR_WORKSPACE, std::string("workspace allocation failed: ") + hipGetErrorString(e));
        }
        c->ws_bytes = bytes;
        c->ws_owned = true;
        c->ws_kind = 0;
    }
    long long b = (long long)(c->ws_bytes / per) - tmk::kWsPadSystems;
    if (b < 1) return set_err(c, TM_ERR_WORKSPACE, "workspace smaller than one system's factors");
    *batch = std::min(b, ns);
    return TM_OK;
}

tm_status ensure_ye(tm_ctx* c) {
    if (c->y_res) return TM_OK;
    const size_t R = c->p.n_rays, RI = (size_t)c->p.n_rays * c->p.n_zones;
    auto dal = [&](double** p, size_t n, const char* what) { return hip_check(c, hipMalloc((void**)p, n * sizeof(double)), what); };
    auto ial = [&](int** p, size_t n, const char* what) { return hip_check(c, hipMalloc((void**)p, n * sizeof(int)), what); };
    TM_TRY(dal(&c->y_res, R, "hipMalloc y_res"));
    TM_TRY(dal(&c->y_res0, R, "hipMalloc y_res0"));
    TM_TRY(dal(&c->y_res_acc, R, "hipMalloc y_res_acc"));
    TM_TRY(dal(&c->y_tgt, R, "hipMalloc y_tgt"));
    TM_TRY(dal(&c->y_alpha, R, "hipMalloc y_alpha"));
    TM_TRY(dal(&c->y_res_sp, 2 * R, "hipMalloc y_res_sp"));
    TM_TRY(dal(&c->y_lev, 2 * R, "hipMalloc y_lev"));
    TM_TRY(dal(&c->y_gy, RI, "hipMalloc y_gy"));
    TM_TRY(dal(&c->y_dy, RI, "hipMalloc y_dy"));
    TM_TRY(ial(&c->y_active, R, "hipMalloc y_active"));
    TM_TRY(ial(&c->y_iters, R, "hipMalloc y_iters"));
    TM_TRY(ial(&c->y_flags, R, "hipMalloc y_flags"));
    TM_TRY(ial(&c->y_pending, R, "hipMalloc y_pending"));
    TM_TRY(ial(&c->y_backtrack, R, "hipMalloc y_backtrack"));
    TM_TRY(ial(&c->y_redo, R, "hipMalloc y_redo"));
    return TM_OK;
}

// Rays per coupled factor launch that fit the workspace; allocates workspace for all rays if none.
tm_status ye_batch(tm_ctx* c, long long* batch) {
    const size_t per = tmk::ye_ws_bytes_per_ray(c->p.n_zones, c->p.n_groups);
    const long long R = c->p.n_rays;
    if (c->ws && c->ws_owned && c->ws_kind != 1) {     // sized for the single-species step: size it again
        TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
        (void)hipFree(c->ws);
        c->ws = nullptr;
    }
    if (!c->ws) {
        size_t freeb = 0, totalb = 0;
        TM_TRY(hip_check(c, hipMemGetInfo(&freeb, &totalb), "hipMemGetInfo"));
        long long b = R;
        while (b > 1 && (double)b * per > 0.7 * (double)freeb) b = (b + 1) / 2;
        hipError_t e = hipMalloc(&c->ws, (size_t)b * per);
        if (e != hipSuccess) {
            c->ws = nullptr;
            return set_err(c, TM_ERR_WORKSPACE, std::string("workspace allocation failed: ") + hipGetErrorString(e));
        }
        c->ws_bytes = (size_t)b * per;
        c->ws_owned = true;
        c->ws_kind = 1;
    }
    const long long b = (long long)(c->ws_bytes / per);
    if (b < 1) return set_err(c, TM_ERR_WORKSPACE, "workspace smaller than one ray's coupled factors");
    *batch = std::min(b, R);
    return TM_OK;
}

tm_status check_ye_inputs(tm_ctx* c, const tm_ye_inputs* y) {
    if (!y) return set_err(c, TM_ERR_INVALID_ARG, "Y_e inputs are NULL");
    if (!y->rho || !y->ye_n) return set_err(c, TM_ERR_INVALID_ARG, "rho and ye_n are required");
    if ((c->p.terms & TM_TERM_EMABS) && (!y->dka_dye || !y->deta_dye))
        return set_err(c, TM_ERR_INVALID_ARG, "dka_dye and deta_dye are required when TM_TERM_EMABS is on");
    if (c->p.n_species < 2) return set_err(c, TM_ERR_INVALID_ARG, "the Y_e coupling needs species 0 and 1 (S >= 2)");
    if (c->p.n_groups > tmk::kYeMaxGroups) return set_err(c, TM_ERR_INVALID_ARG, "the Y_e-coupled step needs N <= 28");
    if (y->pair_amp && (!y->pair_g || !y->pair_eta1))
        return set_err(c, TM_ERR_INVALID_ARG, "pair_amp needs pair_g and pair_eta1");
    return TM_OK;
}

tmk::YeFields ye_fields_of(const tm_ye_inputs& y) {
    tmk::YeFields f;
    f.rho = y.rho;
    f.ye_n = y.ye_n;
    f.dka = y.dka_dye;
    f.deta = y.deta_dye;
    f.pair_amp = y.pair_amp;
    f.pair_g = y.pair_g;
    f.pair_eta1 = y.pair_eta1;
    return f;
}

tm_status run_factor(tm_ctx* c, const tm_inputs* in, const double* psi, const double* rhs, double rhs_sign,
                     double* x, double* psi_out, const int* active, bool fp32, bool transpose,
                     double* dx = nullptr, const double* rhs_max = nullptr) {
    long long batch = 0;
    TM_TRY(factor_batch(c, fp32, &batch));
    const int NT = tmk::padded_groups(c->p.n_groups);
    const size_t es = fp32 ? 4 : 8;
    tmk::FactorArgs a;
    a.sh = shape_of(c->p);
    a.f = fields_of(*in);
    a.cs = c->consts;
    a.psi = psi;
    a.rhs = rhs;
    a.rhs_sign = rhs_sign;
    a.rhs_max = fp32 ? rhs_max : nullptr;
    a.x = x;
    a.psi_out = psi_out;
    a.active = active;
    a.flags = c->flags;
    a.iters = psi_out ? c->iters : nullptr;
    a.guard = c->guard;
    a.growth_limit = c->growth_limit;
    a.dx = psi_out ? dx : nullptr;
    a.pending = psi_out ? c->pending : nullptr;
    a.alpha = psi_out ? c->alpha : nullptr;
    a.wsC = c->ws;
    a.wsY = (char*)c->ws + (size_t)(batch + tmk::kWsPadSystems) * c->p.n_zones * NT * NT * es;
    const long long ns = n_systems(c->p);
    const bool pivot_first = c->pivot_policy == 1;
    if (!pivot_first)
        TM_TRY(hip_check(c, hipMemsetAsync(c->guard, 0, ns * sizeof(int), c->stream), "memset guard"));
    if (c->timing) TM_TRY(hip_check(c, hipEventRecord(c->kt[0], c->stream), "timing event"));
    for (long long s0 = 0; s0 < ns; s0 += batch) {
        a.sys0 = s0;
        a.nsys = std::min(batch, ns - s0);
        TM_TRY(hip_check(c, tmk::launch_factor(a, fp32, transpose, pivot_first, c->stream, c->factor_kernel), "factor kernel"));
    }
    if (c->timing) {
        TM_TRY(hip_check(c, hipEventRecord(c->kt[1], c->stream), "timing event"));
        c->timed = true;
    }
    if (pivot_first) return TM_OK;
    // systems whose diagonal-pivot elimination tripped the growth guard were left untouched:
    // re-factor exactly those with partial pivoting
    TM_TRY(hip_check(c, tmk::launch_mark(c->guard, ns, c->redo, c->count, c->stream), "mark kernel"));
    TM_TRY(hip_check(c, hipMemcpyAsync(c->h_count, c->count, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                     "copy count"));
    TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
    const int nredo = *c->h_count;
    if (nredo == 0) return TM_OK;
    c->pivot_fallbacks += nredo;
    if (c->pivot_policy == 2) return set_err(c, TM_ERR_SINGULAR, "diagonal-pivot growth guard tripped");
    a.active = c->redo;
    for (long long s0 = 0; s0 < ns; s0 += batch) {
        a.sys0 = s0;
        a.nsys = std::min(batch, ns - s0);
        TM_TRY(hip_check(c, tmk::launch_factor(a, fp32, transpose, true, c->stream), "pivoting factor kernel"));
    }
    return TM_OK;
}

// TM_ERR_SINGULAR when some system of the last factorisation met an exactly zero pivot (with partial
// pivoting, so the block is singular): its solution holds non-finite values.  Synchronises the stream.
tm_status check_zero_pivots(tm_ctx* c) {
    TM_TRY(hip_check(c, tmk::launch_count_bits(c->flags, n_systems(c->p), TM_FLAG_ZERO_PIVOT, c->count, c->stream),
                     "count kernel"));
    TM_TRY(hip_check(c, hipMemcpyAsync(c->h_count, c->count, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                     "copy count"));
    TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
    if (*c->h_count > 0)
        return set_err(c, TM_ERR_SINGULAR, std::to_string(*c->h_count) + " system(s) with an exactly zero pivot");
    c->err.clear();
    return TM_OK;
}

// ---------------------------------------------------------------- allocation-free solve
// One scratch array per device for tm_factor_solve_noalloc: grid constants, per-system scalars and the
// factor workspace.  In host code `scratch` names a host-side stand-in, so kernels get the device
// address taken once per device with hipGetSymbolAddress (each device holds its own copy).
constexpr size_t kScratchBytes = TM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up on the device's first call).
tm_status scratch_of(tm_ctx* c, unsigned char** out) {
    if (c->device < 0 || c->device >= kMaxDevices) return set_err(c, TM_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        TM_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
        void* ptr = nullptr;
        TM_TRY(hip_check(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
        if (!ptr) return set_err(c, TM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[c->device] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[c->device]);
    return TM_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Layout of the scratch array for a problem; factor slots are what remains after the small arrays.
struct ScratchPlan {
    size_t o_consts, o_rmax, o_flags, o_guard, o_redo, o_count, o_ws;
    long long batch;                       // systems per factor launch (0: does not fit)
};

ScratchPlan plan_scratch(const tm_problem& p) {
    ScratchPlan pl{};
    const long long ns = n_systems(p);
    size_t o = 0;
    pl.o_consts = o; o += align256(sizeof(tmk::Consts));
    pl.o_rmax = o;   o += align256((size_t)ns * sizeof(double));
    pl.o_flags = o;  o += align256((size_t)ns * sizeof(int));
    pl.o_guard = o;  o += align256((size_t)ns * sizeof(int));
    pl.o_redo = o;   o += align256((size_t)ns * sizeof(int));
    pl.o_count = o;  o += 256;
    pl.o_ws = o;
    const size_t per = tmk::factor_ws_bytes_per_system(p.n_zones, p.n_groups, p.precision == TM_PREC_MIXED);
    pl.batch = 0;
    if (o < kScratchBytes && per > 0) {
        const long long slots = (long long)((kScratchBytes - o) / per);
        pl.batch = std::min(std::max(slots - tmk::kWsPadSystems, 0LL), ns);
    }
    return pl;
}

}  // namespace

extern "C" {

const char* tm_status_string(tm_status s) {
    // a C caller may pass any int: read the argument's bytes rather than load it as the enumeration
    // (a value outside the enumeration's range is undefined behaviour in C++)
    int v;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
        case TM_OK: return "TM_OK";
        case TM_ERR_INVALID_ARG: return "TM_ERR_INVALID_ARG";
        case TM_ERR_HIP: return "TM_ERR_HIP";
        case TM_ERR_SINGULAR: return "TM_ERR_SINGULAR";
        case TM_ERR_NOT_CONVERGED: return "TM_ERR_NOT_CONVERGED";
        case TM_ERR_NONFINITE: return "TM_ERR_NONFINITE";
        case TM_ERR_WORKSPACE: return "TM_ERR_WORKSPACE";
    }
    return "TM_UNKNOWN_STATUS";
}

const char* tm_last_error(const tm_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

tm_status tm_set_kernel_timing(tm_ctx* c, int32_t enable) {
    if (!c) return TM_ERR_INVALID_ARG;
    if (enable && !c->kt[0]) {
        TM_TRY(hip_check(c, hipSetDevice(c->device), "set device"));
        for (hipEvent_t& e : c->kt) TM_TRY(hip_check(c, hipEventCreate(&e), "create timing event"));
    }
    c->timing = enable != 0;
    c->timed = false;
    return TM_OK;
}

tm_status tm_kernel_time_ms(tm_ctx* c, double* ms) {
    if (!c) return TM_ERR_INVALID_ARG;
    if (!ms || !c->timing || !c->timed)
        return set_err(c, TM_ERR_INVALID_ARG, "kernel timing needs timing enabled, ms and a timed call");
    TM_TRY(hip_check(c, hipEventSynchronize(c->kt[1]), "timing event sync"));
    float f = 0.0f;
    TM_TRY(hip_check(c, hipEventElapsedTime(&f, c->kt[0], c->kt[1]), "timing event elapsed"));
    *ms = f;
    return TM_OK;
}

size_t tm_workspace_bytes(const tm_problem* p, int64_t batch_systems) {
    if (!valid_problem(p, nullptr) || batch_systems < 0) return 0;
    const long long ns = n_systems(*p);
    const long long b = batch_systems == 0 ? ns : std::min<long long>(batch_systems, ns);
    return (size_t)(b + tmk::kWsPadSystems) *
           tmk::factor_ws_bytes_per_system(p->n_zones, p->n_groups, p->precision == TM_PREC_MIXED);
}

tm_status tm_create(const tm_problem* p, void* stream, tm_ctx** out) {
    if (!out) return TM_ERR_INVALID_ARG;
    *out = nullptr;
    std::string why;
    if (!valid_problem(p, &why)) return TM_ERR_INVALID_ARG;
    tm_ctx* c = new tm_ctx();
    c->p = *p;
    c->stream = (hipStream_t)stream;
    // test and tuning knobs: TM_PIVOT = auto | always | never, TM_GROWTH_LIMIT = <double>
    if (const char* e = std::getenv("TM_PIVOT")) {
        if (!std::strcmp(e, "always")) c->pivot_policy = 1;
        else if (!std::strcmp(e, "never")) c->pivot_policy = 2;
    }
    if (const char* e = std::getenv("TM_GROWTH_LIMIT")) c->growth_limit = std::atof(e);
    if (const char* e = std::getenv("TM_FACTOR_KERNEL")) {
        if (!std::strcmp(e, "lane")) c->factor_kernel = tmk::kFactorLane;
        else if (!std::strcmp(e, "valu")) c->factor_kernel = tmk::kFactorQuadValu;
        else if (!std::strcmp(e, "mfma")) c->factor_kernel = tmk::kFactorQuadMfma;
        else if (!std::strcmp(e, "window")) c->factor_kernel = tmk::kFactorQuadWindow;
        else if (!std::strcmp(e, "bf16x3")) c->factor_kernel = tmk::kFactorQuadBf16x3;
        else if (!std::strcmp(e, "bf16")) c->factor_kernel = tmk::kFactorQuadBf16;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return TM_ERR_HIP;
    }
    *out = c;
    return TM_OK;
}

tm_status tm_destroy(tm_ctx* c) {
    if (!c) return TM_ERR_INVALID_ARG;
    if (c->consts) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->consts);
        (void)hipFree(c->res);
        (void)hipFree(c->res0);
        (void)hipFree(c->active);
        (void)hipFree(c->iters);
        (void)hipFree(c->flags);
        (void)hipFree(c->count);
        (void)hipHostFree(c->h_count);
        (void)hipFree(c->guard);
        (void)hipFree(c->redo);
        (void)hipFree(c->res_acc);
        (void)hipFree(c->tgt);
        (void)hipFree(c->alpha);
        (void)hipFree(c->pending);
        (void)hipFree(c->backtrack);
    }
    if (c->y_res) {
        (void)hipStreamSynchronize(c->stream);
        for (double* p : {c->y_res, c->y_res0, c->y_res_acc, c->y_tgt, c->y_alpha, c->y_res_sp, c->y_lev, c->y_gy,
                          c->y_dy})
            (void)hipFree(p);
        for (int* p : {c->y_active, c->y_iters, c->y_flags, c->y_pending, c->y_backtrack, c->y_redo}) (void)hipFree(p);
    }
    for (double* p : {c->lp_ka, c->lp_et, c->lp_ks, c->lp_temp, c->lp_amp})
        if (p) (void)hipFree(p);
    if (c->gbuf) (void)hipFree(c->gbuf);
    if (c->dbuf) (void)hipFree(c->dbuf);
    if (c->ws && c->ws_owned) (void)hipFree(c->ws);
    for (hipEvent_t e : c->kt)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return TM_OK;
}

tm_status tm_set_workspace(tm_ctx* c, void* dev, size_t bytes) {
    if (!c) return TM_ERR_INVALID_ARG;
    if ((dev == nullptr) != (bytes == 0))
        return set_err(c, TM_ERR_INVALID_ARG, "workspace pointer and size must both be set or both be 0");
    if (reinterpret_cast<uintptr_t>(dev) % 256 != 0)   // the factor kernels store 16-byte vectors into it
        return set_err(c, TM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (dev) {
        // enough for one launch of either step (each step checks its own need when it runs)
        const size_t one_sys = (size_t)(1 + tmk::kWsPadSystems) *
                               tmk::factor_ws_bytes_per_system(c->p.n_zones, c->p.n_groups,
                                                               c->p.precision == TM_PREC_MIXED);
        const size_t one_ray = tmk::ye_ws_bytes_per_ray(c->p.n_zones, c->p.n_groups);
        const size_t least = one_ray > 0 ? std::min(one_sys, one_ray) : one_sys;
        if (bytes < least) return set_err(c, TM_ERR_WORKSPACE, "workspace smaller than one launch's factors");
    }
    if (c->ws && c->ws_owned) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->ws);
    }
    c->ws = dev;
    c->ws_bytes = bytes;
    c->ws_owned = false;
    return TM_OK;
}

tm_status tm_assemble(tm_ctx* c, const tm_inputs* in, const double* psi_n, const double* psi, double* residual,
                      double* blocks) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    if (!psi_n || !psi || !residual) return set_err(c, TM_ERR_INVALID_ARG, "psi_n, psi and residual are required");
    tm_inputs folded;
    TM_TRY(fold_lapse(c, in, &folded));
    in = &folded;
    TM_TRY(ensure_small(c));
    const tmk::Shape sh = shape_of(c->p);
    const tmk::Fields f = fields_of(*in);
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, sh.N, c->consts, c->stream), "setup kernel"));
    tmk::ResidualOut o{};
    o.mode = tmk::kResPlain;
    o.res = c->res;
    TM_TRY(hip_check(c, tmk::launch_residual(sh, f, c->consts, psi_n, psi, residual, 1.0, o, c->stream),
                     "residual kernel"));
    if (blocks)
        TM_TRY(hip_check(c, tmk::launch_blocks(sh, f, c->consts, psi, blocks, c->stream), "blocks kernel"));
    return TM_OK;
}

tm_status tm_factor_solve(tm_ctx* c, const tm_inputs* in, const double* psi, const double* rhs, double* x,
                          int32_t transpose) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    if (!psi || !rhs || !x) return set_err(c, TM_ERR_INVALID_ARG, "psi, rhs and x are required");
    tm_inputs folded;
    TM_TRY(fold_lapse(c, in, &folded));
    in = &folded;
    TM_TRY(ensure_small(c));
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, c->p.n_groups, c->consts, c->stream),
                     "setup kernel"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->flags, 0, n_systems(c->p) * sizeof(int), c->stream), "memset flags"));
    const bool fp32 = c->p.precision == TM_PREC_MIXED;
    if (fp32)   // per-system max |rhs| for the power-of-two scaling of the float32 solve
        TM_TRY(hip_check(c, tmk::launch_sys_absmax(rhs, n_systems(c->p), (long long)c->p.n_zones * c->p.n_groups,
                                                   c->res, c->stream), "rhs scale kernel"));
    TM_TRY(run_factor(c, in, psi, rhs, 1.0, x, nullptr, nullptr, fp32, transpose != 0, nullptr,
                      fp32 ? c->res : nullptr));
    return check_zero_pivots(c);
}

tm_status tm_factor_solve_noalloc(tm_ctx* c, const tm_inputs* in, const double* psi, const double* rhs, double* x,
                                  int32_t transpose, int32_t* flags) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    if (!psi || !rhs || !x) return set_err(c, TM_ERR_INVALID_ARG, "psi, rhs and x are required");
    TM_TRY(no_lapse(c, in, "tm_factor_solve_noalloc"));
    const ScratchPlan pl = plan_scratch(c->p);
    if (pl.batch < 1)
        return set_err(c, TM_ERR_WORKSPACE, "problem too large for the " + std::to_string(kScratchBytes >> 20) +
                                                " MiB scratch of tm_factor_solve_noalloc (per-system arrays plus "
                                                "one batch of factors must fit)");
    unsigned char* base = nullptr;
    TM_TRY(scratch_of(c, &base));
    const long long ns = n_systems(c->p);
    const bool fp32 = c->p.precision == TM_PREC_MIXED;
    const int NT = tmk::padded_groups(c->p.n_groups);
    const size_t es = fp32 ? 4 : 8;
    tmk::Consts* cs = reinterpret_cast<tmk::Consts*>(base + pl.o_consts);
    double* rmax = reinterpret_cast<double*>(base + pl.o_rmax);
    int* fl = flags ? flags : reinterpret_cast<int*>(base + pl.o_flags);
    int* guard = reinterpret_cast<int*>(base + pl.o_guard);
    int* redo = reinterpret_cast<int*>(base + pl.o_redo);
    int* count = reinterpret_cast<int*>(base + pl.o_count);
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, c->p.n_groups, cs, c->stream), "setup kernel"));
    // the scratch keeps the previous call's contents: flags and the guard start at zero
    TM_TRY(hip_check(c, tmk::launch_fill_i32(fl, ns, 0, c->stream), "fill kernel"));
    TM_TRY(hip_check(c, tmk::launch_fill_i32(guard, ns, 0, c->stream), "fill kernel"));
    if (fp32)
        TM_TRY(hip_check(c, tmk::launch_sys_absmax(rhs, ns, (long long)c->p.n_zones * c->p.n_groups, rmax, c->stream),
                         "rhs scale kernel"));
    tmk::FactorArgs a;
    a.sh = shape_of(c->p);
    a.f = fields_of(*in);
    a.cs = cs;
    a.psi = psi;
    a.rhs = rhs;
    a.rhs_sign = 1.0;
    a.rhs_max = fp32 ? rmax : nullptr;
    a.x = x;
    a.psi_out = nullptr;
    a.active = nullptr;
    a.flags = fl;
    a.iters = nullptr;
    a.guard = guard;
    a.growth_limit = c->growth_limit;
    a.dx = nullptr;
    a.pending = nullptr;
    a.alpha = nullptr;
    a.wsC = base + pl.o_ws;
    a.wsY = base + pl.o_ws + (size_t)(pl.batch + tmk::kWsPadSystems) * c->p.n_zones * NT * NT * es;
    const bool pivot_first = c->pivot_policy == 1;
    for (long long s0 = 0; s0 < ns; s0 += pl.batch) {
        a.sys0 = s0;
        a.nsys = std::min(pl.batch, ns - s0);
        TM_TRY(hip_check(c, tmk::launch_factor(a, fp32, transpose != 0, pivot_first, c->stream, c->factor_kernel), "factor kernel"));
    }
    if (!pivot_first) {
        // no read-back: the partial-pivoting re-run is launched for the marked systems (waves without one
        // return at once)
        TM_TRY(hip_check(c, tmk::launch_mark(guard, ns, redo, count, c->stream), "mark kernel"));
        a.active = redo;
        for (long long s0 = 0; s0 < ns; s0 += pl.batch) {
            a.sys0 = s0;
            a.nsys = std::min(pl.batch, ns - s0);
            TM_TRY(hip_check(c, tmk::launch_factor(a, fp32, transpose != 0, true, c->stream),
                             "pivoting factor kernel"));
        }
    }
    return TM_OK;
}

tm_status tm_newton_step(tm_ctx* c, const tm_inputs* in, const double* psi_n, double* psi, int32_t max_iter,
                         double rtol, tm_stats* stats) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    if (!psi_n || !psi) return set_err(c, TM_ERR_INVALID_ARG, "psi_n and psi are required");
    if (max_iter < 0 || !(rtol >= 0.0)) return set_err(c, TM_ERR_INVALID_ARG, "max_iter >= 0 and rtol >= 0 required");
    tm_inputs folded;
    TM_TRY(fold_lapse(c, in, &folded));
    in = &folded;
    TM_TRY(ensure_small(c));
    TM_TRY(ensure_gbuf(c));
    const long long ns = n_systems(c->p);
    const tmk::Shape sh = shape_of(c->p);
    const tmk::Fields f = fields_of(*in);
    const bool fp32 = c->p.precision == TM_PREC_MIXED;
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, sh.N, c->consts, c->stream), "setup kernel"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->iters, 0, ns * sizeof(int), c->stream), "memset iters"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->flags, 0, ns * sizeof(int), c->stream), "memset flags"));

    auto count_of = [&](const int* flags_arr, int* out_n) -> tm_status {
        TM_TRY(hip_check(c, tmk::launch_count_active(flags_arr, ns, c->count, c->stream), "count kernel"));
        TM_TRY(hip_check(c, hipMemcpyAsync(c->h_count, c->count, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                         "copy count"));
        TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
        *out_n = *c->h_count;
        return TM_OK;
    };
    tmk::ResidualOut o{};
    o.res = c->res;
    o.res0 = c->res0;
    o.res_acc = c->res_acc;
    o.tgt = c->tgt;
    o.alpha = c->alpha;
    o.pending = c->pending;
    o.backtrack = c->backtrack;
    o.active = c->active;
    o.iters = c->iters;
    o.max_iter = max_iter;
    o.rtol = rtol;
    // conservation statistics are taken at every evaluated state, so the last evaluation of a system
    // (its accepted state) leaves those of the returned psi
    o.stats = stats != nullptr;
    if (stats) {
        o.n_tot = stats->n_tot;
        o.e_tot = stats->e_tot;
        o.budget = stats->budget_n;
        o.lum = stats->lum_n;
    }
    TM_TRY(hip_check(c, hipMemsetAsync(c->pending, 0, ns * sizeof(int), c->stream), "memset pending"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->backtrack, 0, ns * sizeof(int), c->stream), "memset backtrack"));
    o.mode = tmk::kResInitial;
    TM_TRY(hip_check(c, tmk::launch_residual(sh, f, c->consts, psi_n, psi, c->gbuf, 1.0, o, c->stream),
                     "residual kernel"));
    const int max_trials = 9;                              // alpha = 1, 1/2, ..., 1/256
    for (int it = 0; it < max_iter; ++it) {
        int nact = 0;
        TM_TRY(count_of(c->active, &nact));
        if (nact == 0) break;
        // Newton update psi += delta for the active systems (delta kept for backtracking)
        // res holds max |G| of the residual in gbuf for every active system (scaling of the float32 solve)
        TM_TRY(run_factor(c, in, psi, c->gbuf, -1.0, nullptr, psi, c->active, fp32, false, c->dbuf, c->res));
        // line search on max|G| with the FP64 residual; a rejected trial is moved back to half the step
        o.mode = tmk::kResTrial;
        for (int t = 0; t < max_trials; ++t) {
            TM_TRY(hip_check(c, tmk::launch_residual(sh, f, c->consts, psi_n, psi, c->gbuf, 1.0, o, c->stream),
                             "residual kernel"));
            int nback = 0;
            TM_TRY(count_of(c->backtrack, &nback));
            if (nback == 0) break;
            TM_TRY(hip_check(c, tmk::launch_backtrack(sh, psi, c->dbuf, c->backtrack, c->alpha, c->stream),
                             "backtrack kernel"));
        }
    }

    // final flags from the last evaluated residual of each system (its accepted state)
    TM_TRY(hip_check(c, tmk::launch_final_flags(ns, c->res, c->tgt, rtol, c->flags, c->stream), "flags kernel"));
    if (stats) {
        auto cp = [&](void* dst, const void* src, size_t bytes) -> tm_status {
            if (!dst) return TM_OK;
            return hip_check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream), "copy stats");
        };
        TM_TRY(cp(stats->res_inf, c->res, ns * sizeof(double)));
        TM_TRY(cp(stats->res0_inf, c->res0, ns * sizeof(double)));
        TM_TRY(cp(stats->iters, c->iters, ns * sizeof(int)));
        TM_TRY(cp(stats->flags, c->flags, ns * sizeof(int)));
    }
    // worst status over systems
    std::vector<int> fl(ns);
    TM_TRY(hip_check(c, hipMemcpyAsync(fl.data(), c->flags, ns * sizeof(int), hipMemcpyDeviceToHost, c->stream),
                     "copy flags"));
    TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
    int any = 0;
    for (int v : fl) any |= v;
    if (any & TM_FLAG_NONFINITE) return set_err(c, TM_ERR_NONFINITE, "non-finite residual in some system");
    if (any & TM_FLAG_ZERO_PIVOT) return set_err(c, TM_ERR_SINGULAR, "zero pivot in some block");
    if (any & TM_FLAG_NOT_CONVERGED) return set_err(c, TM_ERR_NOT_CONVERGED, "some system missed rtol");
    c->err.clear();
    return TM_OK;
}

tm_status tm_adjoint_step(tm_ctx* c, const tm_inputs* in, const double* psi_n, const double* psi_np1,
                          const double* seed, double* mu, double* g_ka, double* g_eta, double* g_ks, double* g_amp) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    if (!psi_np1 || !seed || !mu) return set_err(c, TM_ERR_INVALID_ARG, "psi_np1, seed and mu are required");
    (void)psi_n;
    tm_inputs folded;                      // the lapse's source factors folded in, as in the forward step
    TM_TRY(fold_lapse(c, in, &folded));
    in = &folded;
    TM_TRY(ensure_small(c));
    const tmk::Shape sh = shape_of(c->p);
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, sh.N, c->consts, c->stream), "setup kernel"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->flags, 0, n_systems(c->p) * sizeof(int), c->stream), "memset flags"));
    TM_TRY(run_factor(c, in, psi_np1, seed, 1.0, mu, nullptr, nullptr, /*fp32=*/false, /*transpose=*/true));
    if (g_ka || g_eta || g_ks || g_amp)
        TM_TRY(hip_check(c, tmk::launch_vjp(sh, fields_of(*in), c->consts, psi_np1, mu, g_ka, g_eta, g_ks, g_amp,
                                            c->stream),
                         "vjp kernel"));
    return check_zero_pivots(c);
}

size_t tm_ye_workspace_bytes(const tm_problem* p, int64_t batch_rays) {
    if (!valid_problem(p, nullptr) || batch_rays < 0) return 0;
    const long long R = p->n_rays;
    const long long b = batch_rays == 0 ? R : std::min<long long>(batch_rays, R);
    return (size_t)b * tmk::ye_ws_bytes_per_ray(p->n_zones, p->n_groups);
}

tm_status tm_ye_newton_step(tm_ctx* c, const tm_inputs* in, const tm_ye_inputs* yin, const double* psi_n,
                            double* psi, double* ye, int32_t max_iter, double rtol, tm_ye_stats* stats) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    TM_TRY(check_ye_inputs(c, yin));
    if (yin->pair_amp && !in->r_nu)
        return set_err(c, TM_ERR_INVALID_ARG, "the pair processes need r_nu (their angular factor uses R_nu)");
    if (yin->pair_amp && in->lapse)
        return set_err(c, TM_ERR_INVALID_ARG, "the pair processes take no lapse (lapse must be NULL with pair_amp)");
    if (c->p.precision != TM_PREC_FP64)
        return set_err(c, TM_ERR_INVALID_ARG, "the Y_e-coupled step is FP64 only (precision must be TM_PREC_FP64)");
    if (!psi_n || !psi || !ye) return set_err(c, TM_ERR_INVALID_ARG, "psi_n, psi and ye are required");
    if (max_iter < 0 || !(rtol >= 0.0)) return set_err(c, TM_ERR_INVALID_ARG, "max_iter >= 0 and rtol >= 0 required");
    tm_inputs folded;                      // the lapse's source factors folded in, as in the species step
    TM_TRY(fold_lapse(c, in, &folded));
    in = &folded;
    TM_TRY(ensure_small(c));
    TM_TRY(ensure_gbuf(c));
    TM_TRY(ensure_ye(c));
    const long long R = c->p.n_rays;
    const tmk::Shape sh = shape_of(c->p);
    tmk::Shape sh2 = sh;                  // the species pair as a two-species problem (prefix of the arrays)
    sh2.S = 2;
    const tmk::Fields f = fields_of(*in);
    const tmk::YeFields yf = ye_fields_of(*yin);
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, sh.N, c->consts, c->stream), "setup kernel"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->y_iters, 0, R * sizeof(int), c->stream), "memset iters"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->y_flags, 0, R * sizeof(int), c->stream), "memset flags"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->y_pending, 0, R * sizeof(int), c->stream), "memset pending"));
    TM_TRY(hip_check(c, hipMemsetAsync(c->y_backtrack, 0, R * sizeof(int), c->stream), "memset backtrack"));

    auto count_of = [&](const int* arr, int* out_n) -> tm_status {
        TM_TRY(hip_check(c, tmk::launch_count_active(arr, R, c->count, c->stream), "count kernel"));
        TM_TRY(hip_check(c, hipMemcpyAsync(c->h_count, c->count, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                         "copy count"));
        TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
        *out_n = *c->h_count;
        return TM_OK;
    };
    tmk::ResidualOut o{};
    o.mode = tmk::kResEval;
    o.res = c->y_res_sp;
    o.level = c->y_lev;
    tmk::YeOut yo{};
    yo.res = c->y_res;
    yo.res0 = c->y_res0;
    yo.res_acc = c->y_res_acc;
    yo.tgt = c->y_tgt;
    yo.alpha = c->y_alpha;
    yo.pending = c->y_pending;
    yo.backtrack = c->y_backtrack;
    yo.active = c->y_active;
    yo.iters = c->y_iters;
    yo.lepton = stats ? stats->lepton : nullptr;      // taken at every evaluated state; the last is the returned one
    yo.max_iter = max_iter;
    yo.rtol = rtol;
    auto evaluate = [&](int mode) -> tm_status {
        o.pending = mode == tmk::kResInitial ? nullptr : c->y_pending;
        yo.mode = mode;
        TM_TRY(hip_check(c, tmk::launch_residual(sh2, f, c->consts, psi_n, psi, c->gbuf, 1.0, o, c->stream),
                         "residual kernel"));
        return hip_check(c, tmk::launch_ye_couple(sh, f, yf, c->consts, psi, ye, c->gbuf, c->y_gy, c->y_lev, yo,
                                                  c->stream), "coupling kernel");
    };
    TM_TRY(evaluate(tmk::kResInitial));

    long long batch = 0;
    TM_TRY(ye_batch(c, &batch));
    tmk::YeFactorArgs a;
    a.sh = sh;
    a.f = f;
    a.y = yf;
    a.cs = c->consts;
    a.psi = psi;
    a.ye = ye;
    a.G = c->gbuf;
    a.GY = c->y_gy;
    a.rhs_sign = -1.0;
    a.psi_out = psi;
    a.ye_out = ye;
    a.dx = c->dbuf;
    a.dY = c->y_dy;
    a.active = c->y_active;
    a.flags = c->y_flags;
    a.iters = c->y_iters;
    a.pending = c->y_pending;
    a.alpha = c->y_alpha;
    a.ws = static_cast<double*>(c->ws);
    a.growth_limit = c->growth_limit;
    // Diagonal pivots on lane tiles, with the rays the growth guard sends back re-run with partial
    // pivoting (TM_PIVOT=always: partial pivoting only; =never: a guard trip is an error).  The
    // neutrinosphere options and the pair processes take the partial-pivoting kernel.
    const bool tiled = c->pivot_policy != 1 && tmk::ye_tiled_applies(a);
    const int max_trials = 9;                              // alpha = 1, 1/2, ..., 1/256
    for (int it = 0; it < max_iter; ++it) {
        int nact = 0;
        TM_TRY(count_of(c->y_active, &nact));
        if (nact == 0) break;
        if (tiled && c->pivot_policy == 2)
            TM_TRY(hip_check(c, tmk::launch_fill_i32(c->y_redo, R, 0, c->stream), "fill kernel"));
        for (long long r0 = 0; r0 < R; r0 += batch) {
            a.ray0 = r0;
            a.nray = std::min(batch, R - r0);
            if (tiled) {
                a.redo = c->y_redo;
                TM_TRY(hip_check(c, tmk::launch_ye_factor_tiled(a, c->stream), "coupled tiled factor kernel"));
                if (c->pivot_policy != 2)        // the marked rays of this batch, with partial pivoting
                    TM_TRY(hip_check(c, tmk::launch_ye_factor(a, c->stream), "coupled factor kernel"));
            } else {
                a.redo = nullptr;
                TM_TRY(hip_check(c, tmk::launch_ye_factor(a, c->stream), "coupled factor kernel"));
            }
        }
        if (tiled && c->pivot_policy == 2) {
            int nredo = 0;
            TM_TRY(count_of(c->y_redo, &nredo));
            if (nredo > 0) return set_err(c, TM_ERR_SINGULAR, "diagonal-pivot growth guard tripped in the coupled step");
        }
        for (int t = 0; t < max_trials; ++t) {
            TM_TRY(evaluate(tmk::kResTrial));
            int nback = 0;
            TM_TRY(count_of(c->y_backtrack, &nback));
            if (nback == 0) break;
            TM_TRY(hip_check(c, tmk::launch_ye_backtrack(sh, psi, ye, c->dbuf, c->y_dy, c->y_backtrack, c->y_alpha,
                                                         c->stream), "backtrack kernel"));
        }
    }
    TM_TRY(hip_check(c, tmk::launch_final_flags(R, c->y_res, c->y_tgt, rtol, c->y_flags, c->stream), "flags kernel"));
    if (stats) {
        auto cp = [&](void* dst, const void* src, size_t bytes) -> tm_status {
            if (!dst) return TM_OK;
            return hip_check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream), "copy stats");
        };
        TM_TRY(cp(stats->res_inf, c->y_res, R * sizeof(double)));
        TM_TRY(cp(stats->res0_inf, c->y_res0, R * sizeof(double)));
        TM_TRY(cp(stats->iters, c->y_iters, R * sizeof(int)));
        TM_TRY(cp(stats->flags, c->y_flags, R * sizeof(int)));
    }
    std::vector<int> fl(R);
    TM_TRY(hip_check(c, hipMemcpyAsync(fl.data(), c->y_flags, R * sizeof(int), hipMemcpyDeviceToHost, c->stream),
                     "copy flags"));
    TM_TRY(hip_check(c, hipStreamSynchronize(c->stream), "stream sync"));
    int any = 0;
    for (int v : fl) any |= v;
    if (any & TM_FLAG_NONFINITE) return set_err(c, TM_ERR_NONFINITE, "non-finite residual in some ray");
    if (any & TM_FLAG_ZERO_PIVOT) return set_err(c, TM_ERR_SINGULAR, "zero pivot in some coupled block");
    if (any & TM_FLAG_NOT_CONVERGED) return set_err(c, TM_ERR_NOT_CONVERGED, "some ray missed rtol");
    c->err.clear();
    return TM_OK;
}

tm_status tm_temperature_update(tm_ctx* c, const tm_inputs* in, const tm_ye_inputs* yin, const double* psi,
                                const double* ye, const double* stat_weights, const double* de_dT,
                                const double* de_dye, double* de_out, double* temp_out) {
    if (!c) return TM_ERR_INVALID_ARG;
    TM_TRY(check_inputs(c, in));
    TM_TRY(check_ye_inputs(c, yin));
    if (yin->pair_amp && !in->r_nu)
        return set_err(c, TM_ERR_INVALID_ARG, "the pair processes need r_nu (their angular factor uses R_nu)");
    TM_TRY(no_lapse(c, in, "the temperature update"));
    if (!in->temp) return set_err(c, TM_ERR_INVALID_ARG, "temp (T^n) is required");
    if (!psi || !ye || !stat_weights || !de_dT || !de_dye || !temp_out)
        return set_err(c, TM_ERR_INVALID_ARG, "psi, ye, stat_weights, de_dT, de_dye and temp_out are required");
    if (c->p.n_species > 16) return set_err(c, TM_ERR_INVALID_ARG, "the temperature update takes S <= 16");
    TM_TRY(ensure_small(c));
    const tmk::Shape sh = shape_of(c->p);
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, sh.N, c->consts, c->stream), "setup kernel"));
    return hip_check(c, tmk::launch_ye_temperature(sh, fields_of(*in), ye_fields_of(*yin), c->consts, psi, ye,
                                                   stat_weights, de_dT, de_dye, de_out, temp_out, c->stream),
                     "temperature kernel");
}

tm_status tm_energy_advect(tm_ctx* c, const tm_inputs* in, const tm_eadv_inputs* ea, double* psi, double* xi,
                           int32_t* flags) {
    if (!c) return TM_ERR_INVALID_ARG;
    if (!in || !in->e_edge) return set_err(c, TM_ERR_INVALID_ARG, "e_edge is required");
    if (!ea) return set_err(c, TM_ERR_INVALID_ARG, "energy-advection inputs are NULL");
    if (!psi) return set_err(c, TM_ERR_INVALID_ARG, "psi is required");
    if (ea->mode != TM_EADV_LAGRANGIAN && ea->mode != TM_EADV_LAPSE)
        return set_err(c, TM_ERR_INVALID_ARG, "mode must be TM_EADV_LAGRANGIAN or TM_EADV_LAPSE");
    if (!ea->rho_old != !ea->rho_new) return set_err(c, TM_ERR_INVALID_ARG, "rho_old and rho_new go together");
    if (!ea->lapse_old != !ea->lapse_new)
        return set_err(c, TM_ERR_INVALID_ARG, "lapse_old and lapse_new go together");
    if (ea->mode == TM_EADV_LAPSE && !ea->lapse_old)
        return set_err(c, TM_ERR_INVALID_ARG, "the lapse mode needs lapse_old and lapse_new");
    tmk::EaArgs a;
    a.mode = ea->mode == TM_EADV_LAPSE ? tmk::kEaLapse : tmk::kEaLagrangian;
    a.N = c->p.n_groups;
    a.RI = (long long)c->p.n_rays * c->p.n_zones;
    a.nz = (long long)c->p.n_species * a.RI;
    a.e_edge = in->e_edge;
    const bool lag = a.mode == tmk::kEaLagrangian;
    a.rho_old = lag ? ea->rho_old : nullptr;
    a.rho_new = lag ? ea->rho_new : nullptr;
    a.a_old = ea->lapse_old;
    a.a_new = ea->lapse_new;
    a.dlnR = lag ? ea->dlnR : nullptr;
    a.dlnb = lag ? ea->dlnb : nullptr;
    a.edd = lag ? ea->eddington : nullptr;
    a.psi = psi;
    a.xi = xi;
    a.flags = flags;
    TM_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    return hip_check(c, tmk::launch_energy_advect(a, c->stream), "energy-advection kernel");
}

tm_status tm_luminosity_seed(tm_ctx* c, const tm_inputs* in, const double* add, double* seed) {
    if (!c) return TM_ERR_INVALID_ARG;
    if (!in || !in->r_edge || !in->e_edge) return set_err(c, TM_ERR_INVALID_ARG, "r_edge and e_edge are required");
    if (!seed) return set_err(c, TM_ERR_INVALID_ARG, "seed is required");
    if (!in->lapse != !in->lapse_edge) return set_err(c, TM_ERR_INVALID_ARG, "lapse and lapse_edge go together");
    if (c->p.outer_bc == TM_BC_GEOMETRIC)
        return set_err(c, TM_ERR_INVALID_ARG,
                       "the luminosity seed of TM_BC_GEOMETRIC depends on psi (this entry point takes none)");
    TM_TRY(ensure_small(c));
    const tmk::Shape sh = shape_of(c->p);
    TM_TRY(hip_check(c, tmk::launch_setup(in->e_edge, in->nes_g, sh.N, c->consts, c->stream), "setup kernel"));
    return hip_check(c, tmk::launch_lum_seed(sh, in->r_edge, in->lapse_edge, c->consts, add, seed, c->stream),
                     "seed kernel");
}

}  // extern "C"
