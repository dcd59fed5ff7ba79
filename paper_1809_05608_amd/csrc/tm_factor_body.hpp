// Fused Jacobian assembly + block-Thomas factor/solve of the linearised transport
// step (eq. a62ae), one (species, ray) system per SL-lane group of a wavefront.
//
// Layout on the chip: lane k of a group owns row k of the current zone's dense N x N
// block (N <= NT <= 32, SL = 16 or 32 lanes per system, 4 or 2 systems per wave64).
// The sweep over radial zones is sequential inside the group; systems run in parallel.
// Per zone the row is assembled in registers (flux-limited diffusion derivatives,
// emission/absorption, dense NES coupling), the Schur complement
//   Ahat_i = A_i - diag(bm_i) C_{i-1}
// is formed with the previous factor row still in registers, and an unnormalised
// in-place Gauss-Jordan elimination with partial pivoting produces
//   C_i = Ahat_i^{-1} diag(bp_i)  and  y_i = Ahat_i^{-1} (r_i - bm_i * y_{i-1}).
// Pivot search is a packed-key max over the group (DPP row reductions plus a
// 16-lane swap); the pivot row is broadcast through LDS; row ownership is left
// permuted during the elimination and restored once per zone through LDS.
// C_i and y_i are the only quantities that reach HBM (workspace, [zone][m][k]
// so that both sweeps are coalesced); the backward sweep forms
//   x_i = y_i - C_i x_{i+1}
// and either writes x or adds it to psi (Newton update, eq. a62aa).
// The transposed variant (adjoint) assembles the same rows, transposes the block
// through LDS and swaps the roles of bm and bp.
#pragma once

#include <type_traits>

#include "tm_kernels.hpp"

namespace tmk {

__device__ __forceinline__ double texp(double x) { return exp(x); }
__device__ __forceinline__ float texp(float x) { return __expf(x); }

// Reciprocal from the hardware estimate refined by Newton steps (one for float, two for
// double), instead of the full IEEE division sequence.  Zero gives a non-finite result.
__device__ __forceinline__ float rcp_nr(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Power-of-two scaling of a system's right-hand side for a float32 solve: the solve is linear, so
// x = s solve(J, r / s) with s = 2^e near max|r| keeps right-hand sides (Newton residuals) below the
// float32 range representable, and leaves every in-range float32 rounding unchanged.
struct RhsScale {
    double in, out;       // multiplier of the right-hand side, multiplier of the solution
};
template <typename T>
__device__ __forceinline__ RhsScale rhs_scale(const FactorArgs& A, long long sys) {
    RhsScale r{A.rhs_sign, 1.0};
    if (sizeof(T) == 4 && A.rhs_max) {
        const double m = A.rhs_max[sys];
        if (m > 0.0 && m < INFINITY) {
            const int e = ilogb(m);
            r.in = ldexp(A.rhs_sign, -e);
            r.out = ldexp(1.0, e);
        }
    }
    return r;
}

template <typename T, int NT>
struct alignas(16) SysLds {
    static constexpr int FS = NT + 16 / (int)sizeof(T);   // row stride: >= NT + 2, multiple of 16 bytes
    T prow[FS];        // pivot row: [0, NT) entries, NT right-hand side, NT+1 diagonal of B
    T bc[FS];          // broadcast of a zone's psi row (NES) or of x_{i+1} (back substitution)
    T dd[FS];          // NES neighbour factors exp(-(eps_{j+1} - eps_j)/T)
    T fix[NT][FS];     // row-ownership fix-up and transpose staging
    int sidx[NT];      // slot of the in-place elimination that holds column k of C
};

// PIVOT = false: diagonal pivots with a growth guard.  The blocks of this method are
// column diagonally dominant (identity plus positive diagonal terms; the NES and transport
// couplings conserve number, so their V/W-weighted column sums vanish), for which elimination
// without pivoting is stable.  A system whose multipliers exceed A.growth_limit, or that
// meets a zero or non-finite pivot, is not updated and is marked in A.guard so that the
// host can re-factor it with PIVOT = true (partial pivoting).
// Lanes per system: partial pivoting reduces the pivot key with DPP row operations and needs
// power-of-two groups (16 or 32 lanes); diagonal pivots only talk through LDS, so a system
// takes exactly NT lanes and a wave64 holds floor(64/NT) systems (3 at N = 20).
template <int NT, bool PIVOT>
constexpr int lanes_per_system() { return PIVOT ? (NT > 16 ? 32 : 16) : NT; }

// GEO: the geometric limiter and the geometric outer boundary are compiled in (a separate set of
// instantiations, launched only when the problem asks for either, so that the common path keeps its
// register allocation).
template <typename T, int NT, bool TRANS, bool PIVOT, bool LAPSE = true, bool GEO = false>
__device__ __forceinline__ void factor_sweeps(const FactorArgs& A) {
    constexpr int SL = lanes_per_system<NT, PIVOT>();
    constexpr int SPW = 64 / SL;
    constexpr int SPB = (kBlock / 64) * SPW;
    __shared__ SysLds<T, NT> lds_all[SPB];
    constexpr int PS = NT + 2;                      // row stride of the staged NES shape matrix
    __shared__ T s_P[NT * PS];
    for (int j = threadIdx.x; j < NT * NT; j += kBlock) s_P[(j / NT) * PS + (j % NT)] = (T)A.cs->P[j / NT][j % NT];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);     // uniform over the wave
    const bool in_group = lane < SPW * SL;                                   // lanes past the last group idle
    const int sub = in_group ? lane / SL : SPW - 1;
    const int k = in_group ? lane % SL : SL;                                 // idle lanes own no row
    const long long sb = (long long)blockIdx.x * SPB + wave * SPW + sub;    // system within the batch
    const bool in_batch = sb < A.nsys;
    const long long sbc = in_batch ? sb : A.nsys - 1;                        // clamped for loads
    const long long sys = A.sys0 + sbc;                                      // global system index
    // the same for lane ln, recomputed inside and after the zone loop rather than held live through it
    auto system_of = [&](int ln) -> long long {
        const int s_sub = ln < SPW * SL ? ln / SL : SPW - 1;
        const long long s_b = (long long)blockIdx.x * SPB + wave * SPW + s_sub;
        return A.sys0 + (s_b < A.nsys ? s_b : A.nsys - 1);
    };
    const bool live = in_group && in_batch && (A.active == nullptr || A.active[sys] != 0);
    if (__ballot(live) == 0) return;                                         // whole wave idle

    SysLds<T, NT>& L = lds_all[wave * SPW + sub];
    const Shape& sh = A.sh;
    const int N = sh.N, I = sh.I;
    const bool is_row = k < NT;      // owns a (possibly padded) row of the block
    const bool real = k < N;         // owns a real energy-group row
    const int kk = real ? k : 0;     // safe group index for loads
    const int kr = is_row ? k : 0;   // safe row index for LDS
    const int kp_safe = k < kMaxN ? k : 0;
    const int ray = (int)(sys % sh.R);
    const double* re = A.f.r_edge + (size_t)ray * (I + 1);
    const size_t cell0 = (size_t)sys * I * N;
    const double* psi = A.psi + cell0;
    const double* ka = A.f.kappa_a + cell0;
    const double* et = A.f.eta + cell0;
    const double* ks = A.f.kappa_s + cell0;
    const double* rhs = A.rhs + cell0;
    const double* tz = A.f.temp + (size_t)ray * I;
    const double c = sh.c_dt;
    const bool diff = sh.terms & kDiffusion, emabs = sh.terms & kEmAbs, nes = sh.terms & kNes;
    // Workspace, interleaved by wave group: the SPW systems of group g keep, per zone i and column m
    // (column pair for FP64), one run of SPW * NT entries, system s at offset s * NT and row k at
    // s * NT + k.  A wave's store or load of a column is then one contiguous run (3 * 20 entries at
    // N = 20) rather than SPW separate pieces.  A last partial group has empty slots, which the workspace size allows for
    // (kWsPadSystems); lanes of a clamped system use that system's slot.
    // sbc / SPW, the same for every lane of the wave (a clamped lane's system is the batch's last, which lies
    // in this wave whenever any lane of it is live), so the workspace bases stay scalar
    const long long wg = (long long)blockIdx.x * (SPB / SPW) + wave;
    const int lo = (int)(sbc - wg * SPW) * NT + k;             // this lane's place in a run
    constexpr int zs = SPW * NT;                                // entries per (zone, column) run
    T* wsC = reinterpret_cast<T*>(A.wsC) + (size_t)wg * SPW * I * NT * NT;
    T* wsY = reinterpret_cast<T*>(A.wsY) + (size_t)wg * SPW * I * NT;
    const bool store = live && real;
    // FP64 rows go as column pairs (16 bytes per lane and instruction): run j of a zone holds columns
    // 2j, 2j+1 of every row as pairs.  Float32 rows keep one column per run (pairs spill the 5-wave kernel).
    typedef T V2 __attribute__((ext_vector_type(2)));
    constexpr bool PAIRS = sizeof(T) == 8;
    // FP64 row of zone z as this lane stored it (columns at or beyond N, or !ok, read as 0); nt: non-temporal
    auto ws_row = [&](int z, bool ok, bool nt, T (&c)[NT]) {
        const V2* q = reinterpret_cast<const V2*>(wsC + (size_t)z * NT * zs) + lo;
#pragma unroll
        for (int j = 0; j < NT / 2; ++j) {
            const V2 v = (ok && 2 * j < N) ? (nt ? nt_load(q + (size_t)j * zs) : q[(size_t)j * zs]) : V2{(T)0, (T)0};
            c[2 * j] = v.x;
            c[2 * j + 1] = 2 * j + 1 < N ? v.y : (T)0;
        }
    };

    const T* Prow = s_P + kr * PS;                  // row k of the NES shape (zero outside N x N)
    const double de_k = A.cs->de[kp_safe];
    const double eps_k = A.cs->eps[kp_safe];

    // ---------------------------------------------------------------- forward sweep
    T a[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) a[j] = (T)0;
    T ycar = (T)0;
    double psi_c = real ? psi[kk] : 0.0;
    double sig_c = real ? ka[kk] + et[kk] : 0.0;
    double lam_c = real ? rcp_nr(sig_c + ks[kk]) : 1.0;
    double dHu_lo = 0.0, dHv_lo = 0.0, bp_prev = 0.0;
    bool zp = false;
    // largest |multiplier| as a monotone key (diagonal pivots); for double the key is the upper word, so
    // the guard compares magnitudes to about 2^-20 relative, ample for a growth threshold
    uint32_t gkey = 0;
    const RhsScale rsc = rhs_scale<T>(A, sys);
    // FP64: NES neighbour factors exp(-(eps_{k+1} - eps_k)/T) of every zone, computed before the sweep and
    // parked in the lane's own y slot of the zone, which the same lane overwrites only at the end of that zone
    if constexpr (sizeof(T) == 8) {
        if (nes && live && is_row) {
            for (int i = 0; i < I; ++i)
                wsY[(size_t)i * zs + lo] = (k + 1 < N) ? texp((T)(-de_k / tz[i])) : (T)0;
        }
    }

    for (int i = 0; i < I; ++i) {
        // lane index re-materialised per zone: comparisons with it are evaluated where used
        // instead of being hoisted out of the zone loop as dozens of live lane masks
        int kz = k;
        asm volatile("" : "+v"(kz));
        // the system's cell offset likewise, so the per-array addresses are formed where used rather than
        // held through the zone as one 64-bit pointer per array
        int lnz;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lnz));
        const long long sysz = system_of(lnz);
        const size_t co = (size_t)sysz * I * N;
        // next zone, own group
        double psi_n1 = 0.0, sig_n1 = 0.0, lam_n1 = 1.0;
        if (i + 1 < I && real) {
            const size_t cn = (size_t)(i + 1) * N + kk;
            psi_n1 = A.psi[co + cn];
            sig_n1 = A.f.kappa_a[co + cn] + A.f.eta[co + cn];
            lam_n1 = rcp_nr(sig_n1 + A.f.kappa_s[co + cn]);
        }
        const double rlo = re[i], rhi = re[i + 1];
        const double V = shell_volume(rlo, rhi);
        double iV = rcp_nr(V);
        double A_lo = rlo * rlo, A_hi = rhi * rhi;
        double lap_hi = 1.0;
        if (LAPSE && A.f.lapse) {                           // eq. a58 times a_i c dt: a^3 / V and A / a^2
            const double* lz = A.f.lapse + (size_t)ray * I;
            const double* le = A.f.lapse_edge + (size_t)ray * (I + 1);
            const double a0 = lz[i], e0 = le[i], e1 = le[i + 1];
            iV *= a0 * a0 * a0;
            A_lo /= e0 * e0;
            A_hi /= e1 * e1;
            if (i + 1 < I) {
                const double a1 = lz[i + 1];
                lap_hi = a1 * a1 * a1;
            }
        }
        double dHu_hi = 0.0, dHv_hi = 0.0, V_hi = 1.0;
        if (i + 1 < I) {
            const double rp = re[i + 2];
            const double D_hi = 0.5 * (rhi + rp) - 0.5 * (rlo + rhi);
            V_hi = shell_volume(rhi, rp);
            if (diff && real) {
                const double limb = (GEO && sh.limiter == 2) ? limb_factor(rhi, A.f.r_nu[(size_t)(sysz / sh.R) * N + kk]) : -1.0;
                const EdgeFlux e = edge_flux(psi_c, psi_n1, sqrt(lam_c * lam_n1), D_hi, sh.psi_floor, sh.limiter, limb);
                dHu_hi = e.dHu;
                dHv_hi = e.dHv;
            }
        } else if (sh.outer_bc == 1) {
            dHu_hi = 1.0;                                   // free streaming: H = psi of the last zone
        } else if (GEO && sh.outer_bc == 2 && diff && real) {     // ghost zone of eq. a62af
            const double rnu = A.f.r_nu[(size_t)(sysz / sh.R) * N + kk];
            const Ghost gh = outer_ghost(rlo, rhi, rnu);
            const EdgeFlux e = edge_flux(psi_c, gh.ratio * psi_c, lam_c, gh.D, sh.psi_floor, sh.limiter,
                                         sh.limiter == 2 ? limb_factor(rhi, rnu) : -1.0);
            dHu_hi = e.dHu + gh.ratio * e.dHv;
        }
        double diag = 1.0, bm = 0.0, bp = 0.0, bm_next = 0.0;
        if (diff) {
            diag += c * (A_hi * dHu_hi - A_lo * dHv_lo) * iV;
            if (i + 1 < I) bp = c * A_hi * dHv_hi * iV;
            if (i > 0) bm = -c * A_lo * dHu_lo * iV;
            if (i + 1 < I) bm_next = -c * A_hi * dHu_hi * rcp_nr(V_hi) * lap_hi;
        }
        if (emabs) diag += c * sig_c;

        // ---- row k of Ahat_i = A_i - diag(bm_i) C_{i-1} (A^T for the transposed solve)
        //      NES part of A: -c dt [(1 - psi_k) K^in_{kk'} + psi_k K^out_{kk'}] for every k',
        //      diagonal: 1 + transport + c dt (eta + kappa_a) + c dt sum_k' [K^in psi + K^out (1 - psi)]
        T row[NT];                                     // assembled row (only kept for the transpose)
        T* acc = TRANS ? row : a;
        if constexpr (TRANS) {
#pragma unroll
            for (int kp = 0; kp < NT; ++kp) row[kp] = (T)0;
        } else {
            const T s0 = real ? (T)bm : (T)0;
#pragma unroll
            for (int kp = 0; kp < NT; ++kp) a[kp] = -s0 * a[kp];
        }
        if (nes) {
            const double amp = A.f.nes_amp[(size_t)sysz * I + i];
            const double Tz = tz[i];
            const T pk = (T)psi_c;
            const T ca = (T)(-c * amp);
            if constexpr (sizeof(T) == 4) {
                // FP32 Jacobian: exp(-|eps_k - eps_k'|/T) directly with the hardware exp2, all k' at once;
                // with M = that factor the NES entry is ca P (1 + w (M - 1)), w = psi_k above the diagonal
                // and 1 - psi_k below it, and the diagonal sum is P (1 + v (M - 1)), v = 1 - psi_k' above
                // and psi_k' below
                const float sc = (float)(1.4426950408889634 * rcp_nr(Tz));
                if (is_row) {
                    L.bc[k] = real ? (T)psi_c : (T)0;
                    L.dd[k] = (float)eps_k * sc;
                }
                wave_sync();
                const float xk = (float)eps_k * sc;
                T ds = (T)0;
#pragma unroll
                for (int kp = 0; kp < NT; ++kp) {
                    const float d = L.dd[kp] - xk;           // > 0 above the diagonal
                    const float tM = __builtin_amdgcn_exp2f(-fabsf(d)) - 1.0f;
                    const float pp = L.bc[kp];
                    const bool up = d > 0.0f;
                    const float w = up ? pk : 1.0f - pk;
                    const float v = up ? 1.0f - pp : pp;
                    acc[kp] = fma(ca * Prow[kp], fma(w, tM, 1.0f), acc[kp]);
                    ds = fma(Prow[kp], fma(v, tM, 1.0f), ds);
                }
                diag += c * amp * (double)ds;
            } else {
                if (is_row) {
                    L.bc[k] = real ? (T)psi_c : (T)0;
                    L.dd[k] = live ? wsY[(size_t)i * zs + lo] : (T)0;
                }
                wave_sync();
                const T cap = ca * pk, cam = ca * ((T)1 - pk);
                // out factor: exp(-(eps_k' - eps_k)/T) for k' > k, 1 otherwise (ascending product)
                T er = (T)1, so = (T)0, si = (T)0;
#pragma unroll
                for (int kp = 0; kp < NT; ++kp) {
                    if (kp > 0) er = (kp > kz) ? er * L.dd[kp - 1] : (T)1;
                    const T po = Prow[kp] * er;
                    so = fma(po, (T)1 - L.bc[kp], so);
                    acc[kp] = fma(cap, po, acc[kp]);           // - c dt psi_k K^out_{kk'}
                }
                // in factor: exp(-(eps_k - eps_k')/T) for k' < k, 1 otherwise (descending product)
                T el = (T)1;
#pragma unroll
                for (int kp = NT - 1; kp >= 0; --kp) {
                    el = (kp < kz) ? el * L.dd[kp] : (T)1;
                    const T pi = Prow[kp] * el;
                    si = fma(pi, L.bc[kp], si);
                    acc[kp] = fma(cam, pi, acc[kp]);           // - c dt (1 - psi_k) K^in_{kk'}
                }
                diag += c * amp * (double)(si + so);
            }
        }
        // the diagonal: added here for the transposed or partially pivoted elimination; with diagonal
        // pivots it is added by the owning lane at its own elimination step (entry (k,k) is read by
        // nobody before that step, and the updates before it do not depend on it)
        T dg = real ? (T)diag : (T)1;
        if (TRANS || PIVOT) {
#pragma unroll
            for (int kp = 0; kp < NT; ++kp) acc[kp] = real ? acc[kp] + ((kp == kz) ? dg : (T)0)
                                                          : ((kp == kz) ? (T)1 : (T)0);
            dg = (T)0;
        } else if (!real) {
#pragma unroll
            for (int kp = 0; kp < NT; ++kp) acc[kp] = (T)0;                       // padded identity row
        }
        if (!real) bm = bp = bm_next = 0.0;

        // ---- right-hand side (and, for the transpose, the transposed block plus its Schur update)
        T g = real ? (T)(rsc.in * A.rhs[co + (size_t)i * N + kk]) : (T)0;
        T bcoef;
        if constexpr (!TRANS) {
            g = fma(-(T)bm, ycar, g);
            bcoef = (T)bp;
        } else {
            if (is_row) {
#pragma unroll
                for (int kp = 0; kp < NT; ++kp) L.fix[k][kp] = row[kp];
            }
            wave_sync();
            // the previous factor row, as this lane stored it at the end of the previous zone (read back
            // rather than held in registers through the assembly)
            const T s = real ? (T)bp_prev : (T)0;
            if constexpr (PAIRS) {
                T prev[NT];
                ws_row(i > 0 ? i - 1 : 0, i > 0 && store, false, prev);
#pragma unroll
                for (int m = 0; m < NT; ++m) a[m] = fma(-s, prev[m], is_row ? L.fix[m][kr] : (T)0);
            } else {
                const T* qp = wsC + (size_t)(i > 0 ? i - 1 : 0) * NT * zs + lo;
#pragma unroll
                for (int m = 0; m < NT; ++m) {
                    const T prev = (i > 0 && store && m < N) ? qp[(size_t)m * zs] : (T)0;
                    a[m] = fma(-s, prev, is_row ? L.fix[m][kr] : (T)0);
                }
            }
            wave_sync();
            g = fma(-s, ycar, g);
            bcoef = (T)bm_next;
        }

        // ---- in-place Gauss-Jordan on [Ahat | diag(b) | g]
        if constexpr (PIVOT) {
            // partial pivoting: packed-key max over the group, row ownership left permuted
            bool used = !is_row;
            T mypiv = (T)1;
            int mycol = 0;
#pragma unroll
            for (int cc = 0; cc < NT; ++cc) {
                const T ac = a[cc];
                const uint32_t key =
                    used ? 0u : ((abs_key_bits(ac) & ~(uint32_t)(SL - 1)) | (uint32_t)(SL - 1 - k));
                const uint32_t kmax = group_max<SL>(key);
                const int p = SL - 1 - (int)(kmax & (SL - 1));
                const bool isp = (k == p);
                if (isp) {
#pragma unroll
                    for (int j = 0; j < NT; ++j) L.prow[j] = a[j];
                    L.prow[NT] = g;
                    L.prow[NT + 1] = bcoef;
                }
                wave_sync();
                const T piv = L.prow[cc];
                zp |= (piv == (T)0);
                const T pinv = rcp_nr(piv);
                const T f = isp ? (T)0 : ac * pinv;
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    if (j != cc) a[j] = fma(-f, L.prow[j], a[j]);
                g = fma(-f, L.prow[NT], g);
                const T bpiv = L.prow[NT + 1];
                a[cc] = isp ? bpiv : -f * bpiv;
                if (isp) {
                    used = true;
                    mypiv = piv;
                    mycol = cc;
                }
                wave_sync();
            }
            // restore row ownership: the lane holding unknown mycol writes its scaled row in slot
            // order; slot sidx[m] (the step at which lane m was the pivot) holds column m of C
            if (is_row) {
                const T ip = rcp_nr(mypiv);
#pragma unroll
                for (int cc = 0; cc < NT; ++cc) L.fix[mycol][cc] = a[cc] * ip;
                L.fix[mycol][NT] = g * ip;
                L.sidx[k] = mycol;
            }
            wave_sync();
#pragma unroll
            for (int m = 0; m < NT; ++m) a[m] = is_row ? L.fix[kr][L.sidx[m]] : (T)0;
            ycar = is_row ? L.fix[kr][NT] : (T)0;
            wave_sync();
        } else {
            // diagonal pivots: step cc eliminates with row cc, so rows stay in natural order
            T mypiv = (T)1;
#pragma unroll
            for (int cc = 0; cc < NT; ++cc) {
                const bool isp = (kz == cc);
                if (isp) a[cc] += dg;                     // own diagonal, see above
                const T ac = a[cc];
                if (isp) {
#pragma unroll
                    for (int j = 0; j < NT; ++j) L.prow[j] = a[j];
                    L.prow[NT] = g;
                    L.prow[NT + 1] = bcoef;
                }
                wave_sync();
                const T piv = L.prow[cc];
                const T pinv = rcp_nr(piv);
                const T f = isp ? (T)0 : ac * pinv;
                // the guard key and the own pivot are kept current in every step: left alone, the
                // compiler defers both chains to the end of the zone and holds every step's values
                gkey = max(gkey, abs_key_bits(f));
                asm volatile("" : "+v"(gkey));
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    if (j != cc) a[j] = fma(-f, L.prow[j], a[j]);
                g = fma(-f, L.prow[NT], g);
                const T bpiv = L.prow[NT + 1];
                a[cc] = isp ? bpiv : -f * bpiv;
                mypiv = isp ? piv : mypiv;
                asm volatile("" : "+v"(mypiv));
                wave_sync();
            }
            zp |= !(fabs(mypiv) > (T)0) || !isfinite(mypiv);
            const T ip = rcp_nr(mypiv);
#pragma unroll
            for (int m = 0; m < NT; ++m) a[m] = is_row ? a[m] * ip : (T)0;
            ycar = is_row ? g * ip : (T)0;
        }

        if (store) {
            // non-temporal except where the transposed kernel reads the row back in the next zone
            if constexpr (PAIRS) {
                V2* q = reinterpret_cast<V2*>(wsC + (size_t)i * NT * zs) + lo;
#pragma unroll
                for (int j = 0; j < NT / 2; ++j)
                    if (2 * j < N) {
                        const V2 v = {a[2 * j], a[2 * j + 1]};
                        if (TRANS) q[(size_t)j * zs] = v;
                        else nt_store(q + (size_t)j * zs, v);
                    }
            } else {
                T* q = wsC + (size_t)i * NT * zs + lo;
#pragma unroll
                for (int m = 0; m < NT; ++m)
                    if (m < N) {
                        if (TRANS) q[(size_t)m * zs] = a[m];
                        else nt_store(q + (size_t)m * zs, a[m]);
                    }
            }
            nt_store(wsY + (size_t)i * zs + lo, ycar);
        }

        psi_c = psi_n1;
        sig_c = sig_n1;
        lam_c = lam_n1;
        dHu_lo = dHu_hi;
        dHv_lo = dHv_hi;
        bp_prev = bp;
    }

    // zero-pivot report and, for diagonal pivots, the growth guard (any lane of the system)
    const bool lane_bad = is_row && (zp || gkey > abs_key_bits((T)A.growth_limit));
    int lnb;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lnb));
    const long long sysb = system_of(lnb);
    const size_t cellb = (size_t)sysb * I * N;
    uint32_t any_bad;
    if constexpr (PIVOT) {
        any_bad = group_max<SL>(lane_bad ? 1u : 0u);
    } else {
        const unsigned long long b = __ballot(lane_bad);
        const unsigned long long gm = (SL == 64) ? ~0ull : ((1ull << SL) - 1ull);
        any_bad = ((b >> (sub * SL)) & gm) != 0ull;
    }
    bool skip = false;
    if constexpr (PIVOT) {
        if (live && k == 0 && any_bad && A.flags) A.flags[sysb] |= 4;
    } else {
        skip = any_bad != 0;                          // leave this system to the pivoting re-run
        if (live && k == 0 && any_bad) {
            if (A.guard) A.guard[sysb] = 1;
            if (A.flags) A.flags[sysb] |= 8;
        }
    }
    const bool store_out = store && !skip;

    // ---------------------------------------------------------------- backward sweep
    double* outp = A.psi_out ? A.psi_out + cellb : nullptr;
    double* xp = A.x ? A.x + cellb : nullptr;
    double* dxp = A.dx ? A.dx + cellb : nullptr;
    T cr[NT], crn[NT];
    T yv = (T)0, yn = (T)0;
    if constexpr (PAIRS) {
        ws_row(I - 1, real, true, cr);
    } else {
        const T* q = wsC + (size_t)(I - 1) * NT * zs + lo;
#pragma unroll
        for (int m = 0; m < NT; ++m) cr[m] = (real && m < N) ? nt_load(q + (size_t)m * zs) : (T)0;
    }
    yv = real ? nt_load(wsY + (size_t)(I - 1) * zs + lo) : (T)0;
    T dnext = (T)0;
    for (int i = I - 1; i >= 0; --i) {
        if (i > 0) {
            if constexpr (PAIRS) {
                ws_row(i - 1, real, true, crn);
            } else {
                const T* q = wsC + (size_t)(i - 1) * NT * zs + lo;
#pragma unroll
                for (int m = 0; m < NT; ++m) crn[m] = (real && m < N) ? nt_load(q + (size_t)m * zs) : (T)0;
            }
            yn = real ? nt_load(wsY + (size_t)(i - 1) * zs + lo) : (T)0;
        }
        T dl = yv;
        if (i + 1 < I) {
            if (is_row) L.bc[k] = dnext;
            wave_sync();
#pragma unroll
            for (int m = 0; m < NT; ++m) dl = fma(-cr[m], L.bc[m], dl);
            wave_sync();
        }
        if (store_out) {
            const size_t ci = (size_t)i * N + k;
            const double d = rsc.out * (double)dl;
            if (outp) {
                outp[ci] += d;
                if (dxp) dxp[ci] = d;
            } else {
                xp[ci] = d;
            }
        }
        dnext = dl;
#pragma unroll
        for (int m = 0; m < NT; ++m) cr[m] = crn[m];
        yv = yn;
    }
    if (live && !skip && k == 0 && A.psi_out) {
        if (A.iters) A.iters[sysb] += 1;
        if (A.pending) A.pending[sysb] = 1;               // trial psi + delta awaits the line search
        if (A.alpha) A.alpha[sysb] = 1.0;
    }
}


// waves per SIMD the register allocation is held to: two for the FP64 kernels with diagonal pivots (forward and
// transposed) up to 20 groups (they fit 256 VGPRs without scratch and run a third faster than at one), one
// otherwise
template <typename T, int NT, bool TRANS, bool PIVOT>
constexpr int factor_waves_per_eu() { return (sizeof(T) == 8 && NT <= 20 && !PIVOT) ? 2 : 1; }

template <typename T, int NT, bool TRANS, bool PIVOT, bool GEO>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GEO ? 1 : factor_waves_per_eu<T, NT, TRANS, PIVOT>())))
void k_factor(FactorArgs A) {
    factor_sweeps<T, NT, TRANS, PIVOT, true, GEO>(A);
}

// The float32 forward kernel with diagonal pivots (the mixed-precision Newton update) held to five waves per
// SIMD (95 VGPRs; its LDS allows five blocks per CU), four with the lapse terms, which spill at five: both fit
// without scratch, and left alone the compiler settles a few registers above 128 and runs three.
template <int NT, bool LAPSE, bool GEO>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GEO ? 2 : (LAPSE ? 4 : 5))))
void k_factor_f32(FactorArgs A) {
    factor_sweeps<float, NT, false, false, LAPSE, GEO>(A);
}

template <typename T, int NT, bool TR, bool PV, bool GEO>
static void launch_t(const FactorArgs& a, hipStream_t st) {
    constexpr int SL = lanes_per_system<NT, PV>();
    constexpr int SPB = (kBlock / 64) * (64 / SL);
    const long long blocks = (a.nsys + SPB - 1) / SPB;
    if constexpr (std::is_same<T, float>::value && !TR && !PV && NT <= 20) {
        if (a.f.lapse) hipLaunchKernelGGL((k_factor_f32<NT, true, GEO>), dim3((unsigned)blocks), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_factor_f32<NT, false, GEO>), dim3((unsigned)blocks), dim3(kBlock), 0, st, a);
    } else
        hipLaunchKernelGGL((k_factor<T, NT, TR, PV, GEO>), dim3((unsigned)blocks), dim3(kBlock), 0, st, a);
}

template <typename T, int NT, bool GEO>
static void launch_tp(const FactorArgs& a, bool tr, bool pv, hipStream_t st) {
    if (tr) {
        if (pv) launch_t<T, NT, true, true, GEO>(a, st);
        else launch_t<T, NT, true, false, GEO>(a, st);
    } else {
        if (pv) launch_t<T, NT, false, true, GEO>(a, st);
        else launch_t<T, NT, false, false, GEO>(a, st);
    }
}

template <int NT, bool GEO>
static void launch_nt(const FactorArgs& a, bool fp32, bool tr, bool pv, hipStream_t st) {
    if (fp32) launch_tp<float, NT, GEO>(a, tr, pv, st);
    else launch_tp<double, NT, GEO>(a, tr, pv, st);
}

// Launch of the lane kernels for every padded group count, GEO instantiations or not.
template <bool GEO>
static hipError_t launch_lane(const FactorArgs& a, bool fp32, bool transpose, bool pivot, hipStream_t st) {
    switch (padded_groups(a.sh.N)) {
        case 4: launch_nt<4, GEO>(a, fp32, transpose, pivot, st); break;
        case 8: launch_nt<8, GEO>(a, fp32, transpose, pivot, st); break;
        case 12: launch_nt<12, GEO>(a, fp32, transpose, pivot, st); break;
        case 16: launch_nt<16, GEO>(a, fp32, transpose, pivot, st); break;
        case 20: launch_nt<20, GEO>(a, fp32, transpose, pivot, st); break;
        case 24: launch_nt<24, GEO>(a, fp32, transpose, pivot, st); break;
        case 28: launch_nt<28, GEO>(a, fp32, transpose, pivot, st); break;
        case 32: launch_nt<32, GEO>(a, fp32, transpose, pivot, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tmk
