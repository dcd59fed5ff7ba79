// Float32 fused Jacobian assembly + block-Thomas factor/solve of the linearised transport step
// (eq. a62ae) with one (species, ray) system per quad of four lanes: the mixed-precision Newton
// update with diagonal pivots.
//
// Layout on the chip: a wavefront holds 16 systems, one per quad.  Lane q of a quad owns rows
// k = 4s + q (s = 0..R-1, R = NT/4) of the zone's dense NT x NT block, with the right-hand side and
// the B coefficient of each row, all in registers.  Every value another row needs comes from a
// lane of the same quad through a DPP quad broadcast (quad_perm [p,p,p,p]): the pivot row of each
// elimination step, the group values of the NES coupling and the back-substitution vector.  The
// pivot order is the diagonal one, so the lane and register of every broadcast are compile-time
// constants and the elimination touches neither LDS nor any cross-quad path.
//
// Per zone: the rows are assembled (flux-limited diffusion derivatives in FP64, emission and
// absorption, the dense NES block from the hardware exp2), the Schur complement
//   Ahat_i = A_i - diag(bm_i) C_{i-1}
// is formed from the previous factor still in registers, and an unnormalised in-place Gauss-Jordan
// elimination on [Ahat | diag(bp) | g] produces C_i = Ahat_i^{-1} diag(bp_i) and
// y_i = Ahat_i^{-1}(g_i - bm_i y_{i-1}); each row is divided by its pivot once at the end.  C_i and
// y_i go to the workspace with 1 KB coalesced stores per instruction; the backward sweep reads them
// back, forms x_i = y_i - C_i x_{i+1} and writes x or adds it to psi (Newton update, eq. a62aa).
// A growth guard on the multipliers (or a zero or non-finite pivot) leaves the system untouched and
// flags it for the partial-pivoting kernel, as in the one-row-per-lane kernel.
#include "tm_kernels.hpp"

namespace tmk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Broadcast lane P of every quad to the quad's four lanes.
template <int P>
__device__ __forceinline__ float qbc(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x),
                                                              P | (P << 2) | (P << 4) | (P << 6), 0xF, 0xF, true));
}
__device__ __forceinline__ float qbc(float x, int p) {     // p is a compile-time constant after unrolling
    switch (p & 3) {
        case 0: return qbc<0>(x);
        case 1: return qbc<1>(x);
        case 2: return qbc<2>(x);
        default: return qbc<3>(x);
    }
}

__device__ __forceinline__ float frcp(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

__device__ __forceinline__ double drcp1(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Derivatives of the limited flux H = -lam m (v - u) / (3 D m + lam |v - u|), m = max((u + v)/2, floor)
// (eqs. a59, a20) with respect to the two zone values, for the float32 Jacobian.  They depend on the
// states only through rho = (v - u) / m, which is formed in FP64 (occupations reach 1e-300):
//   dH/d(v - u) = -3 D lam / (3 D + lam |rho|)^2,  dH/dm = -lam^2 w |w|, w = rho / (3 D + lam |rho|).
struct FluxD {
    float dHu, dHv;
};
// With limiter 2 and limb = (1 + mu_nu)/2 > 0 the geometric piece is taken where it is the smaller factor,
// limb (3 D + lam |rho|) < lam |rho|; there H = -limb m sign(v - u) and dH/du = dH/dv = -limb sign / 2.
__device__ __forceinline__ FluxD flux_derivatives(double u, double v, float lam, float D3, double floor,
                                                  int limiter, float limb = -1.0f) {
    FluxD f;
    if (limiter == 0) {
        const float gl = lam / D3;
        f.dHu = gl;
        f.dHv = -gl;
        return f;
    }
    const double mean = 0.5 * (u + v);
    const double m = fmax(mean, floor);
    const double rho64 = (v - u) * drcp1(m);
    const float rho = (float)fmin(fmax(rho64, -1e30), 1e30);      // beyond 1e30 the limits are reached
    const float r = frcp(fmaf(lam, fabsf(rho), D3));
    const float dHd = -D3 * lam * r * r;
    const float w = rho * r;
    const float dHm = (mean > floor) ? -lam * lam * w * fabsf(w) : 0.0f;
    f.dHu = 0.5f * dHm - dHd;
    f.dHv = 0.5f * dHm + dHd;
    if (limiter == 2 && limb > 0.0f && rho != 0.0f && limb * fmaf(lam, fabsf(rho), D3) < lam * fabsf(rho)) {
        const float d = (mean > floor) ? (rho > 0.0f ? -0.5f * limb : 0.5f * limb) : 0.0f;
        f.dHu = d;
        f.dHv = d;
    }
    return f;
}

// (1 + mu_nu)/2 at radius R outside a neutrinosphere of radius rnu (eqs. a24-a26, beta = 0, no ray
// bending), -1 inside it; float32, for the Jacobian.
__device__ __forceinline__ float limb_f(double R, float rnu) {
    const float x = rnu / (float)R;
    return x < 1.0f ? 0.5f * (1.0f + sqrtf(fmaf(-x, x, 1.0f))) : -1.0f;
}

// Scheduling fence: keeps the fully unrolled sweeps from hoisting the loads and broadcasts of later
// steps over earlier ones, which would hold several steps' values live at once (and spill).
__device__ __forceinline__ void fence_sched() { __builtin_amdgcn_sched_barrier(0); }

// Element at a wave-uniform base plus a 32-bit byte offset: the address is a scalar base and one
// vector offset (global load/store with saddr), so no 64-bit address per lane and array is kept
// live through the zone loops.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T& at(T* base, uint32_t byte_off) {
    using G = __attribute__((address_space(1))) T;
    using GC = __attribute__((address_space(1))) char;
    return *(G*)((GC*)base + byte_off);
}
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T& at(const T* base, uint32_t byte_off) {
    using G = const __attribute__((address_space(1))) T;
    using GC = const __attribute__((address_space(1))) char;
    return *(G*)((GC*)base + byte_off);
}
// The same addressing for the factor workspace, with non-temporal stores and loads: C and y are written
// once per zone and read once in the backward sweep, hundreds of zones later, so caching them only
// evicts other data (measured: the launch 5% shorter).
template <typename T>
__device__ __forceinline__ void st_nt(T* base, uint32_t byte_off, T v) {
    using G = __attribute__((address_space(1))) T;
    using GC = __attribute__((address_space(1))) char;
    __builtin_nontemporal_store(v, (G*)((GC*)base + byte_off));
}
template <typename T>
__device__ __forceinline__ T ld_nt(const T* base, uint32_t byte_off) {
    using G = const __attribute__((address_space(1))) T;
    using GC = const __attribute__((address_space(1))) char;
    return __builtin_nontemporal_load((G*)((GC*)base + byte_off));
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}

}  // namespace

constexpr int kQuadBlock = 64;          // one wavefront per workgroup
constexpr int kQuadSystems = 16;        // systems per wavefront

// Workspace of the quad kernel, per wave group of 16 systems and zone: C as R * NT/4 runs of 64 float4
// (entries 4t .. 4t+3 of lane l's row slot s at [s NT/4 + t][l], one 16-byte store or load per lane and
// run), then y as R runs of 64 floats.  A group takes 16 * NT * (NT + 1) floats per zone, the same as 16
// slots of the one-row-per-lane layout.
// Splits x into bf16 parts: x = hi + lo up to 2^-17 |x| (NB = 3), or hi alone (NB = 1).  The matrix-core
// products from the parts are hi hi (NB = 1), or hi hi + hi lo + lo hi (NB = 3, about float32 accuracy:
// the lo lo term is below 2^-16 relative).
template <int NB>
__device__ __forceinline__ void bf16_parts(const float (&x)[8], bf8& hi, bf8& lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        hi[e] = (__bf16)x[e];
        if constexpr (NB == 3) lo[e] = (__bf16)(x[e] - (float)hi[e]);
    }
}
// Forms of the float32 NES block (template argument NES):
//   kNesExp2    entries and diagonal sums on the vector units, one exp2 per entry;
//   kNesWindow  the detailed-balance factor as row and column scalings inside an energy window (two
//               exp2 per row instead of one per entry), entries and diagonal sums on the vector units;
//   kNesBf16, kNesBf16x3  the window scalings for the entries, and the diagonal sums as bf16 matrix-core
//               contractions with float32 accumulation, one bf16 product per term or three (hi/lo parts).
enum NesForm : int { kNesExp2 = 0, kNesWindow = 1, kNesBf16 = 2, kNesBf16x3 = 3 };

template <int NT, bool LAPSE, bool MF, int NES>
__global__ __launch_bounds__(kQuadBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_factor_q(FactorArgs A) {
    // the windowed form runs on energy grids that admit it (checked by the setup kernel); a launch of the
    // exp2 form beside it takes the other grids
    constexpr int NB = NES == kNesBf16 ? 1 : NES == kNesBf16x3 ? 3 : 0;   // bf16 products per term
    if constexpr (NES != kNesExp2) {
        if (A.cs->nes_window == 0) return;
    } else {
        if (A.skip_if_window && A.cs->nes_window != 0) return;
    }
    constexpr int R = NT / 4;              // rows per lane
    constexpr int PS = NT + 4;             // LDS row stride of the NES shape (float4 aligned)
    __shared__ __align__(16) float s_P[NT * PS];
    __shared__ float s_eps[NT];                       // group energies (0 for padding groups)
    for (int j = threadIdx.x; j < NT * PS; j += kQuadBlock) {
        const int r = j / PS, c = j % PS;
        s_P[j] = c < NT ? (float)A.cs->P[r][c] : 0.0f;
    }
    for (int j = threadIdx.x; j < NT; j += kQuadBlock) s_eps[j] = j < A.sh.N ? (float)A.cs->eps[j] : 0.0f;
    __syncthreads();

    const int lane = threadIdx.x;
    const int sub = lane >> 2;
    const long long sb = (long long)blockIdx.x * kQuadSystems + sub;   // system within the batch
    const bool in_batch = sb < A.nsys;
    const long long sbc = in_batch ? sb : A.nsys - 1;
    const long long sys = A.sys0 + sbc;
    const bool live = in_batch && (A.active == nullptr || A.active[sys] != 0);
    if (__ballot(live) == 0) return;

    const Shape& sh = A.sh;
    const int N = sh.N, I = sh.I;
    const double c = sh.c_dt;
    const bool diff = sh.terms & kDiffusion, emabs = sh.terms & kEmAbs, nes = sh.terms & kNes;
    // addressing: wave-uniform bases (the wave's first system, the zone) plus per-lane 32-bit byte offsets
    const long long wsys0 = A.sys0 + (long long)blockIdx.x * kQuadSystems;     // the wave's first system
    const size_t wcell0 = (size_t)wsys0 * I * N;
    const double* ampw = uniform_ptr(A.f.nes_amp ? A.f.nes_amp + (size_t)wsys0 * I : nullptr);
    const long long wg = blockIdx.x;                                    // wave group of 16 systems
    float* wsC = uniform_ptr(reinterpret_cast<float*>(A.wsC) + (size_t)wg * kQuadSystems * I * NT * NT);
    float* wsY = uniform_ptr(reinterpret_cast<float*>(A.wsY) + (size_t)wg * kQuadSystems * I * NT);
    // The per-lane offsets, re-derived from an opaque lane id wherever a loop needs them (a few integer
    // operations per zone) rather than held in registers through the loops.  The system index is below
    // 2^31 (checked by the host), so 32-bit arithmetic serves.
    struct LaneGeo {
        int q;
        uint32_t lb, rb, tb, ab, wl;   // cell offset of row slot 0; edge, zone, sysz arrays; workspace run
    };
    auto geo = [&]() {
        int l;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
        const int sbl = (int)blockIdx.x * kQuadSystems + (l >> 2);
        const int sbcl = sbl < (int)A.nsys ? sbl : (int)A.nsys - 1;
        const int sysl = (int)A.sys0 + sbcl;
        const int lsub = sysl - (int)wsys0;                             // 0..15 (clamped lanes too)
        const int rayl = sysl % sh.R;
        LaneGeo g;
        g.q = l & 3;
        g.lb = (uint32_t)(lsub * I * N + g.q) * 8u;
        g.rb = (uint32_t)rayl * (uint32_t)(I + 1) * 8u;
        g.tb = (uint32_t)rayl * (uint32_t)I * 8u;
        g.ab = (uint32_t)(lsub * I) * 8u;
        g.wl = (uint32_t)l * 4u;
        return g;
    };

    // right-hand side scaling of the float32 solve (power of two near max |rhs| of the system), kept in
    // LDS with the other per-lane values that the zone loops read but registers need not hold
    __shared__ double s_rs[2][kQuadBlock];
    __shared__ float s_y[R][kQuadBlock];              // y_{i-1} of the lane's rows
    __shared__ __align__(16) float s_dg[R][kQuadBlock];
    __shared__ __align__(16) float s_psi[R][kQuadBlock];
    __shared__ float s_bp[R][kQuadBlock];
    {
        double rs_in = A.rhs_sign, rs_out = 1.0;
        if (A.rhs_max) {
            const double m = A.rhs_max[sys];
            if (m > 0.0 && m < INFINITY) {
                const int e = ilogb(m);
                rs_in = ldexp(A.rhs_sign, -e);
                rs_out = ldexp(1.0, e);
            }
        }
        s_rs[0][lane] = rs_in;
        s_rs[1][lane] = rs_out;
    }
    // neutrinosphere radius of the lane's rows, for the geometric limiter and the geometric outer boundary
    __shared__ float s_rnu[R][kQuadBlock];
    if (sh.limiter == 2 || sh.outer_bc == 2) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int k = 4 * s + (lane & 3);
            s_rnu[s][lane] = k < N ? (float)A.f.r_nu[(size_t)(sys / sh.R) * N + k] : 0.0f;
        }
    }


    // ---------------------------------------------------------------- forward sweep
    // rows of the block (C_{i-1} on entry to a zone, then Ahat_i) as float4 runs of columns: entry (s, j)
    // is a4[s][j / 4][j % 4], and each run is one 4x4 accumulator tile of the matrix-core update
    v4f a4[R][NT / 4];
#define AE(s_, j_) a4[s_][(j_) >> 2][(j_) & 3]
    float g[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        s_y[s][lane] = 0.0f;
#pragma unroll
        for (int j = 0; j < NT; ++j) AE(s, j) = 0.0f;
    }
    // derivatives of the flux through the zone's lower edge, carried from the previous zone in LDS
    // rather than in registers (one wavefront per workgroup: [which][row slot][lane])
    __shared__ float s_dh[2][R][kQuadBlock];
#pragma unroll
    for (int s = 0; s < R; ++s) s_dh[0][s][lane] = s_dh[1][s][lane] = 0.0f;
    float gmax = 0.0f;                 // largest |multiplier| (growth guard)
    bool zp = false;                   // a zero or non-finite pivot met

    // bf16 matrix-core form of the NES diagonal sums (NB > 0).  With U and L the strict upper and lower
    // triangles of the shape matrix P (the same for every zone and system), the diagonal sum of row k is
    //   ds_k = [U psi + L (1 - psi)]_k + Ei_k [U (E (1 - psi))]_k + E_k [L (Ei psi)]_k,
    // products of one constant 32 x 32 matrix with a column per system: v_mfma_f32_16x16x32_bf16 with
    // the wave's 16 systems as the 16 columns (A: lane i + 16 h holds row i, entries 8h..8h+7; B: lane
    // j + 16 h holds rows 8h..8h+7 of column j; C: lane j + 16 h holds rows 4h..4h+3 of column j).  The
    // columns are read from the quads' LDS rows ([k / 4][4 j + k % 4]: four consecutive rows of a system
    // are one float4), and each output lane adds -ca_j ds to the diagonal of its four rows in LDS.
    __shared__ __align__(16) float s_E[NES ? R : 1][kQuadBlock];
    __shared__ __align__(16) float s_Ei[NES ? R : 1][kQuadBlock];
    __shared__ float s_ca[kQuadSystems];
    auto nes_diagonal_mfma = [&]() {
        if constexpr (NB > 0) {
            // lane id from an opaque source, so that the operands built from it (the A tiles are the same
            // in every zone) are rebuilt per zone instead of being hoisted and held through the zone loop
            int l;
            asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
            const int j = l & 15, h = l >> 4;
            // rows 8h..8h+7 of column j: two float4 of the LDS rows, zero beyond the last row slot
            auto column = [&](const float (*arr)[kQuadBlock], float (&v)[8]) {
                const bool ok0 = 2 * h < R, ok1 = 2 * h + 1 < R;
                const v4f a = *reinterpret_cast<const v4f*>(&arr[ok0 ? 2 * h : 0][4 * j]);
                const v4f b = *reinterpret_cast<const v4f*>(&arr[ok1 ? 2 * h + 1 : 0][4 * j]);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = ok0 ? a[e] : 0.0f;
                    v[4 + e] = ok1 ? b[e] : 0.0f;
                }
            };
            constexpr int MT = (NT + 15) / 16;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int i = 16 * mt + j;                   // row of the A tile held by this lane
                const int slot = 4 * mt + h;                 // row slot of the C rows held by this lane
#pragma unroll
                for (int tri = 0; tri < 2; ++tri) {          // U, then L
#pragma unroll
                    for (int prod = 0; prod < 2; ++prod) {
                        // prod 0: U psi or L (1 - psi); prod 1: U (E (1 - psi)) or L (Ei psi), scaled by the
                        // row's Ei or E.  Each product is folded into the diagonal before the next starts, and
                        // with NB = 3 the bf16 parts of A are taken one at a time (part 0: hi against both
                        // parts of the column, part 1: lo against its hi part), so few registers are live.
                        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int part = 0; part < (NB == 3 ? 2 : 1); ++part) {
                            bf8 at8, bh, bl;
                            {
                                // A: row i of the triangle, entries 8h..8h+7 (a clamped read is masked)
                                const int ic = i < NT ? i : NT - 1, k0 = 8 * h < PS - 8 ? 8 * h : PS - 8;
                                const v4f pa = *reinterpret_cast<const v4f*>(&s_P[ic * PS + k0]);
                                const v4f pb = *reinterpret_cast<const v4f*>(&s_P[ic * PS + k0 + 4]);
#pragma unroll
                                for (int e = 0; e < 8; ++e) {
                                    const int kk = 8 * h + e;
                                    const bool in = i < NT && kk < NT && (tri == 0 ? kk > i : kk < i);
                                    const float v = in ? (e < 4 ? pa[e] : pb[e - 4]) : 0.0f;
                                    const __bf16 hi = (__bf16)v;
                                    at8[e] = part == 0 ? hi : (__bf16)(v - (float)hi);
                                }
                            }
                            float b8[8];
                            column(s_psi, b8);
                            if (prod == 0) {
#pragma unroll
                                for (int e = 0; e < 8; ++e) b8[e] = tri == 0 ? b8[e] : 1.0f - b8[e];
                            } else {
                                float x8[8];
                                column(tri == 0 ? s_E : s_Ei, x8);
#pragma unroll
                                for (int e = 0; e < 8; ++e) b8[e] = x8[e] * (tri == 0 ? 1.0f - b8[e] : b8[e]);
                            }
                            bf16_parts<NB>(b8, bh, bl);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(at8, bh, acc, 0, 0, 0);
                            if (NB == 3 && part == 0) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(at8, bl, acc, 0, 0, 0);
                            fence_sched();
                        }
                        // C: rows 16 mt + 4h .. +3 of system j
                        if (slot < R) {
                            v4f* dg = reinterpret_cast<v4f*>(&s_dg[slot][4 * j]);
                            const float nca = -s_ca[j];
                            v4f d = *dg;
                            if (prod == 0) {
#pragma unroll
                                for (int r = 0; r < 4; ++r) d[r] = fmaf(nca, acc[r], d[r]);
                            } else {
                                const v4f sc = *reinterpret_cast<const v4f*>(tri == 0 ? &s_Ei[slot][4 * j]
                                                                                     : &s_E[slot][4 * j]);
#pragma unroll
                                for (int r = 0; r < 4; ++r) d[r] = fmaf(nca * sc[r], acc[r], d[r]);
                            }
                            *dg = d;
                        }
                        fence_sched();
                    }
                }
            }
        }
    };

    // Software pipeline over zones: the cell values a zone's assembly needs are loaded into registers one
    // zone ahead (issued before the previous zone's elimination and factor stores, so that waiting for
    // them never waits for those stores); the values of the zone itself are carried in LDS from the zone
    // before (psi in FP64 for the limiter ratio, the float32 sigma = kappa_a + eta and lambda).
    __shared__ double s_cpsi[R][kQuadBlock];
    __shared__ float s_csig[R][kQuadBlock], s_clam[R][kQuadBlock];
    struct Ahead {                     // prefetched for zone i: cells of zone i+1, rhs of zone i, scalars of zone i
        double psi[R], ka[R], et[R], ks[R], rhs[R];
        double r2, T, amp, az, ae;     // r_{i+2}; T_i; amp_i; lapse a_i and a_{i+3/2}
    };
    // loads of the values zone `z` needs (cells of z+1 when it exists, rhs of z, edges and zone scalars)
    auto fetch = [&](int z) {
        Ahead f;
        const LaneGeo gz = geo();
        const bool nxt = z + 1 < I;
        const size_t zn = wcell0 + (size_t)(nxt ? z + 1 : z) * N;
        const double* pz = uniform_ptr(A.psi + zn);
        const double* kz = uniform_ptr(A.f.kappa_a + zn);
        const double* ez = uniform_ptr(A.f.eta + zn);
        const double* sz = uniform_ptr(A.f.kappa_s + zn);
        const double* rz = uniform_ptr(A.rhs + wcell0 + (size_t)z * N);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int k = 4 * s + gz.q;
            const uint32_t o = k < N ? gz.lb + 32u * s : gz.lb - 8u * gz.q;    // padding rows read group 0
            f.psi[s] = at(pz, o);
            f.ka[s] = at(kz, o);
            f.et[s] = at(ez, o);
            f.ks[s] = at(sz, o);
            f.rhs[s] = at(rz, o);
        }
        f.r2 = nxt ? at(uniform_ptr(A.f.r_edge + z + 2), gz.rb) : 0.0;
        f.T = nes ? at(uniform_ptr(A.f.temp + z), gz.tb) : 1.0;
        f.amp = nes ? at(ampw + z, gz.ab) : 0.0;
        f.az = LAPSE ? at(uniform_ptr(A.f.lapse + z), gz.tb) : 1.0;
        f.ae = LAPSE ? at(uniform_ptr(A.f.lapse_edge + z + 1), gz.rb) : 1.0;
        return f;
    };
    double r0, r1, e0 = 1.0;           // edges r_i, r_{i+1} and the lapse at r_i
    {
        const LaneGeo gz = geo();
        const double* pz = uniform_ptr(A.psi + wcell0);
        const double* kz = uniform_ptr(A.f.kappa_a + wcell0);
        const double* ez = uniform_ptr(A.f.eta + wcell0);
        const double* sz = uniform_ptr(A.f.kappa_s + wcell0);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int k = 4 * s + gz.q;
            const bool real = k < N;
            const uint32_t o = real ? gz.lb + 32u * s : gz.lb - 8u * gz.q;
            const double p = at(pz, o), ka = at(kz, o), et = at(ez, o), ks = at(sz, o);
            s_cpsi[s][lane] = real ? p : 0.0;
            s_csig[s][lane] = real ? (float)(ka + et) : 0.0f;
            s_clam[s][lane] = frcp((float)(ka + et + ks));
        }
        const double* re = uniform_ptr(A.f.r_edge);
        r0 = at(re, gz.rb);
        r1 = at(re, gz.rb + 8u);
        if (LAPSE) e0 = at(uniform_ptr(A.f.lapse_edge), gz.rb);
    }
    Ahead ah;                          // zone 0's values are loaded at the top of its iteration

    for (int i = 0; i < I; ++i) {
        if (i == 0) ah = fetch(0);
        const LaneGeo gz = geo();
        const int q = gz.q;
        const uint32_t wl1 = gz.wl;
        double iV = drcp1(shell_volume(r0, r1));
        double A_lo = r0 * r0, A_hi = r1 * r1;
        if (LAPSE) {                   // eq. a58 times a_i c dt: a^3 / V and A / a^2
            iV *= ah.az * ah.az * ah.az;
            A_lo /= e0 * e0;
            A_hi /= ah.ae * ah.ae;
        }
        // c dt A / V of both edges and 3 D of the upper edge, in float32 (Jacobian entries only)
        const float cA_lo = (float)(c * A_lo * iV), cA_hi = (float)(c * A_hi * iV);
        const float D3 = i + 1 < I ? (float)(3.0 * (0.5 * (r1 + ah.r2) - 0.5 * (r0 + r1))) : 0.0f;

        // ---- per-row diffusion and emission/absorption terms, Schur scaling, right-hand side
        // per-row values handed from the assembly to the NES block and the elimination go through LDS
        // ([row slot][lane]: a quad's rows of slot s are the four consecutive lanes)
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int k = 4 * s + q;
            const bool real = k < N;
            const double psi_c = s_cpsi[s][lane];
            const float sig_c = s_csig[s][lane];
            float dHu_hi = 0.0f, dHv_hi = 0.0f;
            if (i + 1 < I) {                                             // uniform branch
                const double psi_n = real ? ah.psi[s] : 0.0;
                const float sig_n = real ? (float)(ah.ka[s] + ah.et[s]) : 0.0f;
                const float lam_n = frcp((float)(ah.ka[s] + ah.et[s] + ah.ks[s]));
                if (diff) {
                    const FluxD e = flux_derivatives(psi_c, psi_n, sqrtf(s_clam[s][lane] * lam_n), D3,
                                                     sh.psi_floor, sh.limiter,
                                                     sh.limiter == 2 ? limb_f(r1, s_rnu[s][lane]) : -1.0f);
                    dHu_hi = real ? e.dHu : 0.0f;
                    dHv_hi = real ? e.dHv : 0.0f;
                }
                // the next zone's own values (each lane reads and writes only its own slots)
                s_cpsi[s][lane] = psi_n;
                s_csig[s][lane] = sig_n;
                s_clam[s][lane] = lam_n;
            } else if (sh.outer_bc == 1) {
                dHu_hi = 1.0f;         // free streaming: H = psi of the last zone
            } else if (sh.outer_bc == 2 && diff) {
                // ghost zone of eq. a62af (R_nu squared): psi_{I+1} = ratio psi_I at the mirror centre
                const double rnu = s_rnu[s][lane];
                const double RI = 0.5 * (r0 + r1), Rg = 2.0 * r1 - RI, qn = 0.25 * rnu * rnu;
                const double den = Rg * Rg - qn;
                const double ratio = den > 0.0 ? fmin(fmax((RI * RI - qn) / den, 0.0), 1.0) : 0.0;
                const FluxD e = flux_derivatives(psi_c, ratio * psi_c, s_clam[s][lane], (float)(3.0 * (Rg - RI)),
                                                 sh.psi_floor, sh.limiter,
                                                 sh.limiter == 2 ? limb_f(r1, (float)rnu) : -1.0f);
                dHu_hi = real ? e.dHu + (float)ratio * e.dHv : 0.0f;
            }
            float diag = 1.0f, bm = 0.0f, bp = 0.0f;
            if (diff) {
                const float dHu_lo = s_dh[0][s][lane], dHv_lo = s_dh[1][s][lane];
                diag += cA_hi * dHu_hi - cA_lo * dHv_lo;
                bp = cA_hi * dHv_hi;
                bm = -cA_lo * dHu_lo;
            }
            if (emabs) diag = fmaf((float)c, sig_c, diag);
            s_dh[0][s][lane] = dHu_hi;
            s_dh[1][s][lane] = dHv_hi;
            if (!real) {
                diag = 1.0f;           // padded identity row
                bm = bp = 0.0f;
            }
            s_dg[s][lane] = diag;
            s_bp[s][lane] = bp;
            s_psi[s][lane] = (float)psi_c;
            // Schur update: row k of -diag(bm) C_{i-1}, right-hand side minus bm y_{i-1}
#pragma unroll
            for (int j = 0; j < NT; ++j) AE(s, j) = -bm * AE(s, j);
            g[s] = real ? (float)(s_rs[0][lane] * ah.rhs[s]) : 0.0f;
            g[s] = fmaf(-bm, s_y[s][lane], g[s]);
            fence_sched();
        }
        const double Tz = ah.T, ampz = ah.amp;
        r0 = r1;
        r1 = ah.r2;
        if (LAPSE) e0 = ah.ae;
        wave_sync();                   // the quad's row values in LDS are read by the other lanes below
        if constexpr (NES != kNesExp2) {
            // window scalings (and the matrix-core NES diagonal sums), before the next zone's loads take
            // their registers
            if (nes) {
                // Energy window of the system: the groups with x = eps log2(e) / T within 200 of group 0.
                // Inside it M = 2^-|x_k - x_k'| is the product of the scalings E = 2^(xm - x) and
                // Ei = 2^(x - xm), xm = x_0 + 100 (both within 2^+-100).  Any pair with a member outside
                // has |x_k - x_k'| >= 200 (1 - eps_{k-1}/eps_k), at least 40 when adjacent groups differ
                // by 25% (the setup kernel checks the grid; on other grids the exp2 form runs), so
                // M < 2^-40 there and is taken as 0.
                const float xs = (float)(1.4426950408889634 * drcp1(Tz));
                const float x0 = s_eps[0] * xs, xm = x0 + 100.0f;
#pragma unroll
                for (int s = 0; s < R; ++s) {
                    const float x = s_eps[4 * s + q] * xs;
                    const bool w = (4 * s + q < N) && (x - x0 <= 200.0f);
                    s_E[s][lane] = w ? __builtin_amdgcn_exp2f(xm - x) : 0.0f;
                    s_Ei[s][lane] = w ? __builtin_amdgcn_exp2f(x - xm) : 0.0f;
                }
                if constexpr (NB > 0) {
                    if (q == 0) s_ca[lane >> 2] = (float)(-c * ampz);
                    wave_sync();
                    nes_diagonal_mfma();
                    wave_sync();
                }
                fence_sched();
            }
        }
        // the next zone's values are requested now, ahead of this zone's elimination and factor stores
        // (the windowed form after its NES entries, which then have the registers to themselves)
        if (NES == kNesExp2 && i + 1 < I) ah = fetch(i + 1);

        // ---- NES block: -c dt [(1 - psi_k) K^in_{kk'} + psi_k K^out_{kk'}] off the diagonal, and the
        //      diagonal sum c dt sum_k' [K^in psi_k' + K^out (1 - psi_k')].  With M = exp(-|eps_k - eps_k'|/T)
        //      the entry is ca P (1 + w (M - 1)), w = psi_k above the diagonal and 1 - psi_k below it, and the
        //      diagonal term is P (1 + v (M - 1)), v = 1 - psi_k' above and psi_k' below.
        if (nes) {
            const float ca = (float)(-c * ampz);
            const float xs = (float)(1.4426950408889634 * drcp1(Tz));  // log2 e / T
            if constexpr (NES == kNesExp2) {
                // Split by the weights: above the diagonal (k' > k) the entry is ca P [(1 - psi_k) + psi_k M] and
                // the diagonal term P [psi_k' + (1 - psi_k') M]; below it psi and 1 - psi trade places.  Whether
                // k' > k is known at compile time except inside the row's own run of four columns (P is 0 on
                // the diagonal and in padding rows and columns, so their side does not matter).
                float xl[R], ds[R], wa[R], wb[R];
#pragma unroll
                for (int s = 0; s < R; ++s) {
                    xl[s] = s_eps[4 * s + q] * xs;
                    ds[s] = 0.0f;
                    wa[s] = ca * s_psi[s][lane];           // ca psi_k
                    wb[s] = ca - wa[s];                    // ca (1 - psi_k)
                }
#pragma unroll
                for (int kp = 0; kp < NT; ++kp) {
                    const float xb = qbc(xl[kp / 4], kp % 4);
                    const float pb = s_psi[kp / 4][(lane & ~3) + kp % 4];
                    const float pc = 1.0f - pb;
#pragma unroll
                    for (int s = 0; s < R; ++s) {
                        const float P = s_P[(4 * s + q) * PS + kp];
                        const float PM = P * __builtin_amdgcn_exp2f(-fabsf(xb - xl[s]));
                        const bool up = kp >= 4 * s + 4 ? true : kp < 4 * s ? false : kp > 4 * s + q;
                        const float c1 = up ? wb[s] : wa[s], c2 = up ? wa[s] : wb[s];
                        const float v1 = up ? pb : pc, v2 = up ? pc : pb;
                        AE(s, kp) = fmaf(c2, PM, fmaf(c1, P, AE(s, kp)));
                        ds[s] = fmaf(v2, PM, fmaf(v1, P, ds[s]));
                    }
                    fence_sched();
                }
#pragma unroll
                for (int s = 0; s < R; ++s) s_dg[s][lane] = fmaf(-ca, ds[s], s_dg[s][lane]);
            } else {
                // entries with M from the energy-window scalings (and, in the matrix-core forms, the diagonal
                // sums already formed above)
                float E[R], Ei[R], ds[R];                    // this zone's scalings, from LDS
#pragma unroll
                for (int s = 0; s < R; ++s) {
                    E[s] = s_E[s][lane];
                    Ei[s] = s_Ei[s][lane];
                    ds[s] = 0.0f;
                }
#pragma unroll
                for (int kp = 0; kp < NT; ++kp) {
                    const float eb = qbc(E[kp / 4], kp % 4), eib = qbc(Ei[kp / 4], kp % 4);
                    const float pb = NES == kNesWindow ? s_psi[kp / 4][(lane & ~3) + kp % 4] : 0.0f;
#pragma unroll
                    for (int s = 0; s < R; ++s) {
                        const int k = 4 * s + q;
                        const float P = s_P[k * PS + kp];
                        const bool up = kp > k;
                        const float tM = (up ? eb * Ei[s] : E[s] * eib) - 1.0f;
                        const float ps = s_psi[s][lane];
                        const float w = up ? ps : 1.0f - ps;
                        AE(s, kp) = fmaf(ca * P, fmaf(w, tM, 1.0f), AE(s, kp));
                        if constexpr (NES == kNesWindow) {
                            const float v = up ? 1.0f - pb : pb;
                            ds[s] = fmaf(P, fmaf(v, tM, 1.0f), ds[s]);
                        }
                    }
                    fence_sched();
                }
                if constexpr (NES == kNesWindow) {
#pragma unroll
                    for (int s = 0; s < R; ++s) s_dg[s][lane] = fmaf(-ca, ds[s], s_dg[s][lane]);
                }
            }
        }
        if (NES != kNesExp2 && i + 1 < I) {
            fence_sched();
            ah = fetch(i + 1);
        }
        // the diagonal: entry (k, k) of slot s sits in column 4s + q, one of the four columns 4s..4s+3
#pragma unroll
        for (int s = 0; s < R; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t) AE(s, 4 * s + t) += (q == t) ? s_dg[s][lane] : 0.0f;
        fence_sched();

        // ---- in-place Gauss-Jordan with diagonal pivots: step cc eliminates with row cc, held by lane
        //      cc % 4 in register row cc / 4
        float pv[R];
#pragma unroll
        for (int s = 0; s < R; ++s) pv[s] = 1.0f;
#pragma unroll
        for (int cc = 0; cc < NT; ++cc) {
            const int p = cc % 4, sp = cc / 4;
            const bool own = q == p;
            const float piv = qbc(AE(sp, cc), p);
            const float npinv = -frcp(piv);
            pv[sp] = own ? piv : pv[sp];
            float nf[R];                                   // minus the multipliers
#pragma unroll
            for (int s = 0; s < R; ++s) {
                nf[s] = AE(s, cc) * npinv;
                if (s == sp) nf[s] = own ? 0.0f : nf[s];
                gmax = fmaxf(gmax, fabsf(nf[s]));
            }
            if constexpr (MF) {
                // rank-1 update on the matrix cores: tile (s, t) holds entries (4s + q, 4t + i) in register i
                // of lane q, so v_mfma_f32_4x4x1f32 (one 4x4 block per quad) with A = the pivot row's entry
                // 4t + i from lane i and B = -f of the lane's own row adds -f_r u_c to every entry.  Lane i
                // takes entry 4t + i of the broadcast pivot row (a 4-way select on the quad lane).
                const bool q1 = q & 1, q2 = q & 2;
                // tiles in the order the next step needs them: the one holding column cc + 1 (the next
                // multipliers and pivot) first
#pragma unroll
                for (int tt = 0; tt < NT / 4; ++tt) {
                    const int t = ((cc + 1) / 4 + tt) % (NT / 4);
                    const float b0 = qbc(AE(sp, 4 * t), p), b1 = qbc(AE(sp, 4 * t + 1), p);
                    const float b2 = qbc(AE(sp, 4 * t + 2), p), b3 = qbc(AE(sp, 4 * t + 3), p);
                    const float ut = q2 ? (q1 ? b3 : b2) : (q1 ? b1 : b0);
#pragma unroll
                    for (int s2 = 0; s2 < R; ++s2) a4[s2][t] = __builtin_amdgcn_mfma_f32_4x4x1f32(ut, nf[s2], a4[s2][t], 0, 0, 0);
                    if (tt % 2 == 1) fence_sched();    // a few pivot-row tiles in flight at a time
                }
            } else {
                // columns in the order the next step needs them: column cc + 1 (the next multipliers and
                // pivot) first, so that the next step's pivot chain can overlap this step's tail
#pragma unroll
                for (int jj = 1; jj < NT; ++jj) {
                    const int j = (cc + jj) % NT;
                    const float u = qbc(AE(sp, j), p);
#pragma unroll
                    for (int s = 0; s < R; ++s) AE(s, j) = fmaf(nf[s], u, AE(s, j));
                }
            }
            const float ug = qbc(g[sp], p);
#pragma unroll
            for (int s = 0; s < R; ++s) g[s] = fmaf(nf[s], ug, g[s]);
            const float bpiv = s_bp[sp][(lane & ~3) + p];
#pragma unroll
            for (int s = 0; s < R; ++s) AE(s, cc) = nf[s] * bpiv;
            AE(sp, cc) = own ? bpiv : AE(sp, cc);
        }
#pragma unroll
        for (int s = 0; s < R; ++s) {
            zp |= !(fabsf(pv[s]) > 0.0f) || !isfinite(pv[s]);
            const float ip = frcp(pv[s]);
#pragma unroll
            for (int j = 0; j < NT; ++j) AE(s, j) *= ip;
            g[s] *= ip;
            s_y[s][lane] = g[s];
        }

        // every quad stores its slot (no branch): a clamped quad repeats the batch's last system and
        // writes the same values to that system's slot
        {
            float* qc = uniform_ptr(wsC + (size_t)i * kQuadSystems * NT * NT);
#pragma unroll
            for (int s = 0; s < R; ++s)
#pragma unroll
                for (int t = 0; t < NT / 4; ++t) st_nt(reinterpret_cast<v4f*>(qc) + (s * (NT / 4) + t) * 64, 4u * wl1, a4[s][t]);
            float* qy = uniform_ptr(wsY + (size_t)i * kQuadSystems * NT);
#pragma unroll
            for (int s = 0; s < R; ++s) st_nt(qy + s * 64, wl1, g[s]);
        }
    }

    // ---- growth guard and zero pivots (any lane of the quad)
    const bool lane_bad = zp || !(gmax <= (float)A.growth_limit);
    const unsigned long long bad = __ballot(lane_bad);
    bool any_bad, store_out;
    {
        int l;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
        any_bad = ((bad >> (l & ~3)) & 0xFull) != 0ull;
        const long long sbl = (long long)blockIdx.x * kQuadSystems + (l >> 2);
        const long long sysl = A.sys0 + (sbl < A.nsys ? sbl : A.nsys - 1);
        const bool livel = sbl < A.nsys && (A.active == nullptr || A.active[sysl] != 0);
        if (livel && (l & 3) == 0 && any_bad) {
            if (A.guard) A.guard[sysl] = 1;
            if (A.flags) A.flags[sysl] |= 8;
        }
        store_out = livel && !any_bad;
    }

    // ---------------------------------------------------------------- backward sweep
    // pipelined like the forward sweep: zone i-1's factors (and, for a Newton update, its psi) are loaded
    // before zone i's back substitution and output stores
    struct Behind {
        v4f c[R][NT / 4];
        float y[R];
        double ps[R];
    };
    auto fetch_back = [&](int z) {
        Behind b;
        const LaneGeo gz = geo();
        const float* qc = uniform_ptr(wsC + (size_t)z * kQuadSystems * NT * NT);
        const float* qy = uniform_ptr(wsY + (size_t)z * kQuadSystems * NT);
        const double* pz = A.psi_out ? uniform_ptr(A.psi_out + wcell0 + (size_t)z * N) : nullptr;
#pragma unroll
        for (int s = 0; s < R; ++s) {
            b.y[s] = ld_nt(qy + s * 64, gz.wl);
#pragma unroll
            for (int t = 0; t < NT / 4; ++t) b.c[s][t] = ld_nt(reinterpret_cast<const v4f*>(qc) + (s * (NT / 4) + t) * 64, 4u * gz.wl);
            const int k = 4 * s + gz.q;
            b.ps[s] = pz ? at(pz, k < N ? gz.lb + 32u * s : gz.lb - 8u * gz.q) : 0.0;
        }
        return b;
    };
    float dn[R];                       // x_{i+1} of the lane's rows
#pragma unroll
    for (int s = 0; s < R; ++s) dn[s] = 0.0f;
    Behind bh = fetch_back(I - 1);
    for (int i = I - 1; i >= 0; --i) {
        Behind nb;
        if (i > 0) nb = fetch_back(i - 1);
        const LaneGeo gz = geo();
        const uint32_t lb = gz.lb;
        const int q = gz.q;
        float dl[R];
#pragma unroll
        for (int s = 0; s < R; ++s) dl[s] = bh.y[s];
        if (i + 1 < I) {
#pragma unroll
            for (int m = 0; m < NT; ++m) {
                const float xm = qbc(dn[m / 4], m % 4);
#pragma unroll
                for (int s = 0; s < R; ++s) dl[s] = fmaf(-bh.c[s][m / 4][m % 4], xm, dl[s]);
            }
        }
        if (store_out) {
            const size_t zc = wcell0 + (size_t)i * N;
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int k = 4 * s + q;
                if (k < N) {
                    const uint32_t o = lb + 32u * s;
                    const double d = s_rs[1][lane] * (double)dl[s];
                    if (A.psi_out) {
                        at(uniform_ptr(A.psi_out + zc), o) = bh.ps[s] + d;
                        if (A.dx) at(uniform_ptr(A.dx + zc), o) = d;
                    } else {
                        at(uniform_ptr(A.x + zc), o) = d;
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < R; ++s) dn[s] = dl[s];
        if (i > 0) bh = nb;
    }
    {
        int l;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
        const long long sbl = (long long)blockIdx.x * kQuadSystems + (l >> 2);
        const long long sysl = A.sys0 + (sbl < A.nsys ? sbl : A.nsys - 1);
        if (store_out && (l & 3) == 0 && A.psi_out) {
            if (A.iters) A.iters[sysl] += 1;
            if (A.pending) A.pending[sysl] = 1;  // trial psi + delta awaits the line search
            if (A.alpha) A.alpha[sysl] = 1.0;
        }
    }
}

// Launch of the quad kernel for the float32 forward solve with diagonal pivots (NT <= 20); returns
// false when the shape is not covered (the caller then uses the one-row-per-lane kernel).  A windowed
// NES form is launched together with the exp2 form of the same elimination, which runs instead of it
// on energy grids that do not admit the window (the setup kernel's flag decides on the device).
bool launch_factor_quad(const FactorArgs& a, hipStream_t st, int kernel) {
    const unsigned blocks = (unsigned)((a.nsys + kQuadSystems - 1) / kQuadSystems);
    const bool lp = a.f.lapse != nullptr;
    FactorArgs ax = a;
    ax.skip_if_window = 1;
    switch (padded_groups(a.sh.N)) {
#define TM_QUAD_LAUNCH(NTV, LP, MFV, NESV, ARGS) \
    hipLaunchKernelGGL((k_factor_q<NTV, LP, MFV, NESV>), dim3(blocks), dim3(kQuadBlock), 0, st, ARGS)
#define TM_QUAD_WIN(NTV, LP, NESV)                   \
    TM_QUAD_LAUNCH(NTV, LP, false, NESV, a);         \
    TM_QUAD_LAUNCH(NTV, LP, false, kNesExp2, ax);
#define TM_QUAD_LP(NTV, LP)                                                        \
    switch (kernel) {                                                              \
        case kFactorQuadMfma: TM_QUAD_LAUNCH(NTV, LP, true, kNesExp2, a); break;   \
        case kFactorQuadValu: TM_QUAD_LAUNCH(NTV, LP, false, kNesExp2, a); break;  \
        case kFactorQuadBf16x3: TM_QUAD_WIN(NTV, LP, kNesBf16x3) break;            \
        case kFactorQuadBf16: TM_QUAD_WIN(NTV, LP, kNesBf16) break;                \
        default: TM_QUAD_WIN(NTV, LP, kNesWindow) break;                           \
    }
#define TM_QUAD_CASE(NTV)             \
    case NTV:                         \
        if (lp) TM_QUAD_LP(NTV, true) \
        else TM_QUAD_LP(NTV, false)   \
        return true;
        TM_QUAD_CASE(4)
        TM_QUAD_CASE(8)
        TM_QUAD_CASE(12)
        TM_QUAD_CASE(16)
        TM_QUAD_CASE(20)
#undef TM_QUAD_CASE
#undef TM_QUAD_LP
#undef TM_QUAD_WIN
#undef TM_QUAD_LAUNCH
        default: return false;
    }
}

}  // namespace tmk
