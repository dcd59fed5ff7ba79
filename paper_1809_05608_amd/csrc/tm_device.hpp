// Internal device-side definitions shared by the libtm kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmk {

constexpr double kEps0 = 10.0;                 // NES kernel energy scale (MeV)
constexpr double kCLight = 2.99792458e10;      // cm/s, for the number luminosity
constexpr int kMaxN = 32;
constexpr int kBlock = 256;                    // threads per block for every kernel

// Grid constants shared by all systems, filled once per call by k_setup:
//   eps[k]  group centre (eq. a01 with eps_k^2 on the left)
//   W[k]    phase-space weight (eq. a01b)
//   de[k]   eps[k+1] - eps[k]
//   P[k][k'] = (eps_k eps_k' / eps0^2) nes_g[k][k'] W_k' / mean(W)   (NES kernel without amplitude
//              and without the detailed-balance factor); P[k][k] = 0 because scattering within a
//              group has no zeroth-moment source (its in and out terms cancel identically)
struct Consts {
    double eps[kMaxN];
    double W[kMaxN];
    double de[kMaxN];
    double P[kMaxN][kMaxN];
    int nes_window;   // 1 when every group energy is at least 1.25 times the one below it
    double wbar;      // mean group weight, sum_k W_k / N
};

struct Shape {
    int S, R, I, N;
    double c_dt;
    int outer_bc;      // 0 zero flux, 1 free streaming, 2 geometric ghost zone (eq. a62af)
    unsigned terms;    // TM_TERM_* bits
    int limiter;       // 0 none, 1 F_intrp, 2 min(F_intrp, F_geom)
    double psi_floor;
};

// Per-call pointers (device).  Cell arrays are [S][R][I][N].
struct Fields {
    const double* r_edge;   // [R][I+1]
    const double* kappa_a;
    const double* eta;
    const double* kappa_s;
    const double* temp;     // [R][I]
    const double* nes_amp;  // [S][R][I]
    const double* lapse;        // [R][I] lapse at zone centres, or nullptr (a = 1)
    const double* lapse_edge;   // [R][I+1] lapse at zone edges (set together with lapse)
    const double* r_nu;         // [S][N] neutrinosphere radius per species and group (limiter 2, outer_bc 2)
};

// Lapse factors of eq. a58 times a_i c dt: the flux difference of zone i carries a_i^3 / V_i and the
// area of edge e becomes A_e / a_e^2 (the sources' factor a_i is folded into the inputs by the host).
__device__ __forceinline__ double lapse_zone3(const Fields& f, size_t zone) {
    if (!f.lapse) return 1.0;
    const double a = f.lapse[zone];
    return a * a * a;
}
__device__ __forceinline__ double lapse_edge_inv2(const Fields& f, size_t edge) {
    if (!f.lapse_edge) return 1.0;
    const double a = f.lapse_edge[edge];
    return 1.0 / (a * a);
}

constexpr unsigned kDiffusion = 1u, kEmAbs = 2u, kNes = 4u;

// Electron-fraction coupling (eq. a62a): zeta = 4 pi m_B / ((hc)^3 rho) turns sum_k W_k psi (MeV^3)
// into neutrinos per baryon.  m_B is taken as the atomic mass unit; both constants are CODATA 2018.
constexpr double kBaryonMassG = 1.66053906660e-24;    // g
constexpr double kHcMeVCm = 1.23984198e-10;           // MeV cm
constexpr double kFourPiOverHc3 = 4.0 * 3.14159265358979323846 / (kHcMeVCm * kHcMeVCm * kHcMeVCm);

// Limited flux at an interior edge between zone values u (inner) and v (outer):
//   H = -lam m (v - u) / (3 D m + lam |v - u|),  m = max((u + v)/2, floor)   (eqs. a59, a20)
// and its partial derivatives with respect to u, v and lam.
struct EdgeFlux {
    double H, dHu, dHv, dHlam;
};

// 1/x from the hardware estimate and two Newton steps (within an ulp of the IEEE quotient).
__device__ __forceinline__ double drcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// (1 + mu_nu)/2 of the geometric limiter at radius R for a neutrinosphere of radius rnu (eqs. a24-a26
// with beta = 0 and no ray bending, mu_nu = sqrt(1 - (R_nu/R)^2)); -1 inside the neutrinosphere, where
// there is no geometric limit (F_geom = 1).
__device__ __forceinline__ double limb_factor(double R, double rnu) {
    if (!(R > rnu)) return -1.0;
    const double x = rnu / R;
    return 0.5 * (1.0 + sqrt(1.0 - x * x));
}

// Ghost zone of the geometric outer boundary (eq. a62af, R_nu squared) for a last zone with edges rlo,
// rhi: centre R_{I+1} at the mirror of R_I across the outer edge, psi_{I+1} = ratio psi_I with
// ratio = (R_I^2 - R_nu^2/4) / (R_{I+1}^2 - R_nu^2/4) clipped to [0, 1], and the outer edge's D.
struct Ghost {
    double ratio, D;
};
__device__ __forceinline__ Ghost outer_ghost(double rlo, double rhi, double rnu) {
    const double RI = 0.5 * (rlo + rhi), Rg = 2.0 * rhi - RI, q = 0.25 * rnu * rnu;
    const double den = Rg * Rg - q;
    Ghost g;
    g.ratio = den > 0.0 ? fmin(fmax((RI * RI - q) / den, 0.0), 1.0) : 0.0;
    g.D = Rg - RI;
    return g;
}

// With limiter 2 and limb = (1 + mu_nu)/2 > 0 (outside the neutrinosphere), F = min(F_intrp, F_geom)
// (eq. a26a), F_geom = limb m / (lam |v - u| / (3 D)) (eq. a23): where it is the smaller factor
// (limb (3 D m + lam |v - u|) < lam |v - u|) the flux is H = -limb m sign(v - u) (eq. a26b).
__device__ __forceinline__ EdgeFlux edge_flux(double u, double v, double lam, double D,
                                              double floor, int limiter, double limb = -1.0) {
    EdgeFlux f;
    const double delta = v - u;
    if (limiter == 0) {
        const double g = lam / (3.0 * D);
        f.H = -g * delta;
        f.dHu = g;
        f.dHv = -g;
        f.dHlam = -delta / (3.0 * D);
        return f;
    }
    const double mean = 0.5 * (u + v);
    const double m = fmax(mean, floor);
    const double ad = fabs(delta);
    const double den = fma(3.0 * D, m, lam * ad);
    if (limiter == 2 && limb > 0.0 && ad > 0.0 && limb * den < lam * ad) {
        const double sg = delta > 0.0 ? 1.0 : -1.0;
        f.H = -limb * m * sg;
        const double d = (mean > floor) ? -0.5 * limb * sg : 0.0;
        f.dHu = d;
        f.dHv = d;
        f.dHlam = 0.0;
        return f;
    }
    const double inv = drcp(den);
    const double r = m * inv;             // m / den
    const double q = delta * inv;         // delta / den
    f.H = -lam * delta * r;
    const double dHd = -3.0 * D * lam * r * r;          // at fixed m
    const double dHm = (mean > floor) ? -lam * lam * q * fabs(q) : 0.0;  // at fixed delta
    f.dHu = 0.5 * dHm - dHd;
    f.dHv = 0.5 * dHm + dHd;
    f.dHlam = -3.0 * D * delta * r * r;
    return f;
}

// Pair processes (eqs. d12, d16-d22).  Cosine of eq. d22 for x = R_nu/R: sqrt(1 - x^2) outside the
// neutrinosphere, -sqrt(x^2 - 1) clipped at -1 inside it (the equation's sign() read as Fortran's SIGN).
__device__ __forceinline__ double pair_limb_cosine(double x) {
    const double v = 1.0 - x * x;
    return fmax(copysign(sqrt(fabs(v)), v), -1.0);
}
// Angular cutoff of the annihilation kernel for a nu of one species and a partner of the other, from
// their flux factors psi1/psi0 (eta) and limb cosines (mu): chi = min(chi_1, chi_2) (eq. d21), with
// chi_1 = 1 - (3/2) eta eta' (the ratio that defines eq. d16) and chi_2 of eq. d19; symmetric in the pair.
__device__ __forceinline__ double pair_chi(double eta, double eta_o, double mu, double mu_o) {
    const double c1 = 1.0 - 1.5 * eta * eta_o;
    const double c2 = 0.125 * (8.0 + (mu * mu_o - 3.0) * (1.0 + mu) * (1.0 + mu_o));
    return fmin(c1, c2);
}

// Monotone 32-bit key of |v| (sign dropped): for double, the upper word, which orders magnitudes to
// about 2^-20 relative; for float, the whole word.
__device__ __forceinline__ uint32_t abs_key_bits(double v) {
    return (uint32_t)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffffu;
}
__device__ __forceinline__ uint32_t abs_key_bits(float v) { return __float_as_uint(v) & 0x7fffffffu; }

// Max of a 32-bit key over each SL-lane group (SL = 16 or 32) of the wavefront.
template <int SL>
__device__ __forceinline__ uint32_t group_max(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    if constexpr (SL == 32) {
        auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);                   // rows 0<->1, 2<->3
        v = max((uint32_t)sw[0], (uint32_t)sw[1]);
    }
    return v;
}

// Non-temporal store and load of a global element (the factor workspaces: written once per zone in the
// forward sweep and read once in the backward sweep, hundreds of zones later, so caching them only
// evicts other data).
template <typename T>
__device__ __forceinline__ void nt_store(T* p, T v) {
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)p);
}
template <typename T>
__device__ __forceinline__ T nt_load(const T* p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}

// Intra-wavefront ordering point for LDS exchange between lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide deterministic reductions over kBlock threads (fixed shuffle + LDS order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < kBlock / 64; ++j) s += sh[j];
    return s;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int j = 1; j < kBlock / 64; ++j) s = fmax(s, sh[j]);
    return s;
}

__device__ __forceinline__ int block_or(int v, double* sh) {
    return block_max(v ? 1.0 : 0.0, sh) > 0.0 ? 1 : 0;
}

// Zone geometry from three consecutive edges (lo = i-1/2, hi = i+1/2, hi2 = i+3/2):
// V_i = (R_hi^3 - R_lo^3)/3, A = R^2, D_{i+1/2} = R_{i+1} - R_i with R_i the mean of its edges.
__device__ __forceinline__ double shell_volume(double rlo, double rhi) {
    return (rhi - rlo) * (rhi * rhi + rhi * rlo + rlo * rlo) * (1.0 / 3.0);
}

}  // namespace tmk
