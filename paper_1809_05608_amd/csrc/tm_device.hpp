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
};

struct Shape {
    int S, R, I, N;
    double c_dt;
    int outer_bc;      // 0 zero flux, 1 free streaming
    unsigned terms;    // TM_TERM_* bits
    int limiter;       // 0 none, 1 F_intrp
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
};

constexpr unsigned kDiffusion = 1u, kEmAbs = 2u, kNes = 4u;

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

__device__ __forceinline__ EdgeFlux edge_flux(double u, double v, double lam, double D,
                                              double floor, int limiter) {
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

// Zone geometry from three consecutive edges (lo = i-1/2, hi = i+1/2, hi2 = i+3/2):
// V_i = (R_hi^3 - R_lo^3)/3, A = R^2, D_{i+1/2} = R_{i+1} - R_i with R_i the mean of its edges.
__device__ __forceinline__ double shell_volume(double rlo, double rhi) {
    return (rhi - rlo) * (rhi * rhi + rhi * rlo + rlo * rlo) * (1.0 / 3.0);
}

}  // namespace tmk
