// Neutrino energy advection: the Lagrangian energy step (eqs. a78-a80), the PPM remap back onto the
// fixed energy grid with the energy-conserving flux scale (eqs. a81, p5-p8), the Pauli over-fill limiter
// (eqs. a81a-a81d), and the remap after a change of the lapse (eqs. p1-p8).
//
// One thread per (species, ray, zone): its N groups are independent of every other zone.  The target
// grid is the shared e_edge (in the lapse mode everything is measured in units of the new local grid,
// E/a^{n+1} times a^{n+1}; the remap is invariant under that common scale).  The source grid is the
// target grid with every edge m multiplied by s_m:
//   Lagrangian:  s_m = 1 + (a^{n+1}/a^n - 1 - dR/R) - (db/b - dR/R) eta2_m   (eq. a79),
//                N_k = (rho a^3)^{n+1} / (rho a^3)^n W_k psi_k                (eq. a78),
//   lapse:       s_m = a^{n+1}/a^n,  N_k = s^3 W_k psi_k                       (eqs. p1, p2),
// with W_k the target weights and eta2_m the Eddington factor at edge m (mean of the two adjacent
// groups; the end edges take the end group's; 1/3 without one).
//
// The remap works on the number per unit energy a_k = N_k / (S_{k+1} - S_k) over the source grid S:
// limited slopes (eqs. h9-h11), edge values of the interpolating cubic (eq. h12), kept between the
// neighbouring averages (eqs. h15-h17), the parabola of each group (eqs. h22-h24), and through each
// interior edge the number in the region between the displaced and the fixed edge (eqs. h60, h61 with
// that width in place of c_s dt).  Before a group's parabola is formed its edge values are adjusted so
// that it has no extremum inside the group (the zone constraint of the PPM method the paper cites, which
// realises its stated aim that no new extrema appear; without it a steeply falling spectrum overshoots
// below zero and the remap produces negative occupations).  Two ghost groups at each end repeat the end
// group; the two outer edges pass nothing.  The unrolled loop over t keeps a window of a few groups in registers: step t
// forms group t's average and width, the slope of group t-1, the edge value at edge t-1, the
// parabola of group t-2, the flux through edge t-2 and the net flux of group t-3.
#include "tm_kernels.hpp"

namespace tmk {

namespace {

// per-zone description of the source grid and number factor
struct EaZone {
    double c;       // N_k = c W_k psi_k
    double s0, s1;  // s_m = s0 - s1 * eta2_m
};

}  // namespace

template <int NT>
__global__ __launch_bounds__(kBlock) void k_energy_advect(EaArgs A) {
    __shared__ double sT[kMaxN + 1], sW[kMaxN], sE[kMaxN], sAl[kMaxN], sBe[kMaxN];
    const int N = A.N;
    for (int m = threadIdx.x; m <= N; m += blockDim.x) sT[m] = A.e_edge[m];
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double lo = sT[k], hi = sT[k + 1];
        sE[k] = sqrt((hi * hi + hi * lo + lo * lo) / 3.0);       // eq. a01
        sW[k] = (hi * hi * hi - lo * lo * lo) / 3.0;              // eq. a01b
    }
    __syncthreads();
    for (int k = threadIdx.x; k + 2 < N; k += blockDim.x) {      // eqs. a81c, a81d coefficients
        const double e0 = sE[k], e1 = sE[k + 1], e2 = sE[k + 2];
        const double w0 = e0 * e0 * (sT[k + 1] - sT[k]);
        const double w1 = e1 * e1 * (sT[k + 2] - sT[k + 1]);
        const double w2 = e2 * e2 * (sT[k + 3] - sT[k + 2]);
        sAl[k] = (e2 - e0) * w0 / ((e2 - e1) * w1);
        sBe[k] = (e1 - e0) * w0 / ((e2 - e1) * w2);
    }
    __syncthreads();

    const long long zs = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (zs >= A.nz) return;
    const long long zi = zs % A.RI;                               // zone index r*I + i
    EaZone z;
    if (A.mode == kEaLapse) {
        const double s = A.a_new[zi] / A.a_old[zi];
        z.c = s * s * s;
        z.s0 = s;
        z.s1 = 0.0;
    } else {
        const double ao = A.a_old ? A.a_old[zi] : 1.0, an = A.a_new ? A.a_new[zi] : 1.0;
        const double ro = A.rho_old ? A.rho_old[zi] : 1.0, rn = A.rho_new ? A.rho_new[zi] : 1.0;
        const double dR = A.dlnR ? A.dlnR[zi] : 0.0, db = A.dlnb ? A.dlnb[zi] : 0.0;
        z.c = (rn * an * an * an) / (ro * ao * ao * ao);
        z.s0 = 1.0 + ((an / ao - 1.0) - dR);
        z.s1 = db - dR;
    }
    double* prow = A.psi + zs * N;
    const double* hrow = A.edd ? A.edd + zs * N : nullptr;

    double ps[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) ps[k] = k < N ? prow[k] : 0.0;

    // source edge m: S_m = s_m T_m; eta2 at the edge from the groups on both sides
    auto eta_at = [&](int k) { return hrow ? hrow[k] : (1.0 / 3.0); };
    auto src_edge = [&](int m, double h_lo, double h_hi) {
        const double h = (m == 0) ? h_hi : (m == N) ? h_lo : 0.5 * (h_lo + h_hi);
        return (z.s0 - z.s1 * h) * sT[m];
    };

    // window values (indices are compile-time after unrolling; entries die after their last use)
    double Av[NT + 3], Dv[NT + 3], SLv[NT + 3], Vv[NT + 3], Fv[NT + 3], Dn[NT];
    double aLv[NT + 3], dav[NT + 3], a6v[NT + 3];
    double e_src = 0.0, e_n = 0.0, e_d = 0.0;
    bool ok = true;
    double h_prev = eta_at(0);
    double S_lo = src_edge(0, h_prev, h_prev);
    double Sv[NT + 3];
    Sv[0] = S_lo;
    // ghost groups below: the values of group 0 (filled at t = 0)
    double A_m1 = 0.0, A_m2 = 0.0, D_m1 = 0.0, D_m2 = 0.0;

#pragma unroll
    for (int t = 0; t <= NT + 2; ++t) {
        // ---- group t: source width and average (groups >= N repeat group N-1)
        if (t < NT) {
            if (t < N) {
                const double h_hi = (t + 1 < N) ? eta_at(t + 1) : h_prev;
                const double S_hi = src_edge(t + 1, h_prev, h_hi);
                h_prev = h_hi;
                const double w = S_hi - S_lo;
                const double Nk = z.c * sW[t] * ps[t];
                Av[t] = Nk / w;
                Dv[t] = w;
                Sv[t + 1] = S_hi;
                ok = ok && (w > 0.0);
                e_src += Nk * sqrt((S_hi * S_hi + S_hi * S_lo + S_lo * S_lo) / 3.0);   // eq. p3, before
                e_n += Nk * sE[t];
                S_lo = S_hi;
            } else {
                Av[t] = Av[t - 1];
                Dv[t] = Dv[t - 1];
                Sv[t + 1] = Sv[t];
            }
        } else {
            Av[t] = Av[t - 1];
            Dv[t] = Dv[t - 1];
        }
        if (t == 0) {
            A_m1 = A_m2 = Av[0];
            D_m1 = D_m2 = Dv[0];
        }
        auto Aat = [&](int j) { return j >= 0 ? Av[j] : (j == -1 ? A_m1 : A_m2); };
        auto Dat = [&](int j) { return j >= 0 ? Dv[j] : (j == -1 ? D_m1 : D_m2); };

        // ---- slope of group t-1 (eqs. h9-h11); groups -1 and below are flat
        {
            const int j = t - 1;
            if (j >= 0) {
                const double am = Aat(j - 1), a0 = Av[j], ap = Av[j + 1];
                const double dm = Dat(j - 1), d0 = Dv[j], dp = Dv[j + 1];
                const double dplus = ap - a0, dminus = a0 - am;
                const double da = d0 / (dm + d0 + dp) *
                                  ((2.0 * dm + d0) / (dp + d0) * dplus + (d0 + 2.0 * dp) / (dm + d0) * dminus);
                const double lim = fmin(fabs(da), fmin(2.0 * fabs(dplus), 2.0 * fabs(dminus)));
                const double sg = da > 0.0 ? 1.0 : (da < 0.0 ? -1.0 : 0.0);
                SLv[j] = (dplus * dminus > 0.0) ? lim * sg : 0.0;
            }
        }
        auto SLat = [&](int j) { return j >= 0 ? SLv[j] : 0.0; };

        // ---- value at edge e = t-1, between groups e-1 and e (eqs. h12, h15, h16)
        {
            const int e = t - 1;
            if (e >= 0) {
                const double aj = Aat(e - 1), aj1 = Av[e];
                const double dm = Dat(e - 2), d0 = Dat(e - 1), d1 = Dv[e], d2 = Dv[e + 1];
                const double sj = SLat(e - 1), sj1 = SLv[e];
                const double diff = aj1 - aj;
                double v = aj + d0 / (d0 + d1) * diff +
                           1.0 / (dm + d0 + d1 + d2) *
                               (2.0 * d1 * d0 / (d0 + d1) *
                                    ((dm + d0) / (2.0 * d0 + d1) - (d2 + d1) / (2.0 * d1 + d0)) * diff -
                                d0 * (dm + d0) / (2.0 * d0 + d1) * sj1 + d1 * (d1 + d2) / (d0 + 2.0 * d1) * sj);
                v = fmax(v, fmin(aj, aj1));
                v = fmin(v, fmax(aj, aj1));
                Vv[e] = v;
            }
        }

        // ---- parabola of group g = t-2 (eqs. h22-h24), its edge values first adjusted so that it has no
        //      extremum inside the group (flat at an extremum of the averages, else the far edge moved)
        {
            const int g = t - 2;
            if (g >= 0) {
                const double a = Av[g];
                double aL = Vv[g], aR = Vv[g + 1];
                if ((aR - a) * (a - aL) <= 0.0) {
                    aL = a;
                    aR = a;
                } else {
                    const double Da = aR - aL, a6 = 6.0 * (a - 0.5 * (aL + aR));
                    if (Da * a6 > Da * Da) aL = 3.0 * a - 2.0 * aR;
                    else if (-Da * Da > Da * a6) aR = 3.0 * a - 2.0 * aL;
                }
                aLv[g] = aL;
                dav[g] = aR - aL;
                a6v[g] = 6.0 * (a - 0.5 * (aL + aR));
            }
        }

        // ---- flux through edge e = t-2 (eq. p5; h60/h61 over the swept width); outer edges pass nothing
        {
            const int e = t - 2;
            if (e >= 0) {
                double F = 0.0;
                if (e >= 1 && e < N && e < NT) {
                    const double delta = Sv[e] - sT[e];
                    if (delta > 0.0) {
                        const int g = e - 1;
                        const double y = delta / Dv[g];
                        ok = ok && (y <= 1.0);
                        const double aR = aLv[g] + dav[g];
                        F = (aR - 0.5 * y * (dav[g] - (1.0 - 2.0 * y / 3.0) * a6v[g])) * delta;
                    } else if (delta < 0.0) {
                        const int g = e;
                        const double y = -delta / Dv[g];
                        ok = ok && (y <= 1.0);
                        F = (aLv[g] + 0.5 * y * (dav[g] + (1.0 - 2.0 * y / 3.0) * a6v[g])) * delta;
                    }
                }
                Fv[e] = F;
            }
        }

        // ---- net flux into group k = t-3: F_{k-1/2} - F_{k+1/2}
        {
            const int k = t - 3;
            if (k >= 0 && k < NT) {
                Dn[k] = (k < N) ? Fv[k] - Fv[k + 1] : 0.0;
                if (k < N) e_d += Dn[k] * sE[k];
            }
        }
    }

    // eq. p8: the flux scale that conserves the energy; eq. p6: the new numbers
    const double num = e_src - e_n;
    const double xi = (e_d != 0.0) ? num / e_d : 1.0;
    int flags = 0;
    if (ok) {
        double pn[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) pn[k] = (k < N) ? (z.c * sW[k] * ps[k] + xi * Dn[k]) / sW[k] : 0.0;
        // over-fill limiter, from the lowest group while groups k+1, k+2 exist (eqs. a81a-a81d)
#pragma unroll
        for (int k = 0; k + 2 < NT; ++k) {
            if (k + 2 < N && pn[k] > 1.0) {
                double rm0 = pn[k] - 1.0;
                double add1 = sAl[k] * rm0;
                double rm2 = sBe[k] * rm0;
                flags |= kEaOverfill;
                if (rm2 > pn[k + 2]) {
                    const double sc = pn[k + 2] / rm2;
                    rm0 *= sc;
                    add1 *= sc;
                    rm2 = pn[k + 2];
                    flags |= kEaOverfillClamp;
                }
                pn[k] -= rm0;
                pn[k + 1] += add1;
                pn[k + 2] -= rm2;
            }
        }
#pragma unroll
        for (int k = 0; k < NT; ++k)
            if (k < N) prow[k] = pn[k];
    } else {
        flags = kEaDisplacement;
    }
    if (A.xi) A.xi[zs] = ok ? xi : 1.0;
    if (A.flags) A.flags[zs] = flags;
}

hipError_t launch_energy_advect(const EaArgs& a, hipStream_t st) {
    if (a.nz <= 0) return hipSuccess;
    const long long blocks = (a.nz + kBlock - 1) / kBlock;
    const int nt = padded_groups(a.N);
    switch (nt) {
#define TM_EA_CASE(T) \
    case T: hipLaunchKernelGGL(k_energy_advect<T>, dim3((unsigned)blocks), dim3(kBlock), 0, st, a); break;
        TM_EA_CASE(4)
        TM_EA_CASE(8)
        TM_EA_CASE(12)
        TM_EA_CASE(16)
        TM_EA_CASE(20)
        TM_EA_CASE(24)
        TM_EA_CASE(28)
        TM_EA_CASE(32)
#undef TM_EA_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tmk
