// Neutrino energy advection: the Lagrangian energy step (eqs. a78-a80), the PPM remap back onto the
// fixed energy grid with the energy-conserving flux scale (eqs. a81, p5-p8), the Pauli over-fill limiter
// (eqs. a81a-a81d), and the remap after a change of the lapse (eqs. p1-p8).
//
// One thread per (species, ray, zone): its N groups are independent of every other zone.  A block of
// 128 zones loads its psi rows into LDS with coalesced loads and stores the new psi the same way; each
// thread reads its Eddington factors from HBM and keeps its net fluxes in registers (staging both rows
// in LDS halves the blocks a CU holds, and the kernel needs the waves to hide its FP64 latency).  The target
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

constexpr int kEaBlock = 128;     // zones per block; their psi and Eddington rows are staged in LDS

template <int NT>
__global__ __launch_bounds__(kEaBlock) void k_energy_advect(EaArgs A) {
    constexpr int LD = NT + 1;                                    // LDS row stride (odd: no bank aliasing)
    __shared__ double sP[kEaBlock * LD];                          // psi rows, then the new psi
    __shared__ double sT[kMaxN + 1], sW[kMaxN], sRW[kMaxN], sE[kMaxN], sAl[kMaxN], sBe[kMaxN];
    const int N = A.N;                                            // groups, N <= NT
    const int tid = threadIdx.x;
    for (int m = tid; m <= N; m += kEaBlock) sT[m] = A.e_edge[m];
    // the block's rows, loaded coalesced: zones [zs0, zs0 + nb)
    const long long zs0 = (long long)blockIdx.x * kEaBlock;
    const int nb = (int)min((long long)kEaBlock, A.nz - zs0);
    double* gP = A.psi + zs0 * N;
    const double* gH = A.edd ? A.edd + zs0 * N : nullptr;
    for (int e = tid; e < nb * N; e += kEaBlock) {
        const int r = e / N, k = e - r * N;
        sP[r * LD + k] = gP[e];
    }
    __syncthreads();
    for (int k = tid; k < N; k += kEaBlock) {
        const double lo = sT[k], hi = sT[k + 1];
        sE[k] = sqrt((hi * hi + hi * lo + lo * lo) / 3.0);       // eq. a01
        sW[k] = (hi * hi * hi - lo * lo * lo) / 3.0;              // eq. a01b
        sRW[k] = 1.0 / sW[k];
    }
    __syncthreads();
    for (int k = tid; k + 2 < N; k += kEaBlock) {                 // eqs. a81c, a81d coefficients
        const double e0 = sE[k], e1 = sE[k + 1], e2 = sE[k + 2];
        const double w0 = e0 * e0 * (sT[k + 1] - sT[k]);
        const double w1 = e1 * e1 * (sT[k + 2] - sT[k + 1]);
        const double w2 = e2 * e2 * (sT[k + 3] - sT[k + 2]);
        sAl[k] = (e2 - e0) * w0 / ((e2 - e1) * w1);
        sBe[k] = (e1 - e0) * w0 / ((e2 - e1) * w2);
    }
    __syncthreads();

    if (tid < nb) {
        const long long zs = zs0 + tid;
        const long long zi = zs % A.RI;                           // zone index r*I + i
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
        double* rowP = sP + tid * LD;
        const double* rowH = gH ? gH + tid * N : nullptr;
        double Dn[NT];

        // source edges S_m = s_m T_m (eq. a79 at edge m; the Eddington factor of an edge is the mean of
        // its two groups, the end groups' own at the two ends)
        double Sv[NT + 1];
#pragma unroll
        for (int m = 0; m <= NT; ++m) {
            if (m <= N) {
                auto hh = [&](int k) { return rowH ? rowH[k] : 1.0 / 3.0; };
                const double h = (m == 0) ? hh(0) : (m == N) ? hh(N - 1) : 0.5 * (hh(m - 1) + hh(m));
                Sv[m] = (z.s0 - z.s1 * h) * sT[m];
            } else {
                Sv[m] = Sv[m - 1];
            }
        }

        // window values (indices are compile-time after unrolling; entries die after their last use).
        // Index j + 2 holds group j, so the two ghost groups below are entries 0 and 1; groups at or above
        // N repeat group N-1.  Q[e + 2] = 1 / (D_{e-1} + D_e) belongs to edge e (groups e-1 and e).
        constexpr int W = NT + 5;
        constexpr double kThird = 1.0 / 3.0, kTwoThirds = 2.0 / 3.0;
        double Av[W], Dv[W], RW[W], Q[W], SL[W], Vv[W], aLv[W], dav[W], a6v[W], Fv[W];
        double e_src = 0.0, e_n = 0.0, e_d = 0.0;
        bool ok = true;

#pragma unroll
        for (int t = 0; t <= NT + 2; ++t) {
            // ---- group t: source width, its reciprocal and the average (groups >= N repeat group N-1)
            const int gt = t + 2;
            if (t < NT && (t < N)) {
                const double S_lo = Sv[t], S_hi = Sv[t + 1];
                const double w = S_hi - S_lo;
                const double rw = drcp(w);
                const double Nk = z.c * sW[t] * rowP[t];
                Av[gt] = Nk * rw;
                Dv[gt] = w;
                RW[gt] = rw;
                ok = ok && (w > 0.0);
                e_src += Nk * sqrt((S_hi * S_hi + S_hi * S_lo + S_lo * S_lo) * kThird);   // eq. p3, before
                e_n += Nk * sE[t];
            } else {
                Av[gt] = Av[gt - 1];
                Dv[gt] = Dv[gt - 1];
                RW[gt] = RW[gt - 1];
            }
            if (t == 0) {
                Av[0] = Av[1] = Av[2];
                Dv[0] = Dv[1] = Dv[2];
            }
            Q[gt] = drcp(Dv[gt - 1] + Dv[gt]);                    // edge t (groups t-1, t)
            if (t == 0) Q[1] = Q[2];                              // edge -1, between the ghost groups

            // ---- slope of group j = t-1 (eqs. h9-h11); the ghost groups are flat
            const int j = t - 1;
            if (j >= 0) {
                const int gj = j + 2;
                const double am = Av[gj - 1], a0 = Av[gj], ap = Av[gj + 1];
                const double dm = Dv[gj - 1], d0 = Dv[gj], dp = Dv[gj + 1];
                const double dplus = ap - a0, dminus = a0 - am;
                const double da = d0 * drcp(dm + d0 + dp) *
                                  ((2.0 * dm + d0) * Q[gj + 1] * dplus + (d0 + 2.0 * dp) * Q[gj] * dminus);
                const double lim = fmin(fabs(da), fmin(2.0 * fabs(dplus), 2.0 * fabs(dminus)));
                const double sg = da > 0.0 ? 1.0 : (da < 0.0 ? -1.0 : 0.0);
                SL[gj] = (dplus * dminus > 0.0) ? lim * sg : 0.0;
            }
            if (t == 0) SL[1] = 0.0;                              // ghost group -1

            // ---- value at edge e = t-1, between groups e-1 and e (eqs. h12, h15, h16)
            const int e = t - 1;
            if (e >= 0) {
                const int g0 = e + 1, g1 = e + 2;                 // entries of groups e-1 and e
                const double aj = Av[g0], aj1 = Av[g1];
                const double dm = Dv[g0 - 1], d0 = Dv[g0], d1 = Dv[g1], d2 = Dv[g1 + 1];
                const double sj = SL[g0], sj1 = SL[g1];
                const double diff = aj1 - aj;
                const double q = Q[g1];                           // 1 / (d0 + d1)
                const double rB = drcp(2.0 * d0 + d1), rC = drcp(2.0 * d1 + d0);
                double v = aj + d0 * q * diff +
                           drcp(dm + d0 + d1 + d2) *
                               (2.0 * d1 * d0 * q * ((dm + d0) * rB - (d2 + d1) * rC) * diff -
                                d0 * (dm + d0) * rB * sj1 + d1 * (d1 + d2) * rC * sj);
                v = fmax(v, fmin(aj, aj1));
                v = fmin(v, fmax(aj, aj1));
                Vv[g1] = v;                                       // entry of the edge below group e
            }

            // ---- parabola of group g = t-2 (eqs. h22-h24), its edge values first adjusted so that it has
            //      no extremum inside the group (flat at an extremum of the averages, else the far edge moved)
            const int g = t - 2;
            if (g >= 0) {
                const int gg = g + 2;
                const double a = Av[gg];
                double aL = Vv[gg], aR = Vv[gg + 1];
                if ((aR - a) * (a - aL) <= 0.0) {
                    aL = a;
                    aR = a;
                } else {
                    const double Da = aR - aL, a6 = 6.0 * (a - 0.5 * (aL + aR));
                    if (Da * a6 > Da * Da) aL = 3.0 * a - 2.0 * aR;
                    else if (-Da * Da > Da * a6) aR = 3.0 * a - 2.0 * aL;
                }
                aLv[gg] = aL;
                dav[gg] = aR - aL;
                a6v[gg] = 6.0 * (a - 0.5 * (aL + aR));
            }

            // ---- flux through edge f = t-2 (eq. p5; h60/h61 over the swept width); outer edges pass nothing
            const int f = t - 2;
            if (f >= 0) {
                double F = 0.0;
                if (f >= 1 && f < NT && (f < N)) {
                    const double delta = Sv[f] - sT[f];
                    if (delta > 0.0) {                            // top of group f-1 moves up
                        const int gg = f + 1;
                        const double y = delta * RW[gg];
                        ok = ok && (y <= 1.0);
                        const double aR = aLv[gg] + dav[gg];
                        F = (aR - 0.5 * y * (dav[gg] - (1.0 - kTwoThirds * y) * a6v[gg])) * delta;
                    } else if (delta < 0.0) {                     // bottom of group f moves down
                        const int gg = f + 2;
                        const double y = -delta * RW[gg];
                        ok = ok && (y <= 1.0);
                        F = (aLv[gg] + 0.5 * y * (dav[gg] + (1.0 - kTwoThirds * y) * a6v[gg])) * delta;
                    }
                }
                Fv[f] = F;
            }

            // ---- net flux into group k = t-3, F_{k-1/2} - F_{k+1/2}, kept in the (consumed) Eddington row
            const int k = t - 3;
            if (k >= 0 && k < NT && (k < N)) {
                const double dn = Fv[k] - Fv[k + 1];
                Dn[k] = dn;
                e_d += dn * sE[k];
            }
        }

        // eq. p8: the flux scale that conserves the energy; eq. p6: the new numbers
        const double xi = (e_d != 0.0) ? (e_src - e_n) / e_d : 1.0;
        int flags = 0;
        if (ok) {
            double pn[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k)
                pn[k] = (k < N) ? (z.c * sW[k] * rowP[k] + xi * Dn[k]) * sRW[k] : 0.0;
            // over-fill limiter, from the lowest group while groups k+1, k+2 exist (eqs. a81a-a81d)
#pragma unroll
            for (int k = 0; k + 2 < NT; ++k) {
                if ((k + 2 < N) && pn[k] > 1.0) {
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
                if (k < N) rowP[k] = pn[k];
        } else {
            flags = kEaDisplacement;                              // the row keeps psi^n
        }
        if (A.xi) A.xi[zs] = ok ? xi : 1.0;
        if (A.flags) A.flags[zs] = flags;
    }
    __syncthreads();
    for (int e = tid; e < nb * N; e += kEaBlock) {
        const int r = e / N, k = e - r * N;
        gP[e] = sP[r * LD + k];
    }
}

hipError_t launch_energy_advect(const EaArgs& a, hipStream_t st) {
    if (a.nz <= 0) return hipSuccess;
    const long long blocks = (a.nz + kEaBlock - 1) / kEaBlock;
    const int nt = padded_groups(a.N);
    switch (nt) {
#define TM_EA_CASE(T) \
    case T: hipLaunchKernelGGL(k_energy_advect<T>, dim3((unsigned)blocks), dim3(kEaBlock), 0, st, a); break;
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
