// FP64 kernels of libtm over cells: grid constants, residual with per-system norms and
// conservation sums, debug Jacobian blocks, and the adjoint vector-Jacobian product.
//
// Mapping of the residual and VJP kernels: one 256-thread block per (species, ray) system,
// one thread per cell (zone, group) of a chunk of zones; each edge flux is computed once
// and shared through LDS, and the block reduces per-system quantities in a fixed order
// (deterministic, no atomics).
#include <algorithm>

#include "tm_kernels.hpp"

namespace tmk {

// ---------------------------------------------------------------- grid constants

__global__ void k_setup(const double* __restrict__ e_edge, const double* __restrict__ nes_g, int N,
                        Consts* __restrict__ out) {
    __shared__ double eps[kMaxN], W[kMaxN];
    __shared__ double wbar;
    const int t = threadIdx.x;
    if (t < N) {
        const double lo = e_edge[t], hi = e_edge[t + 1];
        eps[t] = sqrt((hi * hi + hi * lo + lo * lo) * (1.0 / 3.0));   // eq. a01, square restored
        W[t] = (hi - lo) * (hi * hi + hi * lo + lo * lo) * (1.0 / 3.0); // eq. a01b
    }
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int k = 0; k < N; ++k) s += W[k];
        wbar = s / N;
    }
    __syncthreads();
    if (t < kMaxN) {
        out->eps[t] = t < N ? eps[t] : 0.0;
        out->W[t] = t < N ? W[t] : 0.0;
        out->de[t] = (t + 1 < N) ? eps[t + 1] - eps[t] : 0.0;
    }
    if (t == 0) {
        int ok = 1;
        for (int k = 1; k < N; ++k) ok &= eps[k] >= 1.25 * eps[k - 1];
        out->nes_window = ok;
        out->wbar = wbar;
    }
    for (int idx = t; idx < kMaxN * kMaxN; idx += blockDim.x) {
        const int k = idx / kMaxN, kp = idx % kMaxN;
        double v = 0.0;
        // k' = k (no energy change) is left out: its in and out terms cancel identically (eq. d8b)
        if (k < N && kp < N && kp != k && nes_g != nullptr)
            v = eps[k] * eps[kp] / (kEps0 * kEps0) * nes_g[k * N + kp] * (W[kp] / wbar);
        out->P[k][kp] = v;
    }
}

hipError_t launch_setup(const double* e_edge, const double* nes_g, int N, Consts* out, hipStream_t st) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, e_edge, nes_g, N, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- per-zone pieces

// NES source of one zone: S_k = amp [(1 - p_k) sum_k' P Ein p_k' - p_k sum_k' P Eout (1 - p_k')]
// with the detailed-balance factor exp(-|eps_k - eps_k'|/T) built as a product of
// neighbour factors d_j = exp(-(eps_{j+1} - eps_j)/T) (Eout for k' > k, Ein for k' < k).
// Also returns the two kernel sums (without amp) for the Jacobian diagonal.
template <int NT>
__device__ __forceinline__ void nes_zone(const Consts* __restrict__ cs, int N, double T, const double* p,
                                         double* sin_out, double* sout_out) {
    double d[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) d[j] = (j + 1 < N) ? exp(-cs->de[j] / T) : 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        if (k >= N) break;
        double sin_ = 0.0;
        double sout = 0.0;
        double e = 1.0;
#pragma unroll
        for (int kp = k + 1; kp < NT; ++kp) {          // up-scatter side: out factor decays
            if (kp >= N) break;
            e *= d[kp - 1];
            sout = fma(cs->P[k][kp] * e, 1.0 - p[kp], sout);
            sin_ = fma(cs->P[k][kp], p[kp], sin_);
        }
        e = 1.0;
#pragma unroll
        for (int kp = k - 1; kp >= 0; --kp) {          // down-scatter side: in factor decays
            e *= d[kp];
            sin_ = fma(cs->P[k][kp] * e, p[kp], sin_);
            sout = fma(cs->P[k][kp], 1.0 - p[kp], sout);
        }
        sin_out[k] = sin_;
        sout_out[k] = sout;
    }
}

struct ZoneGeom {
    double V, A_lo, A_hi, D_lo, D_hi, V_lo, V_hi;
};

// Geometry of zone i of a ray; with a lapse (f.lapse set) the volumes are V / a^3 and the areas A / a^2.
__device__ __forceinline__ ZoneGeom zone_geom(const double* __restrict__ re, int i, int I, const Fields& f,
                                              int ray) {
    ZoneGeom g;
    const double rlo = re[i], rhi = re[i + 1];
    const size_t z = (size_t)ray * I + i, e = (size_t)ray * (I + 1) + i;
    g.V = shell_volume(rlo, rhi) / lapse_zone3(f, z);
    g.A_lo = rlo * rlo * lapse_edge_inv2(f, e);
    g.A_hi = rhi * rhi * lapse_edge_inv2(f, e + 1);
    const double rc = 0.5 * (rlo + rhi);
    g.D_lo = 0.0;
    g.V_lo = 1.0;
    g.D_hi = 0.0;
    g.V_hi = 1.0;
    if (i > 0) {
        const double rm = re[i - 1];
        g.D_lo = rc - 0.5 * (rm + rlo);
        g.V_lo = shell_volume(rm, rlo) / lapse_zone3(f, z - 1);
    }
    if (i + 1 < I) {
        const double rp = re[i + 2];
        g.D_hi = 0.5 * (rhi + rp) - rc;
        g.V_hi = shell_volume(rhi, rp) / lapse_zone3(f, z + 1);
    }
    return g;
}

__device__ __forceinline__ double inv_mfp(const Fields& f, size_t c) {
    return 1.0 / (f.kappa_a[c] + f.eta[c] + f.kappa_s[c]);
}

// ---------------------------------------------------------------- residual / statistics

// Mapping: one block per system.  The 256 threads form RZ = 256/NT rows of NT groups (thread =
// cell, so every global access is coalesced); row r of a chunk holds zone z0 - 1 + r, and the
// interior rows z0 .. z0 + RZ - 3 are the chunk's output zones, the first and last rows being
// halo.  Per chunk: every cell brings psi and its transport opacity (one reciprocal for lambda)
// to LDS, together with the chunk's zone edges, temperatures and NES amplitudes (one value per
// thread); every edge flux is computed once, by the cell below the edge, into LDS; then each
// output cell assembles G from the two edge fluxes of its zone, emission/absorption and the
// O(N) NES sums over its zone's LDS row.  The loads of the next chunk are issued before the
// current chunk is processed, so the memory latency overlaps the arithmetic (the barriers wait
// for LDS traffic only).  The NES shape matrix is staged once per block.  Besides max|G| the
// kernel computes the rounding level of G (32 ulp of the largest per-cell sum of term
// magnitudes plus |psi| |dG/dpsi|), below which the Newton stopping rule does not ask for
// further progress.
// LAPSE and GEO compile the lapse factors and the neutrinosphere options (limiter 2, outer boundary 2)
// in; the plain instance leaves their registers out (127 instead of 131 VGPRs: four waves per SIMD
// instead of three).
template <int NT, bool LAPSE, bool GEO>
__global__ __launch_bounds__(kBlock) void k_residual(Shape sh, Fields f, const Consts* __restrict__ cs,
                                                     const double* __restrict__ psi_n,
                                                     const double* __restrict__ psi, double* __restrict__ G_out,
                                                     double g_sign, ResidualOut out) {
    constexpr int RZ = kBlock / NT;             // rows per chunk (zones incl. one halo on each side)
    constexpr int ZB = RZ - 2;                  // output zones per chunk
    constexpr int PS = NT + 1;                  // padded LDS row stride (conflict-free column reads)
    static_assert(3 * RZ + 2 <= kBlock, "one zone value per thread");
    __shared__ double s_P[NT * PS];
    __shared__ double s_psi[RZ][PS];
    __shared__ double2 s_pq[RZ][NT];            // psi and 1 - psi of the row (the NES sums read both at once)
    __shared__ double s_lam[RZ][PS];
    __shared__ double s_d[RZ][PS];
    __shared__ double s_H[RZ][PS];              // flux at the upper edge of the row's zone
    __shared__ double s_du[RZ][PS];             // its derivative with respect to the lower zone
    __shared__ double s_dv[RZ][PS];             // ... and to the upper zone
    __shared__ double s_z[3 * RZ + 2];          // edges z0-1 .. z0+RZ, then T and amp of the rows
    __shared__ double red[kBlock / 64];
    double* const s_re = s_z;
    double* const s_T = s_z + RZ + 2;
    double* const s_amp = s_z + 2 * RZ + 2;
    const long long sys = blockIdx.x;
    if (out.mode == kResTrial && out.pending[sys] == 0) return;         // no trial to evaluate
    if (out.mode == kResEval && out.pending && out.pending[sys % sh.R] == 0) return;
    const int I = sh.I, N = sh.N;
    const int ray = (int)(sys % sh.R);
    const double* re = f.r_edge + (size_t)ray * (I + 1);
    const double c = sh.c_dt;
    const bool diff = sh.terms & kDiffusion, emabs = sh.terms & kEmAbs, nes = sh.terms & kNes;
    const int t = threadIdx.x, zl = t / NT, k = t - zl * NT;
    const bool tile = zl < RZ;
    const bool lane_ok = tile && k < N;
    const bool out_row = zl >= 1 && zl <= RZ - 2;

    if (nes)
        for (int j = t; j < NT * NT; j += kBlock) s_P[(j / NT) * PS + (j % NT)] = cs->P[j / NT][j % NT];

    double gmax = 0.0, gscale = 0.0;
    int bad = 0;
    double s_n = 0.0, s_nold = 0.0, s_e = 0.0, s_q = 0.0, s_nes = 0.0, s_b = 0.0;
    const double Wk = lane_ok ? cs->W[k] : 0.0;
    const double epsk = lane_ok ? cs->eps[k] : 0.0;
    const bool geo = GEO && (sh.limiter == 2 || sh.outer_bc == 2);   // neutrinosphere radii in use
    const double rnuk = (geo && lane_ok) ? f.r_nu[(size_t)(sys / sh.R) * N + k] : 0.0;
    const double dek = (lane_ok && k + 1 < N) ? cs->de[k] : 0.0;
    const size_t sys_cell0 = (size_t)sys * I * N;

    // per-thread inputs of one chunk: the cell's fields and one zone value
    struct In {
        double p, ka, et, ks, pn, zv;
    };
    // Every load is issued unconditionally from a clamped, in-bounds address and the value selected
    // afterwards: straight-line code lets the wait for a chunk's data count exactly the loads
    // issued after it, instead of draining the memory pipe.
    auto load = [&](int z0, In& v) {
        const int i = z0 - 1 + zl;
        const bool in_zone = lane_ok && i >= 0 && i < I;
        const bool outc = in_zone && out_row;
        const size_t cb = sys_cell0 + (in_zone ? (size_t)i * N + k : 0);
        const double lp = psi[cb], lka = f.kappa_a[cb], let = f.eta[cb], lks = f.kappa_s[cb], lpn = psi_n[cb];
        const bool opac = diff ? in_zone : (emabs && outc);
        v.p = (diff ? in_zone : outc) ? lp : 0.0;
        v.ka = opac ? lka : 0.0;
        v.et = opac ? let : 0.0;
        v.ks = (diff && in_zone) ? lks : 0.0;
        v.pn = outc ? lpn : 0.0;
        const double* src = re;
        bool zok = false;
        double zdef = 0.0;
        if (t < RZ + 2) {
            const int j = z0 - 1 + t;
            zok = j >= 0 && j <= I;
            src = re + (zok ? j : 0);
        } else if (t < 2 * RZ + 2) {
            const int j = z0 - 1 + (t - RZ - 2);
            zok = nes && j >= 0 && j < I;
            src = zok ? f.temp + (size_t)ray * I + j : re;
            zdef = 1.0;
        } else if (t < 3 * RZ + 2) {
            const int j = z0 - 1 + (t - 2 * RZ - 2);
            zok = nes && j >= 0 && j < I;
            src = zok ? f.nes_amp + (size_t)sys * I + j : re;
        }
        const double lz = *src;
        v.zv = zok ? lz : zdef;
    };

    In cur;
    load(0, cur);
    for (int z0 = 0; z0 < I; z0 += ZB) {
        In nxt;
        load(z0 + ZB, nxt);                                 // in flight while this chunk is processed
        const int i = z0 - 1 + zl;                          // this row's zone (may be a halo or outside)
        const bool in_zone = lane_ok && i >= 0 && i < I;
        const double p = cur.p;
        const double lam = (diff && in_zone) ? drcp(cur.ka + cur.et + cur.ks) : 0.0;
        __syncthreads();                                    // previous chunk done with the LDS rows
        if (tile) {
            s_psi[zl][k] = p;
            if (nes) s_pq[zl][k] = make_double2(p, 1.0 - p);
            s_lam[zl][k] = lam;
        }
        if (t < 3 * RZ + 2) s_z[t] = cur.zv;
        __syncthreads();
        if (tile) {
            s_d[zl][k] = (nes && in_zone && out_row && k + 1 < N) ? exp(-dek * drcp(s_T[zl])) : 0.0;
            // flux at the upper edge of this row's zone, computed once per edge
            if (diff) {
                double H = 0.0, du = 0.0, dv = 0.0;
                if (in_zone && zl + 1 < RZ) {
                    if (i + 1 < I) {
                        const double rlo = s_re[zl], rhi = s_re[zl + 1], rp = s_re[zl + 2];
                        const double D = 0.5 * (rhi + rp) - 0.5 * (rlo + rhi);
                        const EdgeFlux e = edge_flux(p, s_psi[zl + 1][k], sqrt(lam * s_lam[zl + 1][k]), D,
                                                     sh.psi_floor, sh.limiter,
                                                     (GEO && sh.limiter == 2) ? limb_factor(rhi, rnuk) : -1.0);
                        H = e.H;
                        du = e.dHu;
                        dv = e.dHv;
                    } else if (sh.outer_bc == 1) {
                        H = p;                              // free streaming, eq. a22 limit
                        du = 1.0;
                    } else if (GEO && sh.outer_bc == 2) {   // ghost zone of eq. a62af
                        const double rlo = s_re[zl], rhi = s_re[zl + 1];
                        const Ghost gh = outer_ghost(rlo, rhi, rnuk);
                        const EdgeFlux e = edge_flux(p, gh.ratio * p, lam, gh.D, sh.psi_floor, sh.limiter,
                                                     sh.limiter == 2 ? limb_factor(rhi, rnuk) : -1.0);
                        H = e.H;
                        du = e.dHu + gh.ratio * e.dHv;
                    }
                }
                s_H[zl][k] = H;                             // the edge below zone 0 has zero flux
                s_du[zl][k] = du;
                s_dv[zl][k] = dv;
            }
        }
        __syncthreads();
        const In now = cur;
        cur = nxt;
        if (!in_zone || !out_row) continue;

        const size_t cb = sys_cell0 + (size_t)i * N + k;
        const double pn = now.pn;
        double G = p - pn;
        double scale = fabs(p) + fabs(pn);
        const double rlo = s_re[zl], rhi = s_re[zl + 1];
        double V = shell_volume(rlo, rhi);
        double A_lo = rlo * rlo, A_hi = rhi * rhi;
        if (LAPSE && f.lapse) {                             // eq. a58 times a_i c dt: V / a^3 and A / a^2
            const double a0 = f.lapse[(size_t)ray * I + i];
            const double e0 = f.lapse_edge[(size_t)ray * (I + 1) + i], e1 = f.lapse_edge[(size_t)ray * (I + 1) + i + 1];
            V /= a0 * a0 * a0;
            A_lo /= e0 * e0;
            A_hi /= e1 * e1;
        }
        double Hh = 0.0;
        double jd = 1.0;                                    // |dG_ik/dpsi_ik| bound, for the rounding level
        if (diff) {
            const double Hlo = s_H[zl - 1][k], dlo = s_dv[zl - 1][k];
            Hh = s_H[zl][k];
            const double dhi = s_du[zl][k];
            const double iV = drcp(V);
            G += c * (A_hi * Hh - A_lo * Hlo) * iV;
            scale += c * (fabs(A_hi * Hh) + fabs(A_lo * Hlo)) * iV;
            jd += c * (A_hi * fabs(dhi) + A_lo * fabs(dlo)) * iV;
        }
        const double ka = now.ka, et = now.et;
        if (emabs) {
            G += c * (ka * p - et * (1.0 - p));
            scale += c * (fabs(ka * p) + fabs(et * (1.0 - p)));
            jd += c * (ka + et);
        }
        double S = 0.0;
        if (nes) {
            const double amp = s_amp[zl];
            // The group index goes through an opaque copy: the lane masks of the two loops are then formed here
            // (one compare per term) instead of being hoisted out of the zone loop as 38 live scalar masks.
            int kz = k;
            asm volatile("" : "+v"(kz));
            // k' > k: the out kernel carries exp(-(eps_k' - eps_k)/T) = prod_{j=k}^{k'-1} d_j.  The weighted sum
            // of those products is taken in Horner form from the last group down, one multiply-add and one
            // multiply per term: h <- (h + P_kk' (1 - psi_k')) d_{k'-1}.
            double hup = 0.0, sin_ = 0.0;
#pragma unroll
            for (int kp = NT - 1; kp >= 1; --kp) {
                if (kp > kz) {                         // padding groups add exact zeros (P = 0 there)
                    const double Pk = s_P[k * PS + kp];
                    const double2 pq = s_pq[zl][kp];
                    hup = fma(Pk, pq.y, hup) * s_d[zl][kp - 1];
                    sin_ = fma(Pk, pq.x, sin_);
                }
            }
            // k' < k: the in kernel carries exp(-(eps_k - eps_k')/T) = prod_{j=k'}^{k-1} d_j, in Horner form from
            // group 0 up: h <- (h + P_kk' psi_k') d_k'
            double hdn = 0.0, sout = hup;
#pragma unroll
            for (int kp = 0; kp < NT - 1; ++kp) {
                if (kp < kz) {
                    const double Pk = s_P[k * PS + kp];
                    const double2 pq = s_pq[zl][kp];
                    hdn = fma(Pk, pq.x, hdn) * s_d[zl][kp];
                    sout = fma(Pk, pq.y, sout);
                }
            }
            sin_ += hdn;
            S = amp * ((1.0 - p) * sin_ - p * sout);
            G -= c * S;
            scale += c * amp * (fabs(1.0 - p) * fabs(sin_) + fabs(p) * fabs(sout));
            jd += c * amp * (fabs(sin_) + fabs(sout));
        }
        scale += fabs(p) * jd;                              // G changes by jd * ulp(psi) per ulp of psi
        bad |= !isfinite(G);
        gmax = fmax(gmax, fabs(G));
        gscale = fmax(gscale, scale);
        if (G_out) G_out[cb] = g_sign * G;
        if (out.stats) {
            const double vw = V * Wk;
            s_n = fma(vw, p, s_n);
            s_nold = fma(vw, pn, s_nold);
            s_e = fma(vw * epsk, p, s_e);
            if (emabs) s_q = fma(c * vw, et * (1.0 - p) - ka * p, s_q);
            if (nes) s_nes = fma(c * vw, S, s_nes);
            if (i == I - 1 && diff) s_b = fma(Wk, Hh, s_b);
        }
    }

    const double res = block_max(gmax, red);
    const double floor_g = 32.0 * 2.220446049250313e-16 * block_max(gscale, red);
    bad = block_or(bad, red);
    if (out.stats) {
        s_n = block_sum(s_n, red);
        s_nold = block_sum(s_nold, red);
        s_e = block_sum(s_e, red);
        s_q = block_sum(s_q, red);
        s_nes = block_sum(s_nes, red);
        s_b = block_sum(s_b, red);
    }
    if (threadIdx.x == 0) {
        const double rr = bad ? __builtin_nan("") : res;
        out.res[sys] = rr;
        if (out.level) out.level[sys] = floor_g;
        const int it = out.iters ? out.iters[sys] : 0;
        if (out.mode == kResInitial) {
            // Newton stopping rule: max|G| <= target = max(rtol * max|G_0|, rounding level of G), or no
            // halving of max|G| within 1000x of the target; rtol = 0 means a fixed number of updates
            const double target = fmax(out.rtol * rr, floor_g);
            out.res0[sys] = rr;
            out.res_acc[sys] = rr;
            out.tgt[sys] = target;
            const bool stop = out.rtol > 0.0 && !bad && rr <= target;
            out.active[sys] = (!stop && !bad && it < out.max_iter && rr > 0.0) ? 1 : 0;
        } else if (out.mode == kResTrial) {
            // backtracking line search: accept the trial on sufficient decrease of max|G|, at the
            // shortest step, or when the previous iterate was already within 1000x of its target
            const double racc = out.res_acc[sys], a = out.alpha[sys];
            const bool near = racc <= 1e3 * out.tgt[sys];
            const bool accept = near || rr <= (1.0 - kArmijo * a) * racc || a <= kAlphaMin;
            if (accept) {
                const double target = fmax(out.rtol * out.res0[sys], floor_g);
                out.pending[sys] = 0;
                out.backtrack[sys] = 0;
                out.res_acc[sys] = rr;
                out.tgt[sys] = target;
                const bool stop = out.rtol > 0.0 && !bad && (rr <= target || (rr <= 1e3 * target && rr > 0.5 * racc));
                out.active[sys] = (!stop && !bad && it < out.max_iter && rr > 0.0) ? 1 : 0;
            } else {
                out.backtrack[sys] = 1;
            }
        }
        if (out.stats) {
            const double rout = re[I] * re[I] * (LAPSE ? lapse_edge_inv2(f, (size_t)ray * (I + 1) + I) : 1.0);
            const double b = c * rout * s_b;
            if (out.n_tot) out.n_tot[sys] = s_n;
            if (out.e_tot) out.e_tot[sys] = s_e;
            if (out.budget) out.budget[sys] = s_n - s_nold + b - s_q - s_nes;
            if (out.lum) out.lum[sys] = kCLight * rout * s_b;
        }
    }
}

// ---------------------------------------------------------------- debug Jacobian blocks

template <int NT>
__global__ __launch_bounds__(kBlock) void k_blocks(Shape sh, Fields f, const Consts* __restrict__ cs,
                                                   const double* __restrict__ psi, double* __restrict__ blocks) {
    const long long sys = blockIdx.x;
    const int I = sh.I, N = sh.N;
    const int ray = (int)(sys % sh.R);
    const double* re = f.r_edge + (size_t)ray * (I + 1);
    const double c = sh.c_dt;
    for (int i = threadIdx.x; i < I; i += kBlock) {
        const size_t cb = ((size_t)sys * I + i) * N;
        const ZoneGeom g = zone_geom(re, i, I, f, ray);
        double p[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) p[k] = k < N ? psi[cb + k] : 0.0;
        double si[NT], so[NT];
        double amp = 0.0;
        const bool nes = sh.terms & kNes;
        if (nes) {
            amp = f.nes_amp[(size_t)sys * I + i];
            nes_zone<NT>(cs, N, f.temp[(size_t)ray * I + i], p, si, so);
        }
        double d[NT];
        if (nes) {
#pragma unroll
            for (int j = 0; j < NT; ++j) d[j] = (j + 1 < N) ? exp(-cs->de[j] / f.temp[(size_t)ray * I + i]) : 0.0;
        }
        for (int k = 0; k < N; ++k) {
            double* row = blocks + (cb + k) * (size_t)(N + 2);
            double diag = 1.0, bm = 0.0, bp = 0.0;
            if (sh.terms & kDiffusion) {
                const double lam = inv_mfp(f, cb + k);
                const double rnu = (sh.limiter == 2 || sh.outer_bc == 2) ? f.r_nu[(size_t)(sys / sh.R) * N + k] : 0.0;
                auto limb = [&](double R) { return sh.limiter == 2 ? limb_factor(R, rnu) : -1.0; };
                double dHv_lo = 0.0, dHu_lo = 0.0, dHu_hi = 0.0, dHv_hi = 0.0;
                if (i > 0) {
                    const size_t cm = cb - N + k;
                    const EdgeFlux e = edge_flux(psi[cm], p[k], sqrt(lam * inv_mfp(f, cm)), g.D_lo,
                                                 sh.psi_floor, sh.limiter, limb(re[i]));
                    dHu_lo = e.dHu;
                    dHv_lo = e.dHv;
                }
                if (i + 1 < I) {
                    const size_t cp = cb + N + k;
                    const EdgeFlux e = edge_flux(p[k], psi[cp], sqrt(lam * inv_mfp(f, cp)), g.D_hi,
                                                 sh.psi_floor, sh.limiter, limb(re[i + 1]));
                    dHu_hi = e.dHu;
                    dHv_hi = e.dHv;
                } else if (sh.outer_bc == 1) {
                    dHu_hi = 1.0;
                } else if (sh.outer_bc == 2) {
                    const Ghost gh = outer_ghost(re[i], re[i + 1], rnu);
                    const EdgeFlux e = edge_flux(p[k], gh.ratio * p[k], lam, gh.D, sh.psi_floor, sh.limiter,
                                                 limb(re[i + 1]));
                    dHu_hi = e.dHu + gh.ratio * e.dHv;
                }
                diag += c * (g.A_hi * dHu_hi - g.A_lo * dHv_lo) / g.V;
                bp = (i + 1 < I) ? c * g.A_hi * dHv_hi / g.V : 0.0;
                bm = (i > 0) ? -c * g.A_lo * dHu_lo / g.V : 0.0;
            }
            if (sh.terms & kEmAbs) diag += c * (f.eta[cb + k] + f.kappa_a[cb + k]);
            const double pk = p[k];
            for (int kp = 0; kp < N; ++kp) {
                double v = 0.0;
                if (nes) {
                    // detailed-balance factor exp(-|eps_k - eps_k'|/T) as a neighbour product
                    double e = 1.0;
                    for (int j = min(k, kp); j < max(k, kp); ++j) e *= d[j];
                    const double kout = amp * cs->P[k][kp] * (kp > k ? e : 1.0);
                    const double kin = amp * cs->P[k][kp] * (kp < k ? e : 1.0);
                    v = -c * ((1.0 - pk) * kin + pk * kout);
                }
                row[kp] = v;
            }
            if (nes) diag += c * amp * (si[k] + so[k]);
            row[k] += diag;
            row[N] = bm;
            row[N + 1] = bp;
        }
    }
}

// ---------------------------------------------------------------- adjoint VJP

template <int NT>
__global__ __launch_bounds__(kBlock) void k_vjp(Shape sh, Fields f, const Consts* __restrict__ cs,
                                                const double* __restrict__ psi, const double* __restrict__ mu,
                                                double* g_ka, double* g_eta, double* g_ks, double* g_amp) {
    // one block per system, one thread per cell: rows of NT threads are zones, so a wave's loads of a
    // cell array (and of the neighbouring zones' cells) are contiguous
    constexpr int RZ = kBlock / NT;             // zones per chunk
    constexpr int PS = NT + 1;                  // padded LDS row stride
    __shared__ double s_P[NT * PS];
    __shared__ double s_p[RZ][PS];              // the zone's psi row
    __shared__ double s_d[RZ][PS];              // neighbour detailed-balance factors exp(-(eps_k+1 - eps_k)/T)
    __shared__ double s_m[RZ][PS];              // mu_k c dt
    __shared__ double s_s[RZ][PS];              // (1 - psi_k) S^in_k - psi_k S^out_k
    const long long sys = blockIdx.x;
    const int I = sh.I, N = sh.N;
    const int ray = (int)(sys % sh.R);
    const double* re = f.r_edge + (size_t)ray * (I + 1);
    const double c = sh.c_dt;
    const bool diff = sh.terms & kDiffusion, emabs = sh.terms & kEmAbs, nes = sh.terms & kNes;
    const bool amp = g_amp != nullptr;
    const int t = threadIdx.x, zl = t / NT, k = t - zl * NT;
    const bool tile = zl < RZ;
    const bool lane_ok = tile && k < N;
    if (amp && nes)
        for (int j = t; j < NT * NT; j += kBlock) s_P[(j / NT) * PS + (j % NT)] = cs->P[j / NT][j % NT];

    for (int z0 = 0; z0 < I; z0 += RZ) {
        const int i = z0 + zl;
        const bool in_zone = lane_ok && i < I;
        const size_t cb = ((size_t)sys * I + (in_zone ? i : 0)) * N + (in_zone ? k : 0);
        double pk = 0.0, m0 = 0.0;
        if (in_zone) {
            const ZoneGeom g = zone_geom(re, i, I, f, ray);
            pk = psi[cb];
            m0 = mu[cb];
            const double lam = inv_mfp(f, cb);
            double gchi = 0.0;     // sum over the two edges of (mu-weighted dG/dH) dH/dlam dlam/dchi
            if (diff) {
                const double rnu = (sh.limiter == 2 || sh.outer_bc == 2) ? f.r_nu[(size_t)(sys / sh.R) * N + k] : 0.0;
                auto limb = [&](double R) { return sh.limiter == 2 ? limb_factor(R, rnu) : -1.0; };
                if (i + 1 < I) {
                    const size_t cp = cb + N;
                    const double lam_e = sqrt(lam * inv_mfp(f, cp));
                    const EdgeFlux e = edge_flux(pk, psi[cp], lam_e, g.D_hi, sh.psi_floor, sh.limiter, limb(re[i + 1]));
                    const double w = c * g.A_hi * (m0 / g.V - mu[cp] / g.V_hi);
                    gchi += w * e.dHlam * (-0.5 * lam_e * lam);
                } else if (sh.outer_bc == 2) {
                    // the ghost-zone flux carries the last zone's own mean free path: dlam/dchi = -lam^2
                    const Ghost gh = outer_ghost(re[i], re[i + 1], rnu);
                    const EdgeFlux e = edge_flux(pk, gh.ratio * pk, lam, gh.D, sh.psi_floor, sh.limiter, limb(re[i + 1]));
                    gchi += c * g.A_hi * (m0 / g.V) * e.dHlam * (-lam * lam);
                }
                if (i > 0) {
                    const size_t cm = cb - N;
                    const double lam_e = sqrt(lam * inv_mfp(f, cm));
                    const EdgeFlux e = edge_flux(psi[cm], pk, lam_e, g.D_lo, sh.psi_floor, sh.limiter, limb(re[i]));
                    const double w = c * g.A_lo * (mu[cm] / g.V_lo - m0 / g.V);
                    gchi += w * e.dHlam * (-0.5 * lam_e * lam);
                }
            }
            // with a lapse the fields are lapse-folded (a kappa_a, a eta, and kappa_s carrying the rest of the
            // transport opacity): the gradient with respect to the caller's kappa_a and eta is a times that
            // with respect to the folded ones plus (1 - a) times the kappa_s one, i.e. the sources carry a
            const double az = f.lapse ? f.lapse[(size_t)ray * I + i] : 1.0;
            double gka = gchi, geta = gchi;
            if (emabs) {
                gka += az * m0 * c * pk;
                geta -= az * m0 * c * (1.0 - pk);
            }
            if (g_ka) g_ka[cb] = -gka;
            if (g_eta) g_eta[cb] = -geta;
            if (g_ks) g_ks[cb] = -gchi;
        }
        if (!amp) continue;
        if (nes) {
            // sum_k mu_k c [(1 - psi_k) S^in_k - psi_k S^out_k] over each zone (the NES source of the zone,
            // Phi_0 terms of eq. d8, differentiated with respect to its amplitude)
            __syncthreads();                                // previous chunk done with the rows
            if (tile) {
                s_p[zl][k] = pk;
                s_d[zl][k] = (in_zone && k + 1 < N) ? exp(-cs->de[k] / f.temp[(size_t)ray * I + i]) : 0.0;
            }
            __syncthreads();
            double s1 = 0.0;
            if (in_zone) {
                double sin_ = 0.0, sout = 0.0, e = 1.0;
                for (int kp = k + 1; kp < N; ++kp) {        // up-scatter side: out factor decays
                    e *= s_d[zl][kp - 1];
                    const double pp = s_p[zl][kp], P = s_P[k * PS + kp];
                    sout = fma(P * e, 1.0 - pp, sout);
                    sin_ = fma(P, pp, sin_);
                }
                e = 1.0;
                for (int kp = k - 1; kp >= 0; --kp) {       // down-scatter side: in factor decays
                    e *= s_d[zl][kp];
                    const double pp = s_p[zl][kp], P = s_P[k * PS + kp];
                    sin_ = fma(P * e, pp, sin_);
                    sout = fma(P, 1.0 - pp, sout);
                }
                s1 = (1.0 - pk) * sin_ - pk * sout;
            }
            if (tile) {
                s_m[zl][k] = m0 * c;
                s_s[zl][k] = s1;
            }
            __syncthreads();
            if (tile && k == 0 && i < I) {
                double ga = 0.0;
                for (int kk = 0; kk < N; ++kk) ga = fma(s_m[zl][kk], s_s[zl][kk], ga);
                // the folded amplitude is amp / a: the caller's amplitude gets 1/a of its gradient
                g_amp[(size_t)sys * I + i] = f.lapse ? ga / f.lapse[(size_t)ray * I + i] : ga;
            }
        } else if (tile && k == 0 && i < I) {
            g_amp[(size_t)sys * I + i] = 0.0;
        }
    }
}

// ---------------------------------------------------------------- lapse folding

// With a lapse the emission/absorption and NES sources of eq. a58 (times a_i c dt) carry a_i, and the NES
// kernels are evaluated at the local energies E / a_i.  Both are exact transformations of the inputs:
// kappa_a -> a kappa_a and eta -> a eta, with kappa_s -> kappa_s + (1 - a)(kappa_a + eta) so that the
// transport mean free path 1/(kappa_a + eta + kappa_s) is unchanged; the NES kernel's energy factor
// eps_k eps_k' / eps0^2 becomes 1/a^2 of its value at infinity and its exponent (eps_k' - eps_k)/T becomes
// (eps_k' - eps_k)/(a T), so amp -> amp / a (with the source's a) and T -> a T.
__global__ __launch_bounds__(kBlock) void k_lapse_fold(long long ncell, int N, long long RI, long long nsz,
                                                       const double* __restrict__ lapse,
                                                       const double* __restrict__ ka, const double* __restrict__ et,
                                                       const double* __restrict__ ks, const double* __restrict__ temp,
                                                       const double* __restrict__ amp, double* __restrict__ oka,
                                                       double* __restrict__ oet, double* __restrict__ oks,
                                                       double* __restrict__ otemp, double* __restrict__ oamp) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += stride) {
        const double a = lapse[(c / N) % RI];
        const double k_a = ka[c], e = et[c];
        oka[c] = a * k_a;
        oet[c] = a * e;
        oks[c] = ks[c] + (1.0 - a) * (k_a + e);
    }
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < nsz; j += stride) {
        const long long z = j % RI;
        if (amp) oamp[j] = amp[j] / lapse[z];
        if (temp && j < RI) otemp[j] = lapse[j] * temp[j];
    }
}

hipError_t launch_lapse_fold(const Shape& sh, const double* lapse, const double* ka, const double* et,
                             const double* ks, const double* temp, const double* amp, double* oka, double* oet,
                             double* oks, double* otemp, double* oamp, hipStream_t st) {
    const long long RI = (long long)sh.R * sh.I, nsz = (long long)sh.S * RI, ncell = nsz * sh.N;
    const long long blocks = std::min<long long>((ncell + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_lapse_fold, dim3((unsigned)blocks), dim3(kBlock), 0, st, ncell, sh.N, RI, nsz, lapse, ka, et,
                       ks, temp, amp, oka, oet, oks, otemp, oamp);
    return hipGetLastError();
}

// ---------------------------------------------------------------- luminosity seed

// dL_N/dpsi for L_N = c A_{I+1/2} sum_k W_k H_{I+1/2,k} with free streaming H = psi of the
// last zone: c R_{I+1/2}^2 W_k in the outermost zone (R^2 / a^2 with a lapse), zero elsewhere
// (and zero everywhere when there is no outgoing flux).
__global__ __launch_bounds__(kBlock) void k_lum_seed(Shape sh, const double* __restrict__ r_edge,
                                                     const double* __restrict__ lapse_edge,
                                                     const Consts* __restrict__ cs, const double* add,
                                                     double* seed) {
    const long long sys = blockIdx.x;
    const int I = sh.I, N = sh.N;
    const int ray = (int)(sys % sh.R);
    const bool flux = (sh.terms & kDiffusion) && sh.outer_bc == 1;
    const size_t eo = (size_t)ray * (I + 1) + I;
    const double ae = lapse_edge ? lapse_edge[eo] : 1.0;      // with a lapse the area is R^2 / a^2
    const double ro = r_edge[eo] / ae;
    const size_t n = (size_t)I * N;
    for (size_t j = threadIdx.x; j < n; j += kBlock) {
        const int i = (int)(j / N), k = (int)(j % N);
        const size_t c = (size_t)sys * n + j;
        const double a = add ? add[c] : 0.0;
        seed[c] = ((flux && i == I - 1) ? kCLight * ro * ro * cs->W[k] : 0.0) + a;
    }
}

hipError_t launch_lum_seed(const Shape& sh, const double* r_edge, const double* lapse_edge, const Consts* cs,
                           const double* add, double* seed, hipStream_t st) {
    const long long nsys = (long long)sh.S * sh.R;
    hipLaunchKernelGGL(k_lum_seed, dim3((unsigned)nsys), dim3(kBlock), 0, st, sh, r_edge, lapse_edge, cs, add, seed);
    return hipGetLastError();
}

// ---------------------------------------------------------------- line-search backtrack

__global__ __launch_bounds__(kBlock) void k_backtrack(Shape sh, double* __restrict__ psi, const double* __restrict__ dx,
                                                      int* backtrack, double* alpha) {
    const long long sys = blockIdx.x;
    if (backtrack[sys] == 0) return;
    const double a = alpha[sys];
    const double coef = 0.5 * a - a;
    const size_t n = (size_t)sh.I * sh.N;
    for (size_t j = threadIdx.x; j < n; j += kBlock) {
        const size_t cix = (size_t)sys * n + j;
        psi[cix] = psi[cix] + __dmul_rn(coef, dx[cix]);      // trial moved back to alpha / 2
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        alpha[sys] = 0.5 * a;
        backtrack[sys] = 0;
    }
}

hipError_t launch_backtrack(const Shape& sh, double* psi, const double* dx, int* backtrack, double* alpha,
                            hipStream_t st) {
    const long long nsys = (long long)sh.S * sh.R;
    hipLaunchKernelGGL(k_backtrack, dim3((unsigned)nsys), dim3(kBlock), 0, st, sh, psi, dx, backtrack, alpha);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fill (a kernel rather than a memset node)

__global__ __launch_bounds__(kBlock) void k_fill_i32(int* __restrict__ p, long long n, int v) {
    const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (j < n) p[j] = v;
}

hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------- active-system count

// max |v| over each system's cells (one block per system)
__global__ __launch_bounds__(kBlock) void k_sys_absmax(const double* __restrict__ v, long long per_sys,
                                                       double* __restrict__ out) {
    __shared__ double red[kBlock / 64];
    const double* p = v + (size_t)blockIdx.x * per_sys;
    double m = 0.0;
    for (long long c = threadIdx.x; c < per_sys; c += kBlock) m = fmax(m, fabs(p[c]));
    m = block_max(m, red);
    if (threadIdx.x == 0) out[blockIdx.x] = m;
}

hipError_t launch_sys_absmax(const double* v, long long nsys, long long per_sys, double* out, hipStream_t st) {
    if (nsys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sys_absmax, dim3((unsigned)nsys), dim3(kBlock), 0, st, v, per_sys, out);
    return hipGetLastError();
}

// Final per-system flags of a Newton step from the last evaluated (accepted) residual: keeps the
// factorisation's zero-pivot / fallback bits, sets 1 when rtol > 0 and max|G| is above its target,
// 2 when the residual is not finite.
__global__ __launch_bounds__(kBlock) void k_final_flags(long long n, const double* __restrict__ res,
                                                        const double* __restrict__ tgt, double rtol,
                                                        int* __restrict__ flags) {
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const double r = res[s];
    int fl = flags[s] & (4 | 8);
    if (!isfinite(r)) fl |= 2;
    else if (rtol > 0.0 && !(r <= tgt[s])) fl |= 1;
    flags[s] = fl;
}

hipError_t launch_final_flags(long long n, const double* res, const double* tgt, double rtol, int* flags,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_final_flags, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, res,
                       tgt, rtol, flags);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_count(const int* __restrict__ active, long long n, int* count) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (long long j = threadIdx.x; j < n; j += kBlock) s += active[j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *count = (int)s;
}

hipError_t launch_count_active(const int* active, long long n, int* count, hipStream_t st) {
    hipLaunchKernelGGL(k_count, dim3(1), dim3(kBlock), 0, st, active, n, count);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_mark(const int* __restrict__ guard, long long n, int* __restrict__ act,
                                                 int* count) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (long long j = threadIdx.x; j < n; j += kBlock) {
        const int v = guard[j] != 0;
        act[j] = v;
        s += v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) *count = (int)s;
}

__global__ __launch_bounds__(kBlock) void k_count_bits(const int* __restrict__ flags, long long n, int mask,
                                                       int* count) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (long long j = threadIdx.x; j < n; j += kBlock) s += (flags[j] & mask) != 0;
    s = block_sum(s, red);
    if (threadIdx.x == 0) *count = (int)s;
}

hipError_t launch_count_bits(const int* flags, long long n, int mask, int* count, hipStream_t st) {
    hipLaunchKernelGGL(k_count_bits, dim3(1), dim3(kBlock), 0, st, flags, n, mask, count);
    return hipGetLastError();
}

hipError_t launch_mark(const int* guard, long long n, int* active_out, int* count, hipStream_t st) {
    hipLaunchKernelGGL(k_mark, dim3(1), dim3(kBlock), 0, st, guard, n, active_out, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch on the padded group count

int padded_groups(int N) {
    static const int sizes[] = {4, 8, 12, 16, 20, 24, 28, 32};
    for (int s : sizes)
        if (N <= s) return s;
    return -1;
}

#define TM_DISPATCH_NT(NTV, ...)                                       \
    switch (NTV) {                                                     \
        case 4: { constexpr int NT = 4; __VA_ARGS__; } break;          \
        case 8: { constexpr int NT = 8; __VA_ARGS__; } break;          \
        case 12: { constexpr int NT = 12; __VA_ARGS__; } break;        \
        case 16: { constexpr int NT = 16; __VA_ARGS__; } break;        \
        case 20: { constexpr int NT = 20; __VA_ARGS__; } break;        \
        case 24: { constexpr int NT = 24; __VA_ARGS__; } break;        \
        case 28: { constexpr int NT = 28; __VA_ARGS__; } break;        \
        case 32: { constexpr int NT = 32; __VA_ARGS__; } break;        \
        default: return hipErrorInvalidValue;                          \
    }

hipError_t launch_residual(const Shape& sh, const Fields& f, const Consts* cs, const double* psi_n,
                           const double* psi, double* G_out, double g_sign, const ResidualOut& out,
                           hipStream_t st) {
    const long long nsys = (long long)sh.S * sh.R;
    if (sh.limiter == 2 || sh.outer_bc == 2) {
        TM_DISPATCH_NT(padded_groups(sh.N),
                       hipLaunchKernelGGL((k_residual<NT, true, true>), dim3((unsigned)nsys), dim3(kBlock), 0, st, sh,
                                          f, cs, psi_n, psi, G_out, g_sign, out));
    } else if (f.lapse) {
        TM_DISPATCH_NT(padded_groups(sh.N),
                       hipLaunchKernelGGL((k_residual<NT, true, false>), dim3((unsigned)nsys), dim3(kBlock), 0, st, sh,
                                          f, cs, psi_n, psi, G_out, g_sign, out));
    } else {
        TM_DISPATCH_NT(padded_groups(sh.N),
                       hipLaunchKernelGGL((k_residual<NT, false, false>), dim3((unsigned)nsys), dim3(kBlock), 0, st, sh,
                                          f, cs, psi_n, psi, G_out, g_sign, out));
    }
    return hipGetLastError();
}

hipError_t launch_blocks(const Shape& sh, const Fields& f, const Consts* cs, const double* psi, double* blocks,
                         hipStream_t st) {
    const long long nsys = (long long)sh.S * sh.R;
    TM_DISPATCH_NT(padded_groups(sh.N),
                   hipLaunchKernelGGL(k_blocks<NT>, dim3((unsigned)nsys), dim3(kBlock), 0, st, sh, f, cs, psi,
                                      blocks));
    return hipGetLastError();
}

hipError_t launch_vjp(const Shape& sh, const Fields& f, const Consts* cs, const double* psi, const double* mu,
                      double* g_ka, double* g_eta, double* g_ks, double* g_amp, hipStream_t st) {
    const long long nsys = (long long)sh.S * sh.R;
    TM_DISPATCH_NT(padded_groups(sh.N),
                   hipLaunchKernelGGL(k_vjp<NT>, dim3((unsigned)nsys), dim3(kBlock), 0, st, sh, f, cs, psi, mu,
                                      g_ka, g_eta, g_ks, g_amp));
    return hipGetLastError();
}

}  // namespace tmk
