// Y_e-coupled transport step: the electron-fraction equation (eq. a62a) solved together with the
// electron neutrinos and antineutrinos of each ray (linearised system, eqs. a62ac-a62ae), and the
// matter energy change and temperature after the step (eqs. a62b, a62d).
//
// Unknowns per zone: psi of nu_e (species 0) in rows [0, N), psi of anti-nu_e (species 1) in rows
// [NT, NT + N), Y_e in row 2 NT (NT = N padded to a multiple of 4; padded rows are identity rows).
// Y_e has no radial coupling, so the off-diagonal blocks stay diagonal with zero Y_e entries and the
// diagonal blocks are (2 NT + 1)-square.  The transport mean free path stays at Y_e^n during the step;
// the absorption and emission opacities of the pair are linear in Y_e over the step, with their
// derivatives given as inputs.
//
//   k_ye_couple       one block per ray: completes the species residual (evaluated by the
//                     single-species residual kernel with the opacities of Y_e^n) with the Y_e terms,
//                     evaluates the Y_e residual, max|G|, the rounding level, the lepton number and the
//                     Newton/line-search decisions.
//   k_ye_factor       one wavefront per ray: lane r owns row r of the coupled block.  Per zone the row is
//                     assembled in registers, the Schur complement with the previous factor row is
//                     formed, and in-place Gauss-Jordan elimination with partial pivoting (pivot search
//                     as a max over the wavefront, pivot row read from the pivot lane into scalar
//                     registers) produces
//                     C_i = Ahat_i^{-1} diag(bp_i) and y_i; the backward sweep x_i = y_i - C_i x_{i+1}
//                     applies the Newton update.  The default instance (TILE) eliminates with diagonal
//                     pivots instead, the block spread over 8 x 8 lane tiles, so each step moves 2 T
//                     values per lane through LDS instead of M + 1 broadcasts; a ray that trips its growth
//                     guard is left untouched and re-run by the partial-pivoting instance.
//   k_ye_backtrack    line-search move-back of rejected trials.
//   k_ye_temperature  one thread per zone: energy-weighted collision sources of every species, the
//                     matter energy change and the new temperature.
#include "tm_kernels.hpp"

namespace tmk {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// zeta of eq. a62a at density rho: neutrinos per baryon per unit sum_k W_k psi
__device__ __forceinline__ double ye_zeta(double rho) { return kFourPiOverHc3 * kBaryonMassG / rho; }

// ---------------------------------------------------------------- residual completion and decisions

// PAIR compiles the pair sources in (their loops double the kernel's registers); the launch takes it
// when pair inputs are given.
template <int NT, bool PAIR>
__global__ __launch_bounds__(kBlock) void k_ye_couple(Shape sh, Fields f, YeFields y, const Consts* __restrict__ cs,
                                                      const double* __restrict__ psi, const double* __restrict__ ye,
                                                      double* __restrict__ G, double* __restrict__ GY,
                                                      const double* __restrict__ level_sp, YeOut out) {
    __shared__ double red[kBlock / 64];
    const long long ray = blockIdx.x;
    if (out.mode == kResTrial && out.pending[ray] == 0) return;          // no trial to evaluate
    const int R = sh.R, I = sh.I, N = sh.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane < NT ? 0 : 1;
    const int k = lane - q * NT;
    const bool real = lane < 2 * NT && k < N;                            // species q, group k
    const int kk = real ? k : 0;
    const double sgn = q == 0 ? 1.0 : -1.0;                              // nu_e carries +1, anti-nu_e -1
    const double Wk = real ? cs->W[kk] : 0.0;
    const double c = sh.c_dt;
    const bool emabs = sh.terms & kEmAbs;
    const double* re = f.r_edge + (size_t)ray * (I + 1);
    const size_t cell0 = ((size_t)(real ? q : 0) * R + ray) * I * N;
    const size_t zb = (size_t)ray * I;

    double gmax = 0.0, mag_max = 0.0, lep = 0.0;
    int bad = 0;
    const bool pair = PAIR && y.pair_amp != nullptr;
    __shared__ double s_pair[PAIR ? kBlock / 64 : 1][3][64];   // psi, flux factor, limb cosine of both species' groups
    __shared__ double s_bz[PAIR ? kBlock / 64 : 1][NT];        // exp(-eps_j / T) of the zone
    for (int i = wave; i < I; i += kBlock / 64) {
        const double Y = ye[zb + i], Yn = y.ye_n[zb + i];
        const double dy = Y - Yn;
        double sY = 0.0, sAbs = 0.0, sD = 0.0, sL = 0.0;
        double spair = 0.0;
        if (pair) {
            // pair sources of the zone (eqs. d11-d14, Phi_0 terms, chi of eqs. d16-d22)
            const double Rz = 0.5 * (re[i] + re[i + 1]);
            double pown = 0.0, eown = 0.0, mown = 0.0;
            if (real) {
                const size_t ci = cell0 + (size_t)i * N + kk;
                pown = psi[ci];
                eown = y.pair_eta1[ci];
                mown = pair_limb_cosine(f.r_nu[(size_t)q * N + kk] / Rz);
            }
            s_pair[wave][0][lane] = pown;
            s_pair[wave][1][lane] = eown;
            s_pair[wave][2][lane] = mown;
            if (lane < NT) s_bz[wave][lane] = lane < N ? exp(-cs->eps[lane] / f.temp[zb + i]) : 0.0;
            wave_sync();
            if (real) {
                const double a = y.pair_amp[zb + i], iw = 1.0 / cs->wbar, bzk = s_bz[wave][kk];
                const int o = (1 - q) * NT;
                double cre = 0.0, ann = 0.0;
                for (int kp = 0; kp < N; ++kp) {
                    const double qa = a * y.pair_g[(size_t)kk * N + kp] * cs->W[kp] * iw;
                    const double pb = s_pair[wave][0][o + kp];
                    cre = fma(qa * bzk * s_bz[wave][kp], 1.0 - pb, cre);
                    ann = fma(qa * pair_chi(eown, s_pair[wave][1][o + kp], mown, s_pair[wave][2][o + kp]), pb, ann);
                }
                spair = (1.0 - pown) * cre - pown * ann;
                // rounding level of the pair terms, counted as the other sources are
                mag_max = fmax(mag_max, fabs(pown) + c * (fabs((1.0 - pown) * cre) + fabs(pown * ann))
                                            + fabs(pown) * c * (cre + ann));
            }
            wave_sync();                               // the rows are rewritten for this wave's next zone
        }
        if (real) {
            const size_t ci = cell0 + (size_t)i * N + kk;
            const double p = psi[ci];
            double g = G[ci] - c * spair;
            if (emabs) {
                // with a lapse the fields are lapse-folded (a kappa_a, a eta): the derivatives get the same a
                const double az = f.lapse ? f.lapse[zb + i] : 1.0;
                const double dka = az * y.dka[ci], det = az * y.deta[ci];
                g += c * dy * (dka * p - det * (1.0 - p));              // opacities at Y_e instead of Y_e^n
                const double em = (f.eta[ci] + dy * det) * (1.0 - p);
                const double ab = (f.kappa_a[ci] + dy * dka) * p;
                sY = sgn * Wk * (em - ab);
                sAbs = Wk * (fabs(em) + fabs(ab));
                sD = sgn * Wk * (det * (1.0 - p) - dka * p);
            }
            G[ci] = g;
            sL = sgn * Wk * p;
            bad |= !isfinite(g);
            gmax = fmax(gmax, fabs(g));
        }
        sY = wave_sum(sY);
        sAbs = wave_sum(sAbs);
        sD = wave_sum(sD);
        sL = wave_sum(sL);
        if (lane == 0) {
            const double rho = y.rho[zb + i];
            // with a lapse: the neutrinos of the zone number (V / a^3) sum_k W_k psi and the folded sources
            // carry a, so the Y_e rate per unit folded source is zeta / a^3
            const double ai3 = f.lapse ? 1.0 / (f.lapse[zb + i] * f.lapse[zb + i] * f.lapse[zb + i]) : 1.0;
            const double z = ye_zeta(rho) * ai3;
            double gy = dy, mag = fabs(Y) + fabs(Yn), ayy = 1.0;
            if (emabs) {
                gy += c * z * sY;                                        // eq. a62a times c dt
                mag += c * z * sAbs;
                ayy += c * z * sD;
            }
            mag += fabs(Y) * fabs(ayy);
            GY[zb + i] = gy;
            bad |= !isfinite(gy);
            gmax = fmax(gmax, fabs(gy));
            mag_max = fmax(mag_max, mag);
            lep += shell_volume(re[i], re[i + 1]) * (rho * Y / kBaryonMassG + kFourPiOverHc3 * ai3 * sL);
        }
    }
    const double res = block_max(gmax, red);
    const double mag = block_max(mag_max, red);
    bad = block_or(bad, red);
    if (out.lepton) lep = block_sum(lep, red);
    if (threadIdx.x == 0) {
        const double rr = bad ? __builtin_nan("") : res;
        out.res[ray] = rr;
        const double floor_g = fmax(fmax(level_sp[ray], level_sp[R + ray]), 32.0 * 2.220446049250313e-16 * mag);
        const int it = out.iters ? out.iters[ray] : 0;
        if (out.mode == kResInitial) {
            const double target = fmax(out.rtol * rr, floor_g);
            out.res0[ray] = rr;
            out.res_acc[ray] = rr;
            out.tgt[ray] = target;
            const bool stop = out.rtol > 0.0 && !bad && rr <= target;
            out.active[ray] = (!stop && !bad && it < out.max_iter && rr > 0.0) ? 1 : 0;
        } else {
            // same line search and stopping rule as the single-species step, on the whole coupled system
            const double racc = out.res_acc[ray], a = out.alpha[ray];
            const bool near = racc <= 1e3 * out.tgt[ray];
            const bool accept = near || rr <= (1.0 - kArmijo * a) * racc || a <= kAlphaMin;
            if (accept) {
                const double target = fmax(out.rtol * out.res0[ray], floor_g);
                out.pending[ray] = 0;
                out.backtrack[ray] = 0;
                out.res_acc[ray] = rr;
                out.tgt[ray] = target;
                const bool stop = out.rtol > 0.0 && !bad && (rr <= target || (rr <= 1e3 * target && rr > 0.5 * racc));
                out.active[ray] = (!stop && !bad && it < out.max_iter && rr > 0.0) ? 1 : 0;
            } else {
                out.backtrack[ray] = 1;
            }
        }
        if (out.lepton) out.lepton[ray] = lep;
    }
}

// ---------------------------------------------------------------- coupled block-Thomas factor and solve

template <int NT>
struct alignas(16) YeLds {
    static constexpr int MT = 2 * NT + 1;
    double prow[MT + 3];       // pivot row: [0, MT) entries, MT right-hand side, MT+1 diagonal of B
    double bc[2 * NT];         // psi of the zone (both species); x_{i+1} in the backward sweep
    double dd[NT];             // NES neighbour factors exp(-(eps_{j+1} - eps_j)/T)
    double pe[2 * NT];         // pair processes: flux factors psi1/psi0 of the zone (both species)
    double pm[2 * NT];         // ... and the limb cosines of eq. d22 at the zone centre
    double bz[NT];             // ... and exp(-eps_j / T) of the zone
    double yr[2 * NT];         // Y_e row entries, one per species row
    double ys[2 * NT];         // species terms of dG_Y/dY_e
    double fix[MT][MT + 1];    // row-ownership fix-up after pivoting; the rows between zones
    int plane[MT];             // pivot lane of each elimination step
    // tiled elimination: pivot row (entries, then g) and pivot column of each step, double-buffered
    double urow[2][8 * ((MT + 8) / 8)];
    double ucol[2][8 * ((MT + 8) / 8)];
    double bpv[MT];            // B coefficient of every row
    double pivs[MT];           // pivot of every step
};

template <int NT>
constexpr int ye_waves_per_block() { return NT <= 20 ? 4 : 2; }

// value of v in lane p (p uniform over the wavefront), as a scalar
__device__ __forceinline__ double lane_value(double v, int p) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, p);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), p);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One zone's slot of the coupled factor workspace: C_i's row of lane l (NC values) as NC/2 runs of MT
// pairs, pair j at [j MT + l], then y_i at [NC MT + l].  The slot stride is rounded up to an even number
// of doubles so that every pair is 16-byte aligned.
typedef double yd2 __attribute__((ext_vector_type(2)));
template <int NT>
constexpr size_t ye_slot_doubles() {
    constexpr size_t n = (size_t)(2 * NT + 1) * (2 * NT + 1);
    return n + (n & 1);
}
template <int NC, int MT>
__device__ __forceinline__ void store_slot(double* slot, int lane, const double* row, double y) {
#pragma unroll
    for (int j = 0; j < NC / 2; ++j) {
        const yd2 v = {row[2 * j], row[2 * j + 1]};
        nt_store(reinterpret_cast<yd2*>(slot) + (size_t)j * MT + lane, v);
    }
    nt_store(slot + (size_t)NC * MT + lane, y);
}
template <int NC, int MT>
__device__ __forceinline__ void load_slot(const double* slot, int lane, bool ok, double (&c)[NC], double& y) {
#pragma unroll
    for (int j = 0; j < NC / 2; ++j) {
        const yd2 v = nt_load(reinterpret_cast<const yd2*>(slot) + (size_t)j * MT + lane);
        c[2 * j] = ok ? v.x : 0.0;
        c[2 * j + 1] = ok ? v.y : 0.0;
    }
    const double yy = nt_load(slot + (size_t)NC * MT + lane);
    y = ok ? yy : 0.0;
}

// waves per SIMD the register allocation is held to: two up to 20 groups (256 VGPRs, no scratch), one above
template <int NT>
constexpr int ye_waves_per_eu() { return NT <= 20 ? 2 : 1; }

// In-place Gauss-Jordan on [Ahat | diag(bp) | g] with diagonal pivots, the block and g spread over the
// wavefront as 8 x 8 tiles of T x T entries (T = ceil((MT + 1) / 8), g being column MT): lane 8 a + b holds
// rows T a .. T a + T - 1 and columns T b .. T b + T - 1.  Step cc needs, in each lane, the pivot row's
// entries of its columns and the pivot column's entries of its rows: the lanes holding them put them in
// LDS (T values per lane, double-buffered between steps) and every lane reads its 2 T values back,
// instead of all M + 1 values of the pivot row.  Column cc becomes column cc of C = Ahat^-1 diag(bp) as
// in the row-per-lane elimination; each row is divided by its pivot at the end.  Reads the rows and g
// from L.fix, the B coefficients from L.bpv; writes C and y back to L.fix in natural order.  bad is set
// for a multiplier above limit (growth guard) or a zero or non-finite pivot.
template <int MT, typename Lds>
__device__ __forceinline__ void tile_eliminate(Lds& L, int lane, double limit, bool& bad) {
    constexpr int T = (MT + 8) / 8;
    // the lane id through an opaque copy: the lane masks of the steps are then formed per zone instead of
    // being hoisted out of the zone loop into scalar registers held across the row assembly
    int lo = lane;
    asm volatile("" : "+v"(lo));
    const int ta = lo >> 3, tb = lo & 7;
    // growth guard: at every step each lane checks one multiplier, entry T ta + (tb mod T) of the pivot
    // column, so the eight lanes of a tile row cover its T rows and the wavefront covers the column
    const int gs = T * ta + tb % T;
    double t[T][T];
    double gmax = 0.0;
#pragma unroll
    for (int tr = 0; tr < T; ++tr) {
        const int r = T * ta + tr;
#pragma unroll
        for (int tc = 0; tc < T; ++tc) {
            const int c = T * tb + tc;
            const bool in = r < MT && c <= MT;
            t[tr][tc] = in ? L.fix[in ? r : 0][in ? c : 0] : ((r == c && c != MT) ? 1.0 : 0.0);   // padding: identity
        }
    }
#pragma unroll
    for (int cc = 0; cc < MT; ++cc) {
        const int ap = cc / T, rp = cc % T;            // tile row and column of the pivot: lane 9 ap, (rp, rp)
        double* const ur = L.urow[cc & 1];
        double* const uc = L.ucol[cc & 1];
        if (ta == ap) {
#pragma unroll
            for (int tc = 0; tc < T; ++tc) ur[T * tb + tc] = t[rp][tc];
        }
        if (tb == ap) {                                // the pivot itself goes in as 0: its row's multiplier
#pragma unroll
            for (int tr = 0; tr < T; ++tr) uc[T * ta + tr] = (tr == rp && ta == ap) ? 0.0 : t[tr][rp];
        }
        wave_sync();
        const double piv = ur[cc], bpiv = L.bpv[cc];
        const double npinv = -drcp(piv);
        if (lane == 0) L.pivs[cc] = piv;
        double u[T], nf[T];                            // nf: minus the multipliers
#pragma unroll
        for (int tc = 0; tc < T; ++tc) u[tc] = ur[T * tb + tc];
#pragma unroll
        for (int tr = 0; tr < T; ++tr) nf[tr] = uc[T * ta + tr] * npinv;   // 0 for the pivot row itself
        gmax = fmax(gmax, fabs(uc[gs] * npinv));
#pragma unroll
        for (int tr = 0; tr < T; ++tr)
#pragma unroll
            for (int tc = 0; tc < T; ++tc) t[tr][tc] = fma(nf[tr], u[tc], t[tr][tc]);
        if (tb == ap) {                                // column cc: -f bp_cc, and bp_cc in the pivot row
#pragma unroll
            for (int tr = 0; tr < T; ++tr) t[tr][rp] = (tr == rp && ta == ap) ? bpiv : nf[tr] * bpiv;
        }
        // every entry is materialised at the end of its step: left alone, the compiler sinks each update to
        // the entry's next use and holds every earlier step's multipliers and pivot-row values live
#pragma unroll
        for (int tr = 0; tr < T; ++tr)
#pragma unroll
            for (int tc = 0; tc < T; ++tc) asm volatile("" : "+v"(t[tr][tc]));
        asm volatile("" : "+v"(gmax));
    }
    bad |= !(gmax <= limit);
    wave_sync();                                       // pivs[] is read by other lanes
#pragma unroll
    for (int tr = 0; tr < T; ++tr) {
        const int r = T * ta + tr;
        if (r >= MT) continue;
        const double pv = L.pivs[r];
        bad |= !(fabs(pv) > 0.0) || !isfinite(pv);
        const double ip = drcp(pv);
#pragma unroll
        for (int tc = 0; tc < T; ++tc) {
            const int c = T * tb + tc;
            if (c <= MT) L.fix[r][c] = t[tr][tc] * ip;
        }
    }
    wave_sync();
}

// EXT: the geometric limiter and outer boundary, the pair processes and the lapse compiled in (instantiated
// separately, at one wave per SIMD, and launched only for problems that ask for any of them).
// TILE: the elimination with diagonal pivots on 8 x 8 lane tiles (below) instead of partial pivoting
// with one row per lane.
template <int NT, int WEU, bool EXT, bool TILE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WEU))) void k_ye_factor(YeFactorArgs A) {
    constexpr int MT = 2 * NT + 1;              // rows of a coupled block (<= 57)
    constexpr int NC = 2 * NT;                  // columns of C that can be non-zero (Y_e has bp = 0)
    constexpr int WPB = ye_waves_per_block<NT>();
    constexpr int PS = NT + 2;
    __shared__ YeLds<NT> lds_all[WPB];
    __shared__ double s_P[NT * PS];
    for (int j = threadIdx.x; j < NT * NT; j += blockDim.x) s_P[(j / NT) * PS + (j % NT)] = A.cs->P[j / NT][j % NT];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: ray addressing stays scalar
    const long long rb = (long long)blockIdx.x * WPB + wave;           // ray within the batch
    if (rb >= A.nray) return;                                          // whole wave (no block barrier follows)
    const long long ray = A.ray0 + rb;
    if (A.active && A.active[ray] == 0) return;
    if (!TILE && A.redo && A.redo[ray] == 0) return;                   // the re-run takes marked rays only

    YeLds<NT>& L = lds_all[wave];
    const Shape& sh = A.sh;
    const int N = sh.N, I = sh.I, R = sh.R;
    const bool is_row = lane < MT;
    const bool isY = lane == NC;
    const int q = lane < NT ? 0 : 1;
    const int k = lane - q * NT;
    const bool q0 = q == 0;
    const bool real = lane < NC && k < N;        // a species row of a real energy group
    const int kk = real ? k : 0;
    const int kr = is_row ? lane : 0;
    const double sgn = q0 ? 1.0 : -1.0;
    const size_t cell0 = ((size_t)(real ? q : 0) * R + ray) * I * N;
    const double* psi = A.psi + cell0;
    const double* ka = A.f.kappa_a + cell0;
    const double* et = A.f.eta + cell0;
    const double* ks = A.f.kappa_s + cell0;
    const double* dka = A.y.dka + cell0;
    const double* det = A.y.deta + cell0;
    const double* rhs = A.G + cell0;
    const size_t zb = (size_t)ray * I;
    const double* re = A.f.r_edge + (size_t)ray * (I + 1);
    const double* tz = A.f.temp + zb;
    const bool diff = sh.terms & kDiffusion, emabs = sh.terms & kEmAbs, nes = sh.terms & kNes;
    const double* az = nes ? A.f.nes_amp + ((size_t)(real ? q : 0) * R + ray) * I : nullptr;
    const double c = sh.c_dt;
    const double Wk = real ? A.cs->W[kk] : 0.0;
    const double* Prow = s_P + kk * PS;
    // zone i's slot, ye_slot_doubles(NT) doubles (16-byte aligned): C as NC/2 runs of MT pairs (columns
    // 2j, 2j+1 of lane l at pair j MT + l, one 16-byte store or load per lane and run), then y [MT]
    constexpr size_t SZ = ye_slot_doubles<NT>();
    double* ws = A.ws + (size_t)rb * I * SZ;

    // ---------------------------------------------------------------- forward sweep
    // L.fix holds, between zones, the rows of C_{i-1} (columns [0, MT)) and y_{i-1} (column MT) in natural
    // order.  Each zone: (1) every lane turns its row of that matrix into its row of
    // Ahat_i = A_i - diag(bm_i) C_{i-1} in place (storing C_{i-1}, y_{i-1} to the workspace on the way), so
    // no register-held row is live during the assembly; (2) the row is loaded into registers for the
    // elimination; (3) the eliminated rows go back to L.fix in natural order.
    if (is_row) {
#pragma unroll
        for (int m = 0; m <= MT; ++m) L.fix[kr][m] = 0.0;
    }
    double* frow = L.fix[kr];
    // NES neighbour factors exp(-(eps_{j+1} - eps_j)/T) of every zone, computed before the sweep by lane j and
    // parked in the first row of the zone's workspace slot: the sweep reads them back in that zone and the same
    // lane overwrites them with C only in the next zone.  Out of the zone loop, the exponential's constants do not
    // stay live across the elimination.
    if (nes && lane < NT) {
        const double dej = lane + 1 < N ? A.cs->de[lane] : 0.0;
        for (int i = 0; i < I; ++i)
            ws[(size_t)i * SZ + lane] = (lane + 1 < N) ? exp(-dej / tz[i]) : 0.0;
    }
    double psi_c = real ? psi[kk] : 0.0;
    double sig_c = real ? ka[kk] + et[kk] : 0.0;
    double lam_c = real ? drcp(sig_c + ks[kk]) : 1.0;
    double dHu_lo = 0.0, dHv_lo = 0.0;
    bool zp = false;

    for (int i = 0; i < I; ++i) {
        // lane and group indices re-materialised per zone: comparisons with them are evaluated where used
        // instead of being hoisted out of the zone loop as dozens of live lane masks
        int lz = lane, kz = k;
        asm volatile("" : "+v"(lz), "+v"(kz));
        double psi_n1 = 0.0, sig_n1 = 0.0, lam_n1 = 1.0;
        if (i + 1 < I && real) {
            const size_t cn = (size_t)(i + 1) * N + kk;
            psi_n1 = psi[cn];
            sig_n1 = ka[cn] + et[cn];
            lam_n1 = drcp(sig_n1 + ks[cn]);
        }
        const double rlo = re[i], rhi = re[i + 1];
        double iV = drcp(shell_volume(rlo, rhi));
        double A_lo = rlo * rlo, A_hi = rhi * rhi;
        double alz = 1.0;                              // lapse of the zone (eq. a58 times a_i c dt: a^3/V, A/a^2)
        if (EXT && A.f.lapse) {
            alz = A.f.lapse[zb + i];
            const double e0 = A.f.lapse_edge[(size_t)ray * (I + 1) + i], e1 = A.f.lapse_edge[(size_t)ray * (I + 1) + i + 1];
            iV *= alz * alz * alz;
            A_lo /= e0 * e0;
            A_hi /= e1 * e1;
        }
        double dHu_hi = 0.0, dHv_hi = 0.0;
        if (i + 1 < I) {
            const double D_hi = 0.5 * (rhi + re[i + 2]) - 0.5 * (rlo + rhi);
            if (diff && real) {
                const double limb = (EXT && sh.limiter == 2) ? limb_factor(rhi, A.f.r_nu[(size_t)q * N + kk]) : -1.0;
                const EdgeFlux e = edge_flux(psi_c, psi_n1, sqrt(lam_c * lam_n1), D_hi, sh.psi_floor, sh.limiter, limb);
                dHu_hi = e.dHu;
                dHv_hi = e.dHv;
            }
        } else if (sh.outer_bc == 1) {
            dHu_hi = 1.0;                                   // free streaming: H = psi of the last zone
        } else if (EXT && sh.outer_bc == 2 && diff && real) {     // ghost zone of eq. a62af
            const double rnu = A.f.r_nu[(size_t)q * N + kk];
            const Ghost gh = outer_ghost(rlo, rhi, rnu);
            const EdgeFlux e = edge_flux(psi_c, gh.ratio * psi_c, lam_c, gh.D, sh.psi_floor, sh.limiter,
                                         sh.limiter == 2 ? limb_factor(rhi, rnu) : -1.0);
            dHu_hi = e.dHu + gh.ratio * e.dHv;
        }
        double diag = 1.0, bm = 0.0, bp = 0.0;
        if (diff) {
            diag += c * (A_hi * dHu_hi - A_lo * dHv_lo) * iV;
            if (i + 1 < I) bp = c * A_hi * dHv_hi * iV;
            if (i > 0) bm = -c * A_lo * dHu_lo * iV;
        }
        if (emabs) diag += c * sig_c;
        if (!real) bm = bp = 0.0;

        // Y_e terms of the zone (eq. a62ad: Y_e column of the species rows; eq. a62a: the Y_e row)
        const double dy = A.ye[zb + i] - A.y.ye_n[zb + i];
        // with a lapse the fields are lapse-folded: the opacity derivatives carry a as well, and the Y_e rate
        // per unit folded source is zeta / a^3
        const double z = ye_zeta(A.y.rho[zb + i]) / (alz * alz * alz);
        double ycol = 0.0, yrow = 0.0, ysum = 0.0;
        if (emabs && real) {
            const double dk = alz * dka[(size_t)i * N + kk], de = alz * det[(size_t)i * N + kk];
            diag += c * dy * (dk + de);
            ycol = c * (dk * psi_c - de * (1.0 - psi_c));
            yrow = -sgn * c * z * Wk * (sig_c + dy * (dk + de));
            ysum = sgn * Wk * (de * (1.0 - psi_c) - dk * psi_c);
        }
        ysum = wave_sum(ysum);
        double amp = 0.0;
        const bool pair = EXT && A.y.pair_amp != nullptr;
        if (nes) {
            amp = az[i];
            if (lane < NT) L.dd[lane] = ws[(size_t)i * SZ + lane];
        }
        if (nes || pair) {
            if (lane < NC) L.bc[lane] = real ? psi_c : 0.0;
        }
        if (pair) {
            // flux factors, limb cosines (eq. d22) and exp(-eps/T) of the zone for the pair terms
            const double Rz = 0.5 * (re[i] + re[i + 1]);
            if (lane < NC) {
                L.pe[lane] = real ? A.y.pair_eta1[cell0 + (size_t)i * N + kk] : 0.0;
                L.pm[lane] = real ? pair_limb_cosine(A.f.r_nu[(size_t)q * N + kk] / Rz) : 0.0;
            }
            if (lane < NT) L.bz[lane] = lane < N ? exp(-A.cs->eps[lane] / tz[i]) : 0.0;
        }
        wave_sync();

        // ---- (1) row of Ahat_i in LDS
        double nrow[NT];                               // NES entries of the lane's own species block
#pragma unroll
        for (int kp = 0; kp < NT; ++kp) nrow[kp] = 0.0;
        if (nes && real) {
            // -c dt [(1 - psi_k) K^in_{kk'} + psi_k K^out_{kk'}]; the diagonal sums go to diag
            const double ca = -c * amp;
            const double cap = ca * psi_c, cam = ca * (1.0 - psi_c);
            const double* pq = L.bc + (q0 ? 0 : NT);
            double er = 1.0, so = 0.0, si = 0.0;
#pragma unroll
            for (int kp = 0; kp < NT; ++kp) {
                if (kp > 0) er = (kp > kz) ? er * L.dd[kp - 1] : 1.0;
                const double po = Prow[kp] * er;
                so = fma(po, 1.0 - pq[kp], so);
                nrow[kp] = cap * po;
            }
            double el = 1.0;
#pragma unroll
            for (int kp = NT - 1; kp >= 0; --kp) {
                el = (kp < kz) ? el * L.dd[kp] : 1.0;
                const double pi = Prow[kp] * el;
                si = fma(pi, pq[kp], si);
                nrow[kp] = fma(cam, pi, nrow[kp]);
            }
            diag += c * amp * (si + so);
        }
        double ycar = 0.0;
        if (is_row) {
            ycar = frow[MT];
            if (i > 0) {                               // C_{i-1}, y_{i-1} to the workspace
                store_slot<NC, MT>(ws + (size_t)(i - 1) * SZ, lane, frow, ycar);
            }
        }
        if (real) {
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                double v = -bm * frow[m];
                if (m < NT) v += q0 ? nrow[m] : 0.0;
                else if (m < NC) v += q0 ? 0.0 : nrow[m - NT];
                if (m == NC) v += ycol;
                frow[m] = v;
            }
            frow[lz] += diag;                          // once, at the lane's own column (not a select per column)
        } else if (lane < NC) {
#pragma unroll
            for (int m = 0; m < MT; ++m) frow[m] = (m == lz) ? 1.0 : 0.0;     // padded identity row
        }
        if (pair && real) {
            // pair processes (eqs. d11-d14): -c dt dS/dpsi, the partner species' block
            // c [(1 - psi_k) Q^p_kk' + psi_k Q^a_kk' chi_kk'] and the diagonal c sum_k' [Q^p (1 - pbar) + Q^a chi pbar]
            const double a = A.y.pair_amp[zb + i], iw = 1.0 / A.cs->wbar;
            const double bzk = L.bz[kk], eo = L.pe[lane], mo = L.pm[lane];
            const int o = q0 ? NT : 0;
            double cre = 0.0, ann = 0.0;
            for (int kp = 0; kp < N; ++kp) {
                const double qa = a * A.y.pair_g[(size_t)kk * N + kp] * A.cs->W[kp] * iw;
                const double qp = qa * bzk * L.bz[kp];
                const double qx = qa * pair_chi(eo, L.pe[o + kp], mo, L.pm[o + kp]);
                const double pb = L.bc[o + kp];
                cre = fma(qp, 1.0 - pb, cre);
                ann = fma(qx, pb, ann);
                frow[o + kp] += c * ((1.0 - psi_c) * qp + psi_c * qx);
            }
            frow[lz] += c * (cre + ann);
        }
        wave_sync();
        // the Y_e row: one entry from every species lane, the diagonal from the sum over them
        if (lane < NC) L.fix[NC][lane] = yrow;
        if (isY) L.fix[NC][NC] = emabs ? 1.0 + c * z * ysum : 1.0;
        wave_sync();

        double g = 0.0;
        if (real) g = fma(-bm, ycar, A.rhs_sign * rhs[(size_t)i * N + kk]);
        else if (isY) g = A.rhs_sign * A.GY[zb + i];
        const double bcoef = bp;
        if constexpr (TILE) {
            if (is_row) {
                frow[MT] = g;                          // y_{i-1} was consumed above
                L.bpv[kr] = bcoef;
            }
            wave_sync();
            tile_eliminate<MT>(L, lane, A.growth_limit, zp);
        } else {
        // ---- (2) elimination in registers
        double a[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) a[m] = is_row ? frow[m] : 0.0;

        // in-place Gauss-Jordan on [Ahat | diag(bp) | g], partial pivoting over the wavefront
        // (the step loop must be fully unrolled: a[cc] with a run-time cc would put the row in scratch)
        int used = is_row ? 0 : 1;
        double mypiv = 1.0;
        int mycol = 0;
#pragma unroll
        for (int cc = 0; cc < MT; ++cc) {
            const double ac = a[cc];
            const uint32_t key = used ? 0u : ((abs_key_bits(ac) & ~63u) | (uint32_t)(63 - lz));
            uint32_t km = group_max<32>(key);
            km = max((uint32_t)__builtin_amdgcn_readlane((int)km, 0), (uint32_t)__builtin_amdgcn_readlane((int)km, 32));
            const int p = 63 - (int)(km & 63u);
            const bool isp = lz == p;
            if (isp) L.plane[cc] = lane;
            // the pivot row reaches every lane through scalar registers: each value is read from the pivot
            // lane and used at once as the scalar operand of the row updates
            const double piv = lane_value(ac, p);
            const double pinv = drcp(piv);
            const double fm = isp ? 0.0 : ac * pinv;
#pragma unroll
            for (int j = 0; j < MT; ++j)
                if (j != cc) a[j] = fma(-fm, lane_value(a[j], p), a[j]);
            g = fma(-fm, lane_value(g, p), g);
            const double bpiv = lane_value(bcoef, p);
            a[cc] = isp ? bpiv : -fm * bpiv;
            // kept current in every step: left alone, the compiler defers these selects to the end of the
            // zone and holds every step's pivot and lane mask until then
            used |= isp ? 1 : 0;
            mypiv = isp ? piv : mypiv;
            mycol = isp ? cc : mycol;
            asm volatile("" : "+v"(used), "+v"(mypiv), "+v"(mycol));
        }
        wave_sync();                                   // plane[] is read by other lanes below
        // every pivot is some row's own pivot: a zero one is seen here, once per zone
        zp |= is_row && !(mypiv != 0.0);

        // ---- (3) restore row ownership: the lane holding unknown mycol writes its scaled row, slot cc (which
        //      holds the column of C of the step's pivot lane plane[cc]) going to that column, so rows and
        //      columns come back in natural order
        if (is_row) {
            const double ip = drcp(mypiv);
            double* dst = L.fix[mycol];
#pragma unroll
            for (int cc = 0; cc < MT; ++cc) dst[L.plane[cc]] = a[cc] * ip;
            dst[MT] = g * ip;
        }
        wave_sync();
        }

        psi_c = psi_n1;
        sig_c = sig_n1;
        lam_c = lam_n1;
        dHu_lo = dHu_hi;
        dHv_lo = dHv_hi;
    }
    if constexpr (TILE) {
        // growth guard: a ray with a multiplier above the limit or a zero pivot is left untouched and
        // marked for the partial-pivoting re-run
        const bool bad = __ballot(zp) != 0ull;
        if (lane == 0 && A.redo) A.redo[ray] = bad ? 1 : 0;
        if (bad) return;
    }
    if (is_row) {                                      // C_{I-1}, y_{I-1}
        store_slot<NC, MT>(ws + (size_t)(I - 1) * SZ, lane, frow, frow[MT]);
    }

    // ---------------------------------------------------------------- backward sweep
    // the row index recomputed here rather than kept live through the forward sweep
    int lb;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lb));
    const int kb = lb < MT ? lb : 0;
    // the cell offset of the lane's row likewise
    const int qb = lb < NT ? 0 : 1, kgb = lb - qb * NT;
    const bool realb = lb < NC && kgb < N;
    const size_t cellb = ((size_t)(realb ? qb : 0) * R + ray) * I * N + (realb ? kgb : 0);
    double cr[NC], crn[NC];
    double yv = 0.0, yn = 0.0;
    load_slot<NC, MT>(ws + (size_t)(I - 1) * SZ, kb, is_row, cr, yv);
    double dnext = 0.0;
    for (int i = I - 1; i >= 0; --i) {
        if (i > 0) load_slot<NC, MT>(ws + (size_t)(i - 1) * SZ, kb, is_row, crn, yn);
        double dl = yv;
        if (i + 1 < I) {
            if (lane < NC) L.bc[lane] = dnext;
            wave_sync();
#pragma unroll
            for (int m = 0; m < NC; ++m) dl = fma(-cr[m], L.bc[m], dl);
            wave_sync();
        }
        if (realb) {
            const size_t ci = cellb + (size_t)i * N;
            A.psi_out[ci] += dl;
            A.dx[ci] = dl;
        } else if (lb == NC) {
            A.ye_out[zb + i] += dl;
            A.dY[zb + i] = dl;
        }
        dnext = dl;
#pragma unroll
        for (int m = 0; m < NC; ++m) cr[m] = crn[m];
        yv = yn;
    }
    const bool any_zp = __ballot(zp) != 0ull;
    if (lane == 0) {
        if (any_zp && A.flags) A.flags[ray] |= 4;
        A.iters[ray] += 1;
        A.pending[ray] = 1;                    // trial psi + delta awaits the line search
        A.alpha[ray] = 1.0;
    }
}

size_t ye_ws_bytes_per_ray(int I, int N) {
    const int NT = padded_groups(N);
    if (NT < 0 || N > kYeMaxGroups) return 0;
    const size_t n = (size_t)(2 * NT + 1) * (2 * NT + 1);   // per zone: C [2 NT][MT] and y [MT] ...
    return (size_t)I * (n + (n & 1)) * sizeof(double);     // ... rounded up to an even count (16-byte slots)
}

// ---------------------------------------------------------------- line-search move-back

__global__ __launch_bounds__(kBlock) void k_ye_backtrack(Shape sh, double* __restrict__ psi, double* __restrict__ ye,
                                                         const double* __restrict__ dx, const double* __restrict__ dY,
                                                         int* backtrack, double* alpha) {
    const long long ray = blockIdx.x;
    if (backtrack[ray] == 0) return;
    const double a = alpha[ray];
    const double coef = 0.5 * a - a;
    const size_t n = (size_t)sh.I * sh.N;
    for (int q = 0; q < 2; ++q) {
        const size_t base = ((size_t)q * sh.R + ray) * n;
        for (size_t j = threadIdx.x; j < n; j += kBlock) psi[base + j] = psi[base + j] + __dmul_rn(coef, dx[base + j]);
    }
    const size_t zb = (size_t)ray * sh.I;
    for (int i = threadIdx.x; i < sh.I; i += kBlock) ye[zb + i] = ye[zb + i] + __dmul_rn(coef, dY[zb + i]);
    __syncthreads();
    if (threadIdx.x == 0) {
        alpha[ray] = 0.5 * a;
        backtrack[ray] = 0;
    }
}

// ---------------------------------------------------------------- matter energy and temperature

struct SpeciesWeights {
    double w[16];
};

// de_i = -(4 pi/(hc)^3) (m_B/rho_i) sum_q w_q c dt sum_k eps_k W_k S_qk   (eq. a62b, MeV per baryon)
// T_i^{n+1} = T_i^n + (de_i - (Y_e^{n+1} - Y_e^n) de/dY_e) / (de/dT)      (eq. a62d)
// S_qk is the collision source of species q at psi^{n+1}: emission/absorption (for species 0 and 1 with
// the opacities at Y_e^{n+1}) and NES; isoenergetic scattering exchanges no energy.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_ye_temperature(Shape sh, Fields f, YeFields y, const Consts* __restrict__ cs,
                                                           const double* __restrict__ psi, const double* __restrict__ ye,
                                                           SpeciesWeights wts, const double* __restrict__ de_dT,
                                                           const double* __restrict__ de_dye, double* __restrict__ de_out,
                                                           double* __restrict__ temp_out) {
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nz = (long long)sh.R * sh.I;
    if (idx >= nz) return;
    const int R = sh.R, I = sh.I, N = sh.N;
    const long long ray = idx / I;
    const int i = (int)(idx - ray * I);
    const bool emabs = sh.terms & kEmAbs, nes = sh.terms & kNes;
    const double T = f.temp[idx];
    const double dy = ye[idx] - y.ye_n[idx];
    double d[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) d[j] = (nes && j + 1 < N) ? exp(-cs->de[j] / T) : 0.0;
    double src = 0.0;
    for (int s = 0; s < sh.S; ++s) {
        const size_t cz = (((size_t)s * R + ray) * I + i) * N;
        double p[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) p[k] = k < N ? psi[cz + k] : 0.0;
        const double amp = nes ? f.nes_amp[((size_t)s * R + ray) * I + i] : 0.0;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            if (k >= N) break;
            double sk = 0.0;
            if (emabs) {
                double kap = f.kappa_a[cz + k], eta = f.eta[cz + k];
                if (s < 2) {
                    kap += dy * y.dka[cz + k];
                    eta += dy * y.deta[cz + k];
                }
                sk = eta * (1.0 - p[k]) - kap * p[k];
            }
            if (nes) {
                double sin_ = 0.0, sout = 0.0, e = 1.0;
#pragma unroll
                for (int kp = k + 1; kp < NT; ++kp) {          // k' > k: out factor exp(-(eps_k' - eps_k)/T)
                    if (kp >= N) break;
                    e *= d[kp - 1];
                    sout = fma(cs->P[k][kp] * e, 1.0 - p[kp], sout);
                    sin_ = fma(cs->P[k][kp], p[kp], sin_);
                }
                e = 1.0;
#pragma unroll
                for (int kp = k - 1; kp >= 0; --kp) {          // k' < k: in factor exp(-(eps_k - eps_k')/T)
                    e *= d[kp];
                    sin_ = fma(cs->P[k][kp] * e, p[kp], sin_);
                    sout = fma(cs->P[k][kp], 1.0 - p[kp], sout);
                }
                sk += amp * ((1.0 - p[k]) * sin_ - p[k] * sout);
            }
            acc = fma(cs->eps[k] * cs->W[k], sk, acc);
        }
        src = fma(wts.w[s], sh.c_dt * acc, src);
    }
    if (y.pair_amp) {
        // pair sources of species 0 and 1 (eqs. d11-d14) with their energy weights
        const double* re = f.r_edge + (size_t)ray * (I + 1);
        const double Rz = 0.5 * (re[i] + re[i + 1]);
        const double a = y.pair_amp[idx], iw = 1.0 / cs->wbar;
        double bz[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) bz[j] = j < N ? exp(-cs->eps[j] / T) : 0.0;
        for (int qs = 0; qs < 2; ++qs) {
            const size_t co = (((size_t)qs * R + ray) * I + i) * N, cb = (((size_t)(1 - qs) * R + ray) * I + i) * N;
            double acc = 0.0;
            for (int k = 0; k < N; ++k) {
                const double p = psi[co + k], eo = y.pair_eta1[co + k];
                const double mo = pair_limb_cosine(f.r_nu[(size_t)qs * N + k] / Rz);
                const double bk = exp(-cs->eps[k] / T);
                double cre = 0.0, ann = 0.0;
#pragma unroll
                for (int kp = 0; kp < NT; ++kp) {
                    if (kp >= N) break;
                    const double qa = a * y.pair_g[(size_t)k * N + kp] * cs->W[kp] * iw;
                    const double pb = psi[cb + kp];
                    const double mb = pair_limb_cosine(f.r_nu[(size_t)(1 - qs) * N + kp] / Rz);
                    cre = fma(qa * bk * bz[kp], 1.0 - pb, cre);
                    ann = fma(qa * pair_chi(eo, y.pair_eta1[cb + kp], mo, mb), pb, ann);
                }
                acc = fma(cs->eps[k] * cs->W[k], (1.0 - p) * cre - p * ann, acc);
            }
            src = fma(wts.w[qs], sh.c_dt * acc, src);
        }
    }
    const double de = -kFourPiOverHc3 * kBaryonMassG / y.rho[idx] * src;
    if (de_out) de_out[idx] = de;
    temp_out[idx] = T + (de - dy * de_dye[idx]) / de_dT[idx];
}

// ---------------------------------------------------------------- launchers

#define TM_YE_DISPATCH(NTV, ...)                                        \
    switch (NTV) {                                                      \
        case 4: { constexpr int NT = 4; __VA_ARGS__; } break;           \
        case 8: { constexpr int NT = 8; __VA_ARGS__; } break;           \
        case 12: { constexpr int NT = 12; __VA_ARGS__; } break;         \
        case 16: { constexpr int NT = 16; __VA_ARGS__; } break;         \
        case 20: { constexpr int NT = 20; __VA_ARGS__; } break;         \
        case 24: { constexpr int NT = 24; __VA_ARGS__; } break;         \
        case 28: { constexpr int NT = 28; __VA_ARGS__; } break;         \
        default: return hipErrorInvalidValue;                           \
    }

hipError_t launch_ye_couple(const Shape& sh, const Fields& f, const YeFields& y, const Consts* cs, const double* psi,
                            const double* ye, double* G, double* GY, const double* level_sp, const YeOut& out,
                            hipStream_t st) {
    if (y.pair_amp)
        TM_YE_DISPATCH(padded_groups(sh.N),
                       hipLaunchKernelGGL((k_ye_couple<NT, true>), dim3((unsigned)sh.R), dim3(kBlock), 0, st, sh, f, y, cs,
                                          psi, ye, G, GY, level_sp, out))
    else
        TM_YE_DISPATCH(padded_groups(sh.N),
                       hipLaunchKernelGGL((k_ye_couple<NT, false>), dim3((unsigned)sh.R), dim3(kBlock), 0, st, sh, f, y,
                                          cs, psi, ye, G, GY, level_sp, out))
    return hipGetLastError();
}

hipError_t launch_ye_factor(const YeFactorArgs& a, hipStream_t st) {
    TM_YE_DISPATCH(padded_groups(a.sh.N),
                   constexpr int WPB = ye_waves_per_block<NT>();
                   const long long blocks = (a.nray + WPB - 1) / WPB;
                   if (!ye_tiled_applies(a))
                       hipLaunchKernelGGL((k_ye_factor<NT, 1, true, false>), dim3((unsigned)blocks), dim3(64 * WPB), 0,
                                          st, a);
                   else
                       hipLaunchKernelGGL((k_ye_factor<NT, ye_waves_per_eu<NT>(), false, false>), dim3((unsigned)blocks),
                                          dim3(64 * WPB), 0, st, a))
    return hipGetLastError();
}

bool ye_tiled_applies(const YeFactorArgs& a) {
    return !(a.sh.limiter == 2 || a.sh.outer_bc == 2 || a.y.pair_amp || a.f.lapse);
}

hipError_t launch_ye_factor_tiled(const YeFactorArgs& a, hipStream_t st) {
    if (!ye_tiled_applies(a) || !a.redo) return hipErrorInvalidValue;
    TM_YE_DISPATCH(padded_groups(a.sh.N),
                   constexpr int WPB = ye_waves_per_block<NT>();
                   const long long blocks = (a.nray + WPB - 1) / WPB;
                   hipLaunchKernelGGL((k_ye_factor<NT, ye_waves_per_eu<NT>(), false, true>), dim3((unsigned)blocks),
                                      dim3(64 * WPB), 0, st, a))
    return hipGetLastError();
}

hipError_t launch_ye_backtrack(const Shape& sh, double* psi, double* ye, const double* dx, const double* dY,
                               int* backtrack, double* alpha, hipStream_t st) {
    hipLaunchKernelGGL(k_ye_backtrack, dim3((unsigned)sh.R), dim3(kBlock), 0, st, sh, psi, ye, dx, dY, backtrack, alpha);
    return hipGetLastError();
}

hipError_t launch_ye_temperature(const Shape& sh, const Fields& f, const YeFields& y, const Consts* cs,
                                 const double* psi, const double* ye, const double* weights, const double* de_dT,
                                 const double* de_dye, double* de_out, double* temp_out, hipStream_t st) {
    if (sh.S > 16) return hipErrorInvalidValue;
    SpeciesWeights w{};
    for (int s = 0; s < sh.S; ++s) w.w[s] = weights[s];
    const long long nz = (long long)sh.R * sh.I;
    const unsigned blocks = (unsigned)((nz + kBlock - 1) / kBlock);
    TM_YE_DISPATCH(padded_groups(sh.N),
                   hipLaunchKernelGGL(k_ye_temperature<NT>, dim3(blocks), dim3(kBlock), 0, st, sh, f, y, cs, psi, ye, w,
                                      de_dT, de_dye, de_out, temp_out))
    return hipGetLastError();
}

}  // namespace tmk
