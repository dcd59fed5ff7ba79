// Kernel launch interfaces of libtm (internal; the public C ABI is include/tm.h).
#pragma once

#include "tm_device.hpp"

namespace tmk {

// Newton line-search constants (sufficient decrease, shortest step) shared with the host.
constexpr double kArmijo = 1e-4;
constexpr double kAlphaMin = 1.0 / 256.0;

// Residual pass modes.
enum ResidualMode : int {
    kResPlain = 0,      // max|G| only (tm_assemble)
    kResInitial = 1,    // first Newton pass: res0, accepted residual, target, activity
    kResTrial = 2,      // pending trials only: accept (stopping rule, activity) or ask to backtrack
    kResEval = 3,       // G, max|G| and the rounding level only; with `pending` set, only systems whose
                        // ray (sys % R) has a pending trial (the species part of the Y_e-coupled step)
};

// Inputs/outputs of the residual / statistics kernel, all per system of the launch.
struct ResidualOut {
    int mode;
    double* res;        // max |G| of the evaluated state (required)
    double* res0;       // max |G| at the initial guess
    double* res_acc;    // max |G| of the accepted iterate
    double* tgt;        // stopping target max(rtol res0, rounding level) at the accepted iterate
    double* alpha;      // step length of the pending trial
    int* pending;       // 1 while a trial is under evaluation
    int* backtrack;     // set to 1 when the trial is rejected
    int* active;        // Newton activity flag
    const int* iters;   // updates applied so far
    double* n_tot;      // conservation statistics of the evaluated state (nullable)
    double* e_tot;
    double* budget;
    double* lum;
    double* level;      // rounding level of G of the evaluated state (nullable)
    int stats;
    int max_iter;
    double rtol;
};

struct FactorArgs {
    Shape sh;
    Fields f;
    const Consts* cs;
    const double* psi;        // state at which J is evaluated [S][R][I][N]
    const double* rhs;        // right-hand side, cell array, multiplied by rhs_sign
    double rhs_sign;
    const double* rhs_max;    // per system (global index): max |rhs|, for the float32 power-of-two
                              // scaling of the right-hand side (nullable = no scaling)
    double* x;                // solution output (nullable when psi_out is set)
    double* psi_out;          // Newton: psi_out += delta (nullable)
    const int* active;        // per system (global index), nullable = all active
    int* flags;               // per system, zero-pivot bit (nullable)
    int* iters;               // per system, incremented on update (nullable)
    int* guard;               // per system, set to 1 when the growth guard trips (nullable)
    double* dx;               // Newton: the update delta is also written here (nullable)
    int* pending;             // Newton: set to 1 for updated systems (trial to evaluate)
    double* alpha;            // Newton: set to 1 for updated systems
    double growth_limit;      // largest |multiplier| accepted with diagonal pivots
    void* wsC;                // [batch][I][NT][NT] factors (element type of the kernel)
    void* wsY;                // [batch][I][NT]
    long long sys0;           // first system of the batch
    long long nsys;           // systems in the batch
    int skip_if_window = 0;   // quad kernel, exp2 NES form: do nothing when the energy grid admits the
                              // windowed form (launched beside the windowed kernel)
};

hipError_t launch_setup(const double* e_edge, const double* nes_g, int N, Consts* out, hipStream_t st);

hipError_t launch_residual(const Shape& sh, const Fields& f, const Consts* cs, const double* psi_n,
                           const double* psi, double* G_out, double g_sign, const ResidualOut& out,
                           hipStream_t st);

hipError_t launch_blocks(const Shape& sh, const Fields& f, const Consts* cs, const double* psi,
                         double* blocks, hipStream_t st);

// The float32 forward solve with diagonal pivots (N <= 20) runs on one system per quad of lanes.  Its
// elimination updates run on the vector units, or on the matrix cores (kFactorQuadMfma); its NES block
// takes one exp2 per entry (kFactorQuadValu, kFactorQuadMfma) or the energy-window scalings, with the
// diagonal sums on the vector units (kFactorQuadWindow) or as bf16 matrix-core contractions with float32
// accumulation in three bf16 products per term (kFactorQuadBf16x3) or one (kFactorQuadBf16).
// kFactorLane keeps one row per lane.
enum FactorKernel : int {
    kFactorLane = 0,
    kFactorQuadValu = 1,
    kFactorQuadMfma = 2,
    kFactorQuadWindow = 3,
    kFactorQuadBf16x3 = 4,
    kFactorQuadBf16 = 5
};
hipError_t launch_factor(const FactorArgs& a, bool fp32, bool transpose, bool pivot, hipStream_t st,
                         int kernel = kFactorQuadMfma);
bool launch_factor_quad(const FactorArgs& a, hipStream_t st, int kernel);
hipError_t launch_factor_geo(const FactorArgs& a, bool fp32, bool transpose, bool pivot, hipStream_t st);

hipError_t launch_vjp(const Shape& sh, const Fields& f, const Consts* cs, const double* psi,
                      const double* mu, double* g_ka, double* g_eta, double* g_ks, double* g_amp,
                      hipStream_t st);

hipError_t launch_lum_seed(const Shape& sh, const double* r_edge, const double* lapse_edge, const Consts* cs,
                           const double* add, double* seed, hipStream_t st);

hipError_t launch_final_flags(long long n, const double* res, const double* tgt, double rtol, int* flags,
                              hipStream_t st);
hipError_t launch_sys_absmax(const double* v, long long nsys, long long per_sys, double* out, hipStream_t st);
hipError_t launch_count_active(const int* active, long long n, int* count, hipStream_t st);

// psi += (alpha/2 - alpha) dx and alpha /= 2 for systems with backtrack set (which is cleared)
hipError_t launch_backtrack(const Shape& sh, double* psi, const double* dx, int* backtrack, double* alpha,
                            hipStream_t st);

// p[0..n) = v (a kernel, so that a captured graph holds no memset node)
hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st);

// *count = number of entries j with (flags[j] & mask) != 0
hipError_t launch_count_bits(const int* flags, long long n, int mask, int* count, hipStream_t st);

// active_out[j] = 1 where guard[j] != 0 (else 0); *count = number of such systems
hipError_t launch_mark(const int* guard, long long n, int* active_out, int* count, hipStream_t st);

// ---------------------------------------------------------------- Y_e-coupled step (eqs. a62a-a62ae)

// Extra inputs of the coupled step, all device memory: zone arrays [R][I], and the Y_e derivatives of
// the absorption and emission opacities of species 0 (nu_e) and 1 (anti-nu_e), [2][R][I][N].
struct YeFields {
    const double* rho;
    const double* ye_n;
    const double* dka;
    const double* deta;
    const double* pair_amp;    // [R][I] pair-kernel amplitude, or nullptr (no pair processes)
    const double* pair_g;      // [N][N] symmetric pair-kernel shape
    const double* pair_eta1;   // [2][R][I][N] flux factors psi1/psi0 of species 0 and 1
};

// Per-ray state of the coupled Newton iteration (the same quantities as ResidualOut, per ray).
struct YeOut {
    int mode;           // kResInitial or kResTrial
    double* res;        // max |G| over both species and Y_e
    double* res0;
    double* res_acc;
    double* tgt;
    double* alpha;
    int* pending;
    int* backtrack;
    int* active;
    const int* iters;
    double* lepton;     // total lepton number / (4 pi) of the evaluated state (nullable)
    int max_iter;
    double rtol;
};

struct YeFactorArgs {
    Shape sh;                 // the problem (S >= 2; species 0 and 1 are the coupled pair)
    Fields f;
    YeFields y;
    const Consts* cs;
    const double* psi;        // iterate, cell array [S][R][I][N] (species 0, 1 read)
    const double* ye;         // iterate [R][I]
    const double* G;          // species residual [2][R][I][N] (right-hand side times rhs_sign)
    const double* GY;         // Y_e residual [R][I]
    double rhs_sign;
    double* psi_out;          // psi += delta (species 0, 1)
    double* ye_out;           // ye += delta_Y
    double* dx;               // delta of the species cells [2][R][I][N]
    double* dY;               // delta of Y_e [R][I]
    const int* active;        // per ray, nullable = all
    int* flags;               // per ray: zero-pivot bit
    int* iters;               // per ray
    int* pending;             // per ray
    double* alpha;            // per ray
    double* ws;               // per ray slot: I * (2 NT + 1) * (2 NT + 1) doubles
    long long ray0;           // first ray of the batch
    long long nray;           // rays in the batch
    // Diagonal pivots on 8 x 8 lane tiles (launch_ye_factor_tiled): a ray whose multipliers exceed
    // growth_limit, or that meets a zero or non-finite pivot, is left untouched and marked in redo;
    // the partial-pivoting launch (launch_ye_factor) with redo set then takes only the marked rays.
    int* redo = nullptr;      // per ray (nullable for the partial-pivoting launch: all active rays)
    double growth_limit = 16.0;
};

// Species residual G (from the single-species residual pass, opacities at Y_e^n) completed in place
// with the Y_e terms, the Y_e residual GY, max|G| and the rounding level per ray, and the Newton
// bookkeeping of `out`; level_sp holds the rounding levels of the 2R species systems.
hipError_t launch_ye_couple(const Shape& sh, const Fields& f, const YeFields& y, const Consts* cs, const double* psi,
                            const double* ye, double* G, double* GY, const double* level_sp, const YeOut& out,
                            hipStream_t st);
hipError_t launch_ye_factor(const YeFactorArgs& a, hipStream_t st);
// false when the problem needs the partial-pivoting kernel only (neutrinosphere options, pairs or a lapse)
bool ye_tiled_applies(const YeFactorArgs& a);
hipError_t launch_ye_factor_tiled(const YeFactorArgs& a, hipStream_t st);
// psi (species 0, 1) and ye += (alpha/2 - alpha) delta, alpha /= 2, for rays with backtrack set (cleared)
hipError_t launch_ye_backtrack(const Shape& sh, double* psi, double* ye, const double* dx, const double* dY,
                               int* backtrack, double* alpha, hipStream_t st);
// Matter energy change (eq. a62b) and temperature (eq. a62d) per zone after the step.
hipError_t launch_ye_temperature(const Shape& sh, const Fields& f, const YeFields& y, const Consts* cs,
                                 const double* psi, const double* ye, const double* weights, const double* de_dT,
                                 const double* de_dye, double* de_out, double* temp_out, hipStream_t st);
size_t ye_ws_bytes_per_ray(int I, int N);
constexpr int kYeMaxGroups = 28;          // 2 NT + 1 rows of a coupled block fit one wavefront

// Lapse folded into the inputs (source factor a, NES at local energies); writes the folded copies.
hipError_t launch_lapse_fold(const Shape& sh, const double* lapse, const double* ka, const double* et,
                             const double* ks, const double* temp, const double* amp, double* oka, double* oet,
                             double* oks, double* otemp, double* oamp, hipStream_t st);

// Energy advection (eqs. a78-a81d) and lapse remap (eqs. p1-p8), one thread per (species, ray, zone).
constexpr int kEaLagrangian = 0, kEaLapse = 1;                            // TM_EADV_* modes
constexpr int kEaDisplacement = 1, kEaOverfill = 2, kEaOverfillClamp = 4;  // TM_EADV_FLAG_* bits
struct EaArgs {
    int mode;
    int N;
    long long nz;             // zone-systems S * R * I
    long long RI;             // zones per species, R * I
    const double* e_edge;     // [N+1] target grid
    const double* rho_old;    // zone [R][I], nullable
    const double* rho_new;
    const double* a_old;      // lapse, zone, nullable (required in the lapse mode)
    const double* a_new;
    const double* dlnR;       // zone, nullable
    const double* dlnb;
    const double* edd;        // cell, nullable (1/3)
    double* psi;              // cell, in place
    double* xi;               // sysz, nullable
    int* flags;               // sysz, nullable
};
hipError_t launch_energy_advect(const EaArgs& a, hipStream_t st);

// Factor workspace: C and y per system slot; a batch of b systems takes b + kWsPadSystems slots (the
// layout is interleaved by wave group of at most 16 systems, and a last partial group keeps empty slots).
constexpr int kWsPadSystems = 15;
size_t factor_ws_bytes_per_system(int I, int N, bool fp32);
int padded_groups(int N);

}  // namespace tmk
