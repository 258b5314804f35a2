// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rh.h"

namespace rh {

// Physical constants, CGS (this library's own copy).
constexpr double kC = 2.99792458e10;       // speed of light, cm/s
constexpr double kKB = 1.380649e-16;       // Boltzmann, erg/K
constexpr double kMH = 1.6735575e-24;      // hydrogen atom mass, g
constexpr double kEV = 1.602176634e-12;    // erg per eV
constexpr double kSigmaT = 6.6524587321e-25;
constexpr double kARad = 7.565723e-15;
constexpr double kME = 9.1093837015e-28;
constexpr double kTcmb0 = 2.725;
constexpr double kMpc = 3.0856775814913673e24;
constexpr double kH100 = 1.0e7 / kMpc;     // 100 km/s/Mpc in 1/s

constexpr int kBlock = 256;                // threads per block of the 1-D kernels
constexpr int kRedBlocks = 1024;           // grid of the one-cell-per-thread reducing kernels
// Block partial sums: part[slot * kPartCap + block]; each reducing kernel
// also stores its block count at part[RS_COUNT * kPartCap + slot], which the
// finalize pass reads, so kernels with different grids can share the buffer
// (the last writer of a slot before a finalize defines it).
constexpr int kPartCap = 16384;
constexpr int kMaxLevels = 16;
constexpr int kCoarseMaxCells = 512;

// Per-step scalars seen by the kernels (passed by value).
struct StepK {
  int nx, ny, nz;
  long long N;
  int bc[6];
  int iso, rates, cooling, theta_lt1;
  double h, dt, theta;
  double a_n, a_1, H_n, H_1;
  double sigma_E, K_Gamma, K_G, hnu0;
  double T_iso, alphaB, gamma, compton;
  double E_floor, R_min;
  double cf_scale;      // dt theta / (a_1^2 h^2): face D -> dimensionless coefficient
  double expl_ratio;    // (1-theta)/theta (a_1/a_n)^2: implicit -> explicit coefficient
  double E_s;           // norm scale of E
  // multigroup: the group's cross-sections of HeI and HeII (sigma_E above is
  // the hydrogen one; the opacity adds sig_he[0] n_HeI + sig_he[1] n_HeII
  // where the helium fields are given) and its share of the source
  double sig_he[2];
  double src_frac;
};

// bfloat16 <-> float: a bfloat16 is the upper half of an FP32 bit pattern
// (rounded to nearest even; the values stored here are finite).
__host__ __device__ inline float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, sizeof f);
  return f;
}
__host__ __device__ inline uint16_t bf16_round(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, sizeof u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Operator of an FP32 multigrid level, one 8-byte record per cell (a
// single load): the cell's + face coefficients along x, y, z and its shift
// (the diagonal minus the six face coefficients of the cell), in bfloat16.
// The diagonal is formed where it is used, as op_diag below, so the level's
// operator is a symmetric M-matrix whose energy is within 1 +- 2^-8 of the
// exact operator's (faces and shift are non-negative and each enters the
// energy with a non-negative weight).  FP64 levels keep the diagonal and the
// faces as separate double arrays.
struct __align__(8) Op16 {
  uint16_t f[3];  // + faces along x, y, z (0 on a non-periodic last face)
  uint16_t s;     // shift
};
// The diagonal of an FP32 level from a cell's shift and its six faces, in
// this order everywhere (absent faces enter as 0).
__host__ __device__ inline float op_diag(float s, float xp, float xm, float yp, float ym, float zp,
                                         float zm) {
  return (((((s + xp) + xm) + yp) + ym) + zp) + zm;
}

template <class T>
struct LevelOp;
template <>
struct LevelOp<double> {
  double* diag;   // diagonal of the Schur operator
  double* cf[3];  // + face coefficients (dimensionless, 0 on a non-periodic last face)
};
template <>
struct LevelOp<float> {
  Op16* op;       // packed operator records
};

// One multigrid level (T = float or double).
template <class T>
struct LevelK : LevelOp<T> {
  int nx, ny, nz;
  long long N;
  int per[3];           // periodic per dimension
  T* x;                 // correction
  T* x2;                // second correction buffer (output of a fused sweep)
  T* b;                 // right-hand side
  T* r;                 // residual scratch
};

// Source-centred boxes of one multigrid level for the block smoother
// (rh_blocks.hip): n boxes of extent ex x ey x ez (m = ex ey ez cells,
// at most kBlockMaxCells), each given by its lowest corner (3 ints, boxes
// never wrap), ordered by colour; inv holds each box's inverse (m x m,
// symmetric, so row and column order coincide).
constexpr int kBlockMaxCells = 125;  // boxes of radius <= 2
constexpr int kMaxBlockLevels = 4;
template <class T>
struct BlockSet {
  int n;
  int ex, ey, ez, m;
  const int* start;
  T* inv;
};

// Reduction slots (partials laid out [slot][kRedBlocks]).
enum RedSlot {
  RS_FE2 = 0,      // sum (f_E/E_s)^2
  RS_FN2,          // sum (f_n/n_H)^2
  RS_FE_LOC2,      // sum (f_e/e^n)^2
  RS_RMAX,         // max |r|
  RS_LOCAL_FAIL,   // max over cells: 1 if the local solve failed
  RS_LOCAL_ITS,    // max local iterations
  RS_R2,           // sum r^2 (plain)
  RS_EMAX,         // max E^n
  RS_SMAX,         // max src
  RS_NONFINITE,    // max over cells: 1 if an input / local output is not finite
  RS_BAD_RES,      // max over cells: 1 if f_E or the Schur diagonal is not finite
  RS_PQ,           // sum p.q   (conjugate gradients)
  RS_ZR,           // sum z.r
  RS_ZQ,           // sum z.q
  RS_CHG2,         // sum of squared weighted changes U^{n+1} - U^n (step controller)
  RS_NEGE,         // max over cells of -E/E_s (positivity check)
  RS_COURANT,      // max over cells of the outgoing Courant number (advection)
  RS_MAG2,         // sum of squared weighted term magnitudes (coupled multigroup residual)
  RS_COUNT
};
static_assert(RS_COUNT <= 32, "slot masks are 32-bit");
constexpr unsigned kAllSlots = (1u << RS_COUNT) - 1;
constexpr unsigned slot_bit(int s) { return 1u << s; }


// ---- host helpers (rh_host.cpp) -------------------------------------------
// Parameter validation as rh_setup does it (message into err on failure).
bool params_valid(const rh_params* p, char* err, size_t n);
// The per-step scalars of a step from t_n over dt (grey constants,
// expansion factors, limiter floor, coefficient scales); E_s = 1.
StepK step_scalars(const rh_params& p, double t_n, double dt);
// Message returned by rh_last_error(NULL) on this thread.
void set_last_error(const char* msg);

// ---- launchers (rh_kernels.hip) ------------------------------------------
// Weighted change of a step and its most negative E: partial sums of
// (dE/E_s)^2 + (de/e^n)^2 + (dn/n_H)^2 (RS_CHG2; no e term when e is null)
// and max(-E/E_s) (RS_NEGE).
void launch_change_norm(hipStream_t s, long long N, double E_s, const double* E, const double* e,
                        const double* n, const double* En, const double* en, const double* nn,
                        const double* nH, double* part);
// E = E0, n = keep nH, e = e0 (e may be null); RS_NONFINITE flags a bad nH.
void launch_init_state(hipStream_t s, long long N, double E0, double keep, double e0,
                       const double* nH, double* E, double* e, double* n, double* part);
// out = scale in; RS_NONFINITE flags a negative or non-finite input.
void launch_scale_field(hipStream_t s, long long N, double scale, const double* in, double* out,
                        double* part);
// y1n, y2n: n_HeI^n, n_HeII^n of a multigroup step (both null: hydrogen only).
void launch_step_setup(hipStream_t s, const StepK& k, const double* En, const double* nn,
                       const double* y1n, const double* y2n,
                       const double* src, double* cf64_x, double* cf64_y, double* cf64_z,
                       Op16* op32, double* rhsn,
                       double* part);

// mode 0: solve the local equations at E = E_k + lam dE (dE may be null);
// mode 1: evaluate at the given (E, e, n) without solving.
struct LocalArgs {
  const double* Ek; const double* dE; double lam;
  const double* ek; const double* nk;                 // initial guess / given state
  const double* pBCn; const double* pBCe;              // predictor data of U_k (may be null)
  const double* pBfn; const double* pBfe;
  const double* En; const double* en; const double* nn; const double* nH;
  double* Et; double* et; double* nt;                  // outputs (mode 0)
  double* BCn; double* BCe; double* Bfn; double* Bfe;  // local terms at the result
  double* fn_out; double* fe_out;                      // optional residual outputs
  int mode;
};
void launch_local(hipStream_t s, const StepK& k, const LocalArgs& a, double* part);

struct ResidArgs {
  const double* E; const double* n; const double* En; const double* nn;
  const double* cf[3]; const double* rhsn;
  const double* BCn; const double* Bfn;
  double* rS; double* diag64; double* fE_out;
  Op16* op32;  // FP32 finest level: its shift is written (faces come from the step setup)
  // multigroup (all null for the grey step): helium densities of the state
  // and of U^n, and the group's Schur terms from the local elimination
  // (kB = sum_s J_gs (B^-1 f)_s, Kgg = sum_s J_gs (B^-1 C)_sg), which then
  // replace the grey JEn Bfn and JEn BCn
  const double* y1; const double* y2; const double* y1n; const double* y2n;
  const double* kB; const double* Kgg;
};
void launch_residual(hipStream_t s, const StepK& k, const ResidArgs& a, double* part);

// Sums / maxima of the partials of a reducing launch over N fine cells.
// Reduces the slots whose bits are set in mask (bit s = slot s) into out[s].
void launch_finalize(hipStream_t s, const double* part, double* out, unsigned mask);

template <class T>
void launch_coarsen_faces(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c);
template <class T>
void launch_coarse_diag(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c);
template <class T>
void launch_coarsest_inverse(hipStream_t s, const LevelK<T>& c, double* A, double* Inv,
                             T* InvT);
template <class T>
void launch_coarsest_solve(hipStream_t s, const LevelK<T>& c, const T* InvT);
template <class T>
void launch_rbgs(hipStream_t s, const LevelK<T>& l, int color, int zero_init, int fine);
// One full red-black sweep (first_color, then the other) reading l.x and
// writing l.x2; returns false (nothing launched) unless rbgs_march_fits(l,
// min_tiles), and the caller then sweeps colour by colour in place.
// With dots != NULL (finest level, last sweep of a V-cycle) the launch also
// stores the block partials of z.r (RS_ZR) and z.q (RS_ZQ, q may be NULL)
// for z = sigma * (the sweep's output); it then returns false, launching
// nothing, if the grid has more workgroups than the partial buffer holds.
struct SweepDots {
  double sigma;
  const double* r;
  const double* q;
  double* part;
};
template <class T>
bool launch_rbgs_march(hipStream_t s, const LevelK<T>& l, int first_color, int zero_init,
                       int fine, long long min_tiles, const SweepDots* dots);
// The level has a second buffer, the shape the marching tiles need, fewer
// than 2^31 cells and at least min_tiles tiles (one workgroup each).
template <class T>
bool rbgs_march_fits(const LevelK<T>& l, long long min_tiles);
template <class T>
void launch_mg_residual(hipStream_t s, const LevelK<T>& l);
// r = b - A x on f fused with the restriction of r into c.b (f.r is not
// written); returns false (nothing launched) unless resid_restrict_fits(f,
// min_tiles): even dimensions and enough of its tiles.
template <class T>
bool launch_resid_restrict_march(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c,
                                 long long min_tiles);
template <class T>
bool resid_restrict_fits(const LevelK<T>& f, long long min_tiles);
template <class T>
void launch_restrict(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c);
template <class T>
void launch_prolong(hipStream_t s, const LevelK<T>& c, const LevelK<T>& f);
template <class T>
void launch_cast_scale(hipStream_t s, long long N, const double* r, double inv_sigma, T* b);

struct DefectArgs {
  const double* rS; const double* dE_in; double* dE_out;
  const double* diag64; const double* cf[3];
  int first;           // dE_in is zero
  double sigma_x;      // correction = sigma_x * x
  double inv_sigma_b;  // b = r * inv_sigma_b
};
template <class T>
void launch_accum_defect(hipStream_t s, const StepK& k, const DefectArgs& a, const T* x, T* b,
                         double* part);

// p_out = z + beta p_in (z = sigma zT; p_out = z when first), q = S p_out and
// the partial sums of p_out . q
// The previous iteration's x update folded into the direction kernel:
// mode 0 none, 1 x = alpha p_in, 2 x += alpha p_in (p_in is that iteration's p).
struct XFold {
  double* x;
  double alpha;
  int mode;
};
template <class T>
void launch_pcg_dir(hipStream_t s, const StepK& k, const double* diag, const double* const cf[3],
                    const T* zT, double sigma, const double* p_in, double* p_out, double* q,
                    double beta, int first, const XFold& xf, double* part);
// x = (first ? 0 : x) + alpha p
void launch_xaxpy(hipStream_t s, long long N, double alpha, const double* p, double* x, int first);
// r -= alpha q, b = r * inv_sigma, norms of r; x += alpha p unless x == NULL
template <class T>
void launch_pcg_update(hipStream_t s, const StepK& k, double alpha, const double* p,
                       const double* q, double* x, double* r, double inv_sigma, T* b, int first,
                       double* part);
template <class T>
void launch_pcg_precond(hipStream_t s, const StepK& k, double sigma, const T* zT, const double* r,
                        const double* q, double* part);

// block smoother (rh_blocks.hip)
// count[g] = source cells (src > 0) among cells [g chunk, (g+1) chunk)
void launch_src_count(hipStream_t s, long long N, long long chunk, int groups, const double* src,
                      int* count);
// list[offset[g] + rank] = the source cells of range g, in cell order
void launch_src_list(hipStream_t s, long long N, long long chunk, int groups, const double* src,
                     const int* offset, int* list);
template <class T>
void launch_block_inverse(hipStream_t s, const LevelK<T>& l, const BlockSet<T>& bs);
// x += A_box^-1 (b - A x)_box on boxes [b0, b0 + nb) (one colour)
template <class T>
void launch_block_relax(hipStream_t s, const LevelK<T>& l, const BlockSet<T>& bs, int b0, int nb);

// ---- hydrogen + helium chemistry with multigroup radiation (rh_groups.hip)
// Local unknowns per cell, in this order: e, n_HI, n_HeI, n_HeII (an
// isothermal run keeps e = 0 with a trivial equation; a run without helium
// keeps the helium densities at 0 the same way).  Group fields are stored
// group after group ([G][N]); species fields [3][N] (n_HI, n_HeI, n_HeII).
constexpr int kMaxGroups = RH_MAX_GROUPS;
constexpr int kLoc = 4;
static_assert(kMaxGroups <= kLoc, "the local solves share one 4 x 4 elimination");
struct GroupK {
  int G;                              // groups
  int he;                             // helium present (y_he > 0)
  double y_he;                        // n_He / n_H
  double KGam[3][kMaxGroups];         // Gamma_s = c sum_g KGam[s][g] E_g (E proper)
  double KG[3][kMaxGroups];           // heating c sum_s sum_g KG[s][g] n_s E_g
  double sigE[3][kMaxGroups];         // opacity of group g: sum_s sigE[s][g] n_s
};
struct GroupLocalArgs {
  const double* Ek; const double* dE; double lam;  // E_k [G][N]; trial E = E_k + lam dE
  const double* ek; const double* yk;              // e [N] (null: isothermal), species [3][N]
  const double* pBf; const double* pBC;            // predictor data of U_k (may be null)
  const double* En; const double* en; const double* yn; const double* nH;
  double* Et; double* et; double* yt;              // outputs (mode 0)
  double* Bf;                                      // [4][N]  B^-1 f_loc
  double* BC;                                      // [4][G][N]  B^-1 C
  double* K;                                       // [G][G][N]  J B^-1 C
  double* kB;                                      // [G][N]  J B^-1 f_loc
  double* fe_out; double* fy_out;                  // optional residual outputs
  int mode;                                        // 0: solve at E, 1: evaluate
};
// Local solve (mode 0) or evaluation (mode 1) with partial sums of
// (f_e/e^n)^2 (RS_FE_LOC2), (f_HI/n_H)^2 + (f_HeI/n_He)^2 + (f_HeII/n_He)^2
// (RS_FN2), failures, iterations and non-finite values.
void launch_local_groups(hipStream_t s, const StepK& k, const GroupK& m, const GroupLocalArgs& a,
                     double* part);
// b = rS_g - S_gg x_g + sum_{h != g} K_gh x_h (the coupled Schur residual of
// group g at x), with partial sums of (b/E_s)^2 (RS_FE2), b^2 (RS_R2) and
// max |b| (RS_RMAX); diag and cf are group g's operator.
void launch_group_coupled(hipStream_t s, const StepK& k, int G, int g, const double* rS,
                       const double* diag, const double* const cf[3], const double* K,
                       const double* x, double* b, double* part);
// The G groups' Schur operators (diagonal and + face coefficients, each on
// its own grey handle), right-hand sides and norm scales.
struct GroupOps {
  const double* rS[kMaxGroups];
  const double* diag[kMaxGroups];
  const double* cf[kMaxGroups][3];
  double E_s[kMaxGroups];
};
// B[g] = rS_g - S_gg x_g + sum_{h != g} K_gh x_h for every group at once
// (rS_g null: B[g] = S_gg x_g - sum_{h != g} K_gh x_h, the operator applied
// to x), with the partial sums of sum_g (B_g / E_s,g)^2 (RS_FE2) and of the
// same sum over the magnitudes of the terms that make B_g (RS_MAG2: the
// scale of its rounding error).
void launch_groups_coupled(hipStream_t s, const StepK& k, int G, const GroupOps& o,
                           const double* K, const double* x, double* B, double* part);
// Krylov vectors over [G][N] fields with the inner product
// <u, v>_W = sum_g w[g] sum_P u v (w[g] = 1 / E_s,g^2, the norm's weights).
constexpr int kKrylovMax = 12;    // vectors one call combines or dots against
constexpr int kKrylovGrid = 1024; // workgroups of the Krylov kernels
struct WeightK {
  double w[kMaxGroups];
};
struct Coefs {
  double c[kKrylovMax];
};
// out[i] = <u, V_i>_W for i < nv (V_i = V + i stride); part: kKrylovMax *
// kKrylovGrid doubles of scratch; out may be mapped host memory.
void launch_wdots(hipStream_t s, long long N, int G, const WeightK& wk, const double* u,
                  const double* V, long long stride, int nv, double* part, double* out);
// y = a y + sum_{i < nv} c_i V_i (a = 0: y is overwritten); with norm_out,
// also *norm_out = ||y||_W^2 after the update.
void launch_wcombine(hipStream_t s, long long N, int G, const WeightK& wk, double* y, double a,
                     const double* V, long long stride, int nv, const Coefs& c, double* part,
                     double* norm_out);
// E_g = frac[g] E0, n_HI = (1 - x0) n_H, with helium n_HeI = (1 - x0) n_He
// and n_HeII = x0 n_He, e = e0 (e null: isothermal); RS_NONFINITE flags a
// bad n_H.
void launch_groups_init(hipStream_t s, long long N, const GroupK& m, const double* frac, double E0,
                    double x0, double e0, const double* nH, double* E, double* e, double* y,
                    double* part);

// advection of the step's fields (operator split, step (iv)), rh_advect.hip
struct AdvK {
  int nx, ny, nz;
  long long N;
  int bc[6];
  int iso;                  // 1: e is not advected
  double scale;             // substep / (a h): face velocity -> face Courant number
  const double* v[3];       // cell-centred proper peculiar velocity per axis
  const double* qi[4];      // n_H, E, n_HI, e of the substep's start
  double* qo[4];            // the same after the substep
};
// partial maxima of the outgoing Courant number per cell into RS_COURANT
void launch_advect_courant(hipStream_t s, const AdvK& a, double* part);
// one donor-cell substep qi -> qo (qo must not alias qi)
void launch_advect(hipStream_t s, const AdvK& a);

// adjoint step
struct AdjArgs {
  const double* E1; const double* e1; const double* n1;   // U^{n+1}
  const double* En; const double* en; const double* nn;   // U^n
  const double* nH; const double* muE;                     // mu_E of the Schur solve
  double* lE; double* le; double* ln;                      // in: lambda^{n+1}; out: lambda^n
  double* g_src; double* g_nH;                             // accumulated
};
void launch_adj_rhs(hipStream_t s, const StepK& k, const double* lE, const double* le,
                    const double* ln, const double* BCn, const double* BCe, double* r,
                    double* part);
void launch_adj_local(hipStream_t s, const StepK& k, const AdjArgs& a);
void launch_adj_limiter(hipStream_t s, const StepK& k, const AdjArgs& a);

}  // namespace rh
