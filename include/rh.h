/*
 * rh.h -- C ABI of the MI355X implementation of the coupled implicit
 * radiation / ionisation / photoheating step of Norman, Reynolds & So,
 * "Cosmological Radiation Hydrodynamics with Enzo" (arXiv:0908.2654).
 *
 * The step is the implicit subsystem of the paper's operator split
 * (Algorithm section, step (v)): given the state U^n = (E, e, n_HI) at
 * t_n, the hydrogen density n_H and the emissivity src = 4 pi eta, find
 * U^{n+1} with f(U^{n+1}) = 0, where f stacks the gas-energy residual, the
 * chemistry residual and the theta-method residual of the grey
 * flux-limited-diffusion equation (equations gas_residual,
 * chemistry_residual, radiation_residual; limiter from equation limiter;
 * convergence in the RMS norm of equation rmsnorm).  Newton's linear
 * systems are reduced by a Schur complement to a 7-point variable-
 * coefficient diffusion system (the paper's "modified radiation
 * equation"), solved by geometric multigrid V-cycles.
 *
 * Conventions shared by every entry point
 *  - Grid: nx*ny*nz cubic cells of comoving width h = box_comoving_cm/nx.
 *  - Every field argument is a contiguous float64 array in device memory
 *    of nx*ny*nz entries, C order [x][y][z] (z fastest, index
 *    (i*ny + j)*nz + k), comoving CGS units:
 *      E    radiation energy density      erg cm^-3
 *      e    specific gas energy           erg g^-1
 *      nHI  neutral hydrogen density      cm^-3
 *      nH   total hydrogen density        cm^-3
 *      src  4 pi eta (emissivity)         erg cm^-3 s^-1
 *  - Device pointers must be distinct, 8-byte aligned and resident on the
 *    device that was current at rh_setup.  The caller owns all device
 *    memory, including the workspace; the library owns only its handle and
 *    a few bytes of pinned host memory.  No entry point allocates device
 *    memory after rh_setup.
 *  - Work is enqueued on the stream given to rh_setup; calls return after
 *    the last host-side convergence decision, with outputs complete on that
 *    stream.  A handle is bound to one stream and is not thread safe.
 *  - Every entry point returns an rh_status; rh_last_error gives the
 *    message.  RH_EINVAL is returned before any device work is enqueued.
 */
#ifndef RH_H
#define RH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RH_OK = 0,
  RH_EINVAL = 1,     /* invalid parameter, size or pointer                        */
  RH_ENOMEM = 2,     /* workspace smaller than rh_workspace_bytes                 */
  RH_EHIP = 3,       /* a HIP runtime call failed                                 */
  RH_ENONFINITE = 4, /* a residual or an input became NaN / Inf                   */
  RH_ENEWTON = 5,    /* Newton or its line search did not converge                */
  RH_ELINEAR = 6     /* the local per-cell solve or the linear solve broke down   */
} rh_status;

enum { RH_BC_ZEROFLUX = 0, RH_BC_PERIODIC = 1, RH_BC_OUTFLOW = 2 };
enum { RH_SPEC_MONO = 0, RH_SPEC_BLACKBODY = 1 };
enum { RH_RATES_CONST = 0, RH_RATES_FIT = 1 };
enum { RH_COOL_RECB = 1, RH_COOL_COLLEXC = 2, RH_COOL_COMPTON = 4 };
/* Expansion laws (Physical Model section; Friedmann equation): static a = 1;
 * Einstein-de Sitter (Omega_m = 1); flat LCDM (Omega_m + Omega_L = 1); open
 * (Omega_L = 0, 0 < Omega_m < 1: the q0 = Omega_m / 2 = 0.05 rows of the
 * verification section's table). */
enum { RH_COSMO_STATIC = 0, RH_COSMO_EDS = 1, RH_COSMO_FLAT_LCDM = 2, RH_COSMO_OPEN = 3 };
enum { RH_PREC_FP64 = 0, RH_PREC_MIXED = 1 };

/* Problem and solver parameters (plain data, validated by rh_setup). */
typedef struct rh_params {
  int32_t nx, ny, nz;          /* grid; multigrid halves all three while they are even  */
  int32_t bc[6];               /* per face x-, x+, y-, y+, z-, z+ (periodic in pairs)   */
  double box_comoving_cm;      /* comoving x edge of the box                             */
  int32_t isothermal;          /* 1: T fixed at T_iso_K, e is neither read nor written  */
  int32_t spectrum;            /* RH_SPEC_*: grey constants (equation grey_definition)  */
  double T_iso_K;
  double T_bb_K;               /* blackbody temperature (paper: 1e5 K)                   */
  double hnu0_eV;              /* ionisation threshold (13.6 eV)                         */
  double sigma0_cm2;           /* threshold cross-section sigma(nu) = sigma0 (nu0/nu)^3  */
  int32_t rates;               /* RH_RATES_CONST: alpha_B = alphaB_const; _FIT: fits     */
  int32_t cooling_mask;        /* RH_COOL_* bits (ignored when isothermal)               */
  double alphaB_const;         /* cm^3 s^-1 (paper: 2.59e-13)                            */
  int32_t cosmology;           /* RH_COSMO_*: expansion factor a(t), Hubble rate H(t)    */
  int32_t precision;           /* RH_PREC_FP64: all FP64; _MIXED: FP32 V-cycles inside  */
                               /* the FP64 outer iteration, each FP32 level's operator   */
                               /* held as bfloat16 faces and shift (diagonal minus the   */
                               /* faces), 8 bytes per cell; the outer iteration and the  */
                               /* Newton residual stay on the exact FP64 operator        */
  double hubble_h, Omega_m, Omega_L;
  double theta;                /* time-centring of the theta method, (0, 1]; 1 = backward Euler */
  double E_floor;              /* floor of face-mean E in the limiter (default 1e-40)    */
  double R_min;                /* limiter floor on |grad E|/E; <= 0 selects 1/(a_n box)  */
  double gamma;                /* ratio of specific heats (5/3)                          */
  double newton_tol;           /* stop when ||f(U)|| <= newton_tol (RMS norm)            */
  int32_t newton_max_it;       /* Newton iterations before RH_ENEWTON                    */
  int32_t ls_max_cuts;         /* line-search halvings per iteration                     */
  double lin_forcing;          /* linear solve to ||r|| <= lin_forcing ||f(U_k)|| (1e-13) */
  int32_t lin_max_it;          /* outer linear iterations (V-cycles) per solve (500).     */
                               /* rh_implicit_step: a solve that stops here without      */
                               /* reaching its forcing is used as an inexact Newton      */
                               /* direction (Newton still stops only at newton_tol) and  */
                               /* is counted in rh_step_stats.lin_cap_hits.              */
                               /* rh_adjoint_step: returns RH_ELINEAR instead (nothing   */
                               /* corrects an inexact transpose solve).                  */
  int32_t mg_pre, mg_post;     /* red-black Gauss-Seidel sweeps before / after coarsening */
  int32_t mg_coarse_max;       /* stop coarsening at <= this many cells (<= 512)         */
  int32_t krylov;              /* outer linear iteration: 1 = conjugate gradients with   */
                               /* the V-cycle as preconditioner (default), 0 = plain     */
                               /* defect correction x += V(b - S x)                      */
  int32_t smoother;            /* multigrid kernel form: 0 = auto (the red-black sweep   */
                               /* as one marching launch for both colours, and the       */
                               /* residual fused with the restriction, on levels where   */
                               /* they get >= 256 (sweep) / 512 (residual) workgroups,   */
                               /* with the longest x chunks that keep that many;         */
                               /* elsewhere one launch per colour and separate residual  */
                               /* and restriction), 1 =                                  */
                               /* always the separate launches, 2 = the marching         */
                               /* launches on every level their tiles fit (FP32 levels:  */
                               /* nz >= 64, ny >= 16; FP64: nz >= 32, ny >= 8; nx >= 4). */
                               /* Same iterates up to rounding order.                    */
  int32_t mg_block_radius;     /* block smoother around point sources (default 2; 0 off,  */
                               /* at most 2): on the finest mg_block_levels levels the   */
                               /* V-cycle also solves the operator exactly on a box of   */
                               /* (2R+1)^3 cells around each cell holding a source (src  */
                               /* > 0; on coarse levels the cell containing it), after   */
                               /* the pre-smoothing and before the post-smoothing.  The  */
                               /* face-limited diffusion is strongly anisotropic around  */
                               /* sources (radial faces see the steep fall-off of E,     */
                               /* tangential ones R = R_min), and those modes need it.   */
  int32_t mg_block_levels;     /* levels with source boxes (default 2, at most 4)        */
  int32_t mg_block_max;        /* most source cells with boxes; 0 (default): one per     */
                               /* 4096 cells, at least 64, at most 8192.  The workspace  */
                               /* grows by 4 (FP32) or 8 (FP64) x (2R+1)^6 bytes per box */
                               /* and level; a step with more source cells runs without  */
                               /* boxes                                                  */
} rh_params;

/* Per-step statistics (host memory). */
typedef struct rh_step_stats {
  int32_t newton_its;          /* Newton iterations taken                                */
  int32_t lin_its_total;       /* V-cycles over all Newton iterations                    */
  int32_t ls_cuts;             /* line-search halvings                                   */
  int32_t local_its_max;       /* most per-cell local Newton iterations in any call      */
  double res0, res_final;      /* ||f|| at the start and at the end                      */
  double lin_res_max;          /* largest final linear residual of a Newton iteration,   */
                               /* relative to that iteration's ||f|| (E-weighted norm);  */
                               /* the forcing is met when <= lin_forcing                 */
  double t_ms[8];              /* GPU time (ms) from events on the handle's stream:      */
                               /* [0] the whole call; [1..5] partition it by phase:      */
                               /* 1 state copies, face limiter, coarse face hierarchy;   */
                               /* 2 local solves, residuals and norms (Newton iterates   */
                               /* and line-search trials; the adjoint's local terms);    */
                               /* 3 coarse-level operators and the coarsest inverse;     */
                               /* 4 V-cycles; 5 the outer linear iteration (conjugate-   */
                               /* gradient or defect-correction kernels and their        */
                               /* reductions).  Host latency between launches counts in  */
                               /* the phase it interrupts.  [6], [7] are 0.  The same    */
                               /* phases are ROCTx ranges (host time, enqueues + waits)  */
                               /* inside one range per call, for a profiler's marker     */
                               /* trace.                                                 */
  int32_t lin_cap_hits;        /* linear solves that stopped without reaching their      */
                               /* target (at lin_max_it, on stagnation or breakdown)     */
  int32_t lin_its_max;         /* most V-cycles in one linear solve of the call          */
  int32_t source_boxes;        /* boxes of the block smoother on the finest level (0:    */
                               /* none this step)                                        */
} rh_step_stats;

/* Statistics of rh_advance (host memory). */
typedef struct rh_advance_stats {
  int32_t steps;               /* accepted implicit steps                                */
  int32_t rejected;            /* rejected attempts (failed step or negative E)          */
  int32_t newton_its;          /* Newton iterations over the accepted steps              */
  int32_t lin_its_total;       /* V-cycles over the accepted steps                       */
  double dt_min, dt_max;       /* smallest / largest accepted step (s)                   */
  double dt_next;              /* step the controller proposes for the next call (s)     */
  double change_max;           /* largest weighted change of an accepted step            */
  double change_last;          /* weighted change of the last accepted step              */
} rh_advance_stats;

/* Statistics of rh_advect (host memory). */
typedef struct rh_advect_stats {
  int32_t substeps;            /* donor-cell substeps taken                               */
  double courant;              /* largest outgoing Courant number over the whole dt      */
  double courant_substep;      /* the same per substep (<= cfl)                          */
} rh_advect_stats;

typedef struct rh_handle rh_handle;

/* Fill p with the defaults (a 16^3 static zero-flux grid; every solver
 * setting at its documented default).  Never fails. */
void rh_default_params(rh_params* p);

/* Bytes of device workspace rh_setup needs for p, or 0 if p is invalid. */
size_t rh_workspace_bytes(const rh_params* p);

/* Validate p, compute the grey constants (grey_definition, host FP64
 * series), plan the multigrid levels and carve the workspace.
 * workspace: device memory of ws_bytes >= rh_workspace_bytes(p), owned by
 * the caller and untouched by it while the handle lives.  hip_stream: a
 * hipStream_t (NULL = default stream).  *out receives the handle. */
rh_status rh_setup(const rh_params* p, void* workspace, size_t ws_bytes, void* hip_stream,
                   rh_handle** out);

/* One implicit step from t_n to t_n + dt_s (Algorithm section, step (v)).
 * In: E, e, nHI hold U^n.  Out: they hold U^{n+1}.  nH, src are read only.
 * On RH_ENEWTON, RH_ELINEAR or RH_ENONFINITE the arrays are restored to
 * U^n, so the caller may retry with a smaller step.  stats may be NULL. */
rh_status rh_implicit_step(rh_handle* h, double t_n_s, double dt_s, const double* nH,
                           const double* src, double* E, double* e, double* nHI,
                           rh_step_stats* stats);

/* Adjoint of one implicit step (implicit-function theorem at the converged
 * U^{n+1}).  With f(U^{n+1}; U^n, nH, src) = 0 and lambda^{n+1} = dJ/dU^{n+1}
 * given in (lE, le, lnHI), solve J_U^T mu = lambda^{n+1} (the transposed
 * Newton system; after local elimination the same symmetric Schur operator
 * as the forward step) and return lambda^n = -(df/dU^n)^T mu in (lE, le,
 * lnHI) (overwritten), and accumulate g_src += -(df/dsrc)^T mu and
 * g_nH += -(df/dnH)^T mu.  The transposed solve runs to ||r||_2 <= lin_forcing
 * (default 1e-13) of its right-hand side; if it stops short (lin_max_it reached, stagnation)
 * the call returns RH_ELINEAR and leaves lE, le, lnHI, g_src, g_nH as they
 * were.  E_n..nHI_n and E_1..nHI_1 are the checkpoints
 * U^n and U^{n+1} (read only).  le and the e-checkpoints are ignored for
 * isothermal runs.  stats may be NULL. */
rh_status rh_adjoint_step(rh_handle* h, double t_n_s, double dt_s, const double* nH,
                          const double* src, const double* E_n, const double* e_n,
                          const double* nHI_n, const double* E_1, const double* e_1,
                          const double* nHI_1, double* lE, double* le, double* lnHI,
                          double* g_src, double* g_nH, rh_step_stats* stats);

/* Advance (E, e, nHI) in place from t0 to t_end with implicit steps whose
 * size follows the temporal accuracy tau_tol (Verification section: the
 * solver settings name tau_tol next to theta and the norm exponent p = 2;
 * the controller itself is given in the method's companion paper, this is
 * its reading): after an accepted step the weighted RMS change
 *   w = sqrt(sum_P [(dE/E_s)^2 + (de/e^n)^2 + (dn_HI/n_H)^2] / (N nvars)),
 * with the weights of the Newton norm (equation rmsnorm, E_s as there), sets
 * the next step dt * clamp(tau_tol / w, 0.1, 2), capped by dt_max_s and
 * shortened to land on t_end.  An attempt is rejected and retried with half
 * the step when rh_implicit_step fails (RH_ENEWTON, RH_ELINEAR,
 * RH_ENONFINITE) or when some E^{n+1} < -1e-10 E_s (positivity safeguard for
 * theta < 1: the explicit part can flip the sign of E in optically thick
 * cells); a rejected attempt leaves the state at U^n.  dt0_s is the first
 * attempted step.  Returns RH_OK on reaching t_end; otherwise the status of
 * the last failed attempt after 12 consecutive rejections (state at the last
 * accepted time, reported by *t_reached).  stats and t_reached may be NULL.
 * Device fields as for rh_implicit_step. */
rh_status rh_advance(rh_handle* h, double t0_s, double t_end_s, double dt0_s, double tau_tol,
                     double dt_max_s, const double* nH, const double* src, double* E, double* e,
                     double* nHI, rh_advance_stats* stats, double* t_reached);

/* Advect (nH, E, e, nHI) in place from t0_s to t0_s + dt_s with the
 * prescribed velocity (vx, vy, vz): the part of the operator split's
 * hydrodynamic step that moves the number densities and the radiation
 * energy before the implicit step (Algorithm section, step (iv); equations
 * enzo-chemical_ionization and enzo-cons_radiation: d_t q + (1/a) div(q v)
 * = 0, comoving divergence, proper peculiar velocity).  Call rh_implicit_step
 * on the advected fields afterwards to complete the split step.
 *   - Velocities: cell-centred, cm/s, device FP64 fields like the others
 *     (read only; must not alias the advected fields).  A face takes the
 *     mean of its two cells; 0 at an RH_BC_ZEROFLUX wall (closed box); the
 *     boundary cell's velocity at an RH_BC_OUTFLOW wall, where the ghost
 *     cell repeats the boundary cell's values; periodic axes wrap.
 *   - Conserved per cell: nH, E, nHI and nH * e (e is energy per unit
 *     mass); e is recovered as (nH e) / nH.  e is neither read nor written
 *     when isothermal (may be NULL then).
 *   - Scheme: first-order donor-cell (upwind) fluxes, unsplit over the three
 *     axes, in m equal substeps, m = max(1, ceil(C / cfl)) where C is the
 *     largest outgoing Courant number of a cell (sum over its faces of
 *     dt v_face / (a h) pointing out of it) at a(t0); each substep uses a at
 *     its midpoint.  With cfl <= 1 every substep is a convex combination:
 *     fields stay non-negative and e, nHI / nH stay within their
 *     neighbours' range.
 * 0 < cfl <= 1.  Uses the handle's workspace as scratch (not during another
 * call on h).  Returns RH_ENONFINITE, fields untouched, when a velocity is
 * not finite; RH_EINVAL when more than 2^20 substeps would be needed or when
 * two advected fields, or a velocity and a field, are the same array.
 * The call synchronises its stream.  stats may be NULL. */
rh_status rh_advect(rh_handle* h, double t0_s, double dt_s, const double* vx, const double* vy,
                    const double* vz, double cfl, double* nH, double* E, double* e, double* nHI,
                    rh_advect_stats* stats);

/* Evaluate the residual f(U) of the step from U^n = (E_n, e_n, nHI_n) at
 * the state U = (E, e, nHI), exactly as rh_implicit_step does (face limiter
 * from U^n, theta-method radiation residual, local residuals).  Outputs
 * fE, fe, fn (device, may be NULL to skip; fe unused when isothermal) and
 * *norm_out (host) = ||f(U)|| in the RMS norm. */
rh_status rh_residual(rh_handle* h, double t_n_s, double dt_s, const double* nH,
                      const double* src, const double* E_n, const double* e_n,
                      const double* nHI_n, const double* E, const double* e,
                      const double* nHI, double* fE, double* fe, double* fn,
                      double* norm_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as rh_residual, with no handle and no workspace.  p as for
 * rh_setup (validated the same way); hip_stream a hipStream_t (NULL = the
 * default stream) of the current device.  The face coefficients, local
 * terms and reduction partials live in a static device array of the
 * library (about 18.3 MiB per GPU, held until the process ends), so grids
 * are limited to 64^3 = 262144 cells (larger: RH_EINVAL, nothing
 * enqueued).  Calls on one GPU share that array: calls that overlap in
 * time on the same GPU (other host threads or streams) race and must be
 * serialised by the caller; nothing in the array needs to start at zero
 * (every value a call reads was written earlier in that call).  Calls no
 * hipMalloc or hipFree (the first call on a device looks up the array's
 * address); synchronises hip_stream twice.  Errors: rh_last_error(NULL). */
rh_status rh_residual_noalloc(const rh_params* p, void* hip_stream, double t_n_s, double dt_s,
                              const double* nH, const double* src, const double* E_n,
                              const double* e_n, const double* nHI_n, const double* E,
                              const double* e, const double* nHI, double* fE, double* fe,
                              double* fn, double* norm_out);

/* Write the Schur operator S of the Newton system at U = (E, e, nHI) of the
 * step from U^n (Algorithm section: the radiation equation after the local
 * unknowns are eliminated), the operator rh_schur_solve inverts:
 *   (S x)_P = diag_P x_P - sum_d [cf_d,P x_{P+e_d} + cf_d,P-e_d x_{P-e_d}],
 * where cf_d,P couples cell P with its + neighbour along axis d (x, y, z),
 * wrapping on periodic axes; cf_d,P is 0 for the last cell along a
 * non-periodic axis.  diag, cf_x, cf_y, cf_z: device fields (FP64, z
 * fastest, caller-owned), overwritten; the call synchronises its stream. */
rh_status rh_schur_operator(rh_handle* h, double t_n_s, double dt_s, const double* nH,
                            const double* src, const double* E_n, const double* e_n,
                            const double* nHI_n, const double* E, const double* e,
                            const double* nHI, double* diag, double* cf_x, double* cf_y,
                            double* cf_z);

/* Solve S x = b with the configured multigrid (defect correction in FP64,
 * V-cycles in FP32 or FP64 by p->precision), where S is the Schur operator
 * of the Newton system at U = (E, e, nHI) of the step from U^n: the
 * modified radiation equation (Algorithm section), with the outer iteration
 * chosen by p->krylov.  b, x: device fields.
 * Stops when ||b - S x||_2 <= rel_tol ||b||_2 or after max_it cycles;
 * *iters and *rel_res (host, may be NULL) report what was reached. */
rh_status rh_schur_solve(rh_handle* h, double t_n_s, double dt_s, const double* nH,
                         const double* src, const double* E_n, const double* e_n,
                         const double* nHI_n, const double* E, const double* e,
                         const double* nHI, const double* b, double* x, double rel_tol,
                         int32_t max_it, int32_t* iters, double* rel_res);

/* Initial fields of a run (verification and reionisation sections start
 * from uniform radiation, a given ionised fraction and a given temperature):
 * E = E0 everywhere, nHI = (1 - x0) nH and, when e is not NULL, the specific
 * gas energy of temperature T0_K at ionised fraction x0 from the ideal-gas
 * relation T = (gamma - 1) mu m_H e / k_B with mu = 1 / (1 + x0) (pure
 * hydrogen; the printed temperature and equation-of-state equations compose
 * to an extra factor gamma - 1, which is not used).  Isothermal runs use
 * T_iso_K instead of T0_K and accept e == NULL; otherwise e is required.
 * nH: device, read only (every entry finite and > 0, else RH_ENONFINITE,
 * outputs then partly written).  0 <= x0 < 1, T0_K > 0, finite E0 >= 0,
 * else RH_EINVAL.  Synchronises the stream. */
rh_status rh_initial_state(rh_handle* h, const double* nH, double x0, double T0_K, double E0,
                           double* E, double* e, double* nHI);

/* Emissivity src = 4 pi eta (erg cm^-3 s^-1, comoving) of point sources
 * from their photon rates: photon_rate[P] (photons s^-1 emitted in cell P;
 * the sum of the sources in that cell) times the mean photon energy of the
 * spectrum (equation grey_definition) over the comoving cell volume h^3.
 * Device arrays; RH_ENONFINITE if a rate is negative or not finite (src
 * then written anyway).  Synchronises the stream. */
rh_status rh_source_field(rh_handle* h, const double* photon_rate, double* src);

/* Derived constants of the handle: out[0] sigma_E (cm^2), out[1] K_Gamma
 * (cm^2 erg^-1), out[2] K_G (cm^2), out[3] eps_bar (erg, mean photon energy),
 * out[4] h nu_0 (erg), out[5] cell width h (comoving cm), out[6] number of
 * multigrid levels, out[7] cells on the coarsest level.  n >= 8. */
rh_status rh_get_constants(const rh_handle* h, double* out, int32_t n);

/* Per-kernel GPU timing for measurement.  When enabled, every kernel launch
 * of the step is bracketed by a pair of hipEvents recorded on the handle's
 * stream (a fixed pool created here, read back at the step's own
 * synchronisation points).  Adds host overhead; off by default. */
rh_status rh_set_kernel_timing(rh_handle* h, int32_t enable);

/* Accumulated time (ms) and launch count per kernel class since the last
 * reset, for classes 0..n-1: 0 step setup (face limiter), 1 local solve,
 * 2 radiation residual + Schur diagonal, 3 reduction finalize, 4 red-black
 * Gauss-Seidel sweep (both colours, one launch) on the finest level, 5 multigrid residual
 * (finest; fused with the restriction when the level takes the fused sweep), 6 restriction
 * (finest, when not fused), 7 prolongation (finest), 8 coarse levels
 * (all work below the finest level), 9 conjugate-gradient direction and
 * S p, 10 conjugate-gradient update, 11 preconditioner rescale, 12 defect
 * correction update, 13 right-hand-side cast, 14 one colour of a sweep on
 * a finest level too small for the fused sweep, 15 the last fused sweep of
 * a V-cycle on the finest level when it also forms the conjugate-gradient
 * dot products (class 11 then has no launches), 16 advection substep
 * (rh_advect), 17 its Courant-number reduction, 18 block relaxation around the
 * sources on the finest level, 19 the box inverses of the block smoother
 * (all levels; block relaxation below the finest level counts in 8); 20..22 are used by
 * the multigroup step (rh_multigroup_get_kernel_timing).  ms / counts are host arrays
 * (either may be NULL); reset != 0 clears the totals afterwards. */
rh_status rh_get_kernel_timing(rh_handle* h, double* ms, int64_t* counts, int32_t n,
                               int32_t reset);

/* Expansion factor and Hubble rate at cosmic time t_s (host, pure):
 * a(t) and H(t) = (da/dt)/a from the Friedmann equation for p. */
rh_status rh_cosmology_at(const rh_params* p, double t_s, double* a, double* H);

/* Cosmic time at which a(t) = a (host, pure; not for the static case). */
rh_status rh_cosmic_time(const rh_params* p, double a, double* t_s);

/* Message of the last failed call on h (host string, valid until the next
 * call on h).  h may be NULL: then the message of the last failed
 * rh_setup / rh_workspace_bytes on this thread. */
const char* rh_last_error(const rh_handle* h);

/* Release the handle (not the caller's workspace).  NULL is accepted. */
void rh_destroy(rh_handle* h);

/* ---- Hydrogen + helium chemistry with multigroup radiation -------------
 * The extension the Conclusions and outlook section names first: the
 * multi-frequency radiation equation (equation cons_radiation_multifreq)
 * integrated over G frequency groups instead of one, and helium ionisation
 * (electron density with helium: equation electron_density, second
 * branch).  The paper prints neither; these are this library's definitions.
 *
 *  - Groups: lower edges edge_eV[0] = p->hnu0_eV < edge_eV[1] < ... (the
 *    last group extends to infinity).  Within a group the spectrum keeps the
 *    shape of the T_bb_K blackbody (equation grey_definition applied per
 *    group).  With x = h nu / (k T_bb) and b(x) = 1 / (e^x - 1):
 *      I_g = int_g x^3 b dx (group energy), f_g = I_g / sum_h I_h (share of
 *      the source energy), and per species s = HI, HeI, HeII, with
 *      sigma_s(nu) = sigma_s0 (nu_s / nu)^sigma_power above its threshold
 *      nu_s (HI: hnu0_eV, sigma0_cm2; HeI: 24.587 eV, 7.42e-18 cm^2; HeII:
 *      4 hnu0_eV, sigma0_cm2 / 4):
 *        sigma_E[s][g] = int_g sigma_s x^3 b dx / I_g              (opacity)
 *        K_Gamma[s][g] = int_g sigma_s x^2 b dx / (k T_bb I_g)      (ionisation)
 *        K_G[s][g]     = sigma_E[s][g] - h nu_s K_Gamma[s][g]       (heating)
 *    by host quadrature.  One group without helium gives the grey constants.
 *  - Fields (device FP64, z fastest as above): E [G][N] (group energies,
 *    group after group, erg cm^-3), e [N], y [3][N] = (n_HI, n_HeI, n_HeII)
 *    (cm^-3, comoving); n_He = y_he n_H, n_HII = n_H - n_HI,
 *    n_HeIII = n_He - n_HeI - n_HeII, n_e = n_HII + n_HeII + 2 n_HeIII,
 *    mu = (n_H + 4 n_He) / (n_H + n_He + n_e), T = (gamma - 1) mu m_H e / k_B.
 *    Without helium rows 1 and 2 of y are neither read nor written.
 *  - Chemistry (equation chemical_ionization for each species):
 *      dn_HI/dt   = alpha_H n_e n_HII - Gamma_HI n_HI
 *      dn_HeI/dt  = alpha_HeII n_e n_HeII - Gamma_HeI n_HeI
 *      dn_HeII/dt = Gamma_HeI n_HeI - (Gamma_HeII + alpha_HeII n_e) n_HeII
 *                   + alpha_HeIII n_e n_HeIII
 *    with Gamma_s = c sum_g K_Gamma[s][g] E_g (proper), alpha_H the grey
 *    step's recombination rate, alpha_HeII = 1.26e-14 (570670 K / T)^0.75
 *    cm^3 s^-1, alpha_HeIII(T) = 2 alpha_H(T / 4).
 *  - Gas energy: heating c sum_s sum_g K_G[s][g] n_s E_g; the grey step's
 *    cooling terms with the full n_e (recombination cooling n_e n_HII) and,
 *    with RH_COOL_RECB, helium recombination cooling
 *    k_B T alpha_HeII n_e n_HeII + 8 L_recB(T / 4) n_e n_HeIII.
 *  - Discretisation: the grey step's, per group (opacity sum_s sigma_E[s][g]
 *    n_s, face limiter from E_g^n and that opacity at t_n, source f_g src,
 *    no exchange between groups) and per species (theta method with a and
 *    M frozen at the implicit level:
 *    (I + theta dt M(U)) S = y^n + dt [theta a(U) + (1 - theta)(a^n - M^n y^n)]).
 *  - Norm: RMS over G + 4 unknowns per cell (one fewer when isothermal, two
 *    fewer without helium), weights E_s of each group (as the grey E_s),
 *    e^n, n_H for n_HI and n_He for the helium species.
 * Solver: Newton with the local unknowns eliminated per cell.  The Schur
 * system couples the groups only within a cell; it is solved by flexible
 * GMRES (restart 8, the norm's weights in its inner product), preconditioned
 * by one block Gauss-Seidel sweep over the groups in which each group's
 * 7-point system is solved by the configured multigrid to 1/50 of its
 * residual, until the coupled residual is below lin_forcing ||f|| or at its
 * FP64 rounding floor (1e-15 of the RMS of the terms it sums), for at most
 * lin_max_it sweeps.  Isothermal runs accept e == NULL. */
#define RH_MAX_GROUPS 4
typedef struct rh_multigroup_params {
  int32_t groups;                /* 1 .. RH_MAX_GROUPS                                  */
  int32_t reserved;              /* 0                                                   */
  double edge_eV[RH_MAX_GROUPS]; /* lower group edges, increasing, edge_eV[0] = hnu0_eV */
  double y_he;                   /* n_He / n_H (0: hydrogen only)                       */
  double sigma_power;            /* power of the cross-sections' frequency law (3)      */
} rh_multigroup_params;

typedef struct rh_multigroup rh_multigroup;

/* Group constants for p (p->spectrum must be RH_SPEC_BLACKBODY) and mg,
 * host only: out[0 .. G) f_g; then sigma_E, K_Gamma and K_G, each [3][G]
 * (species HI, HeI, HeII; cm^2, cm^2 erg^-1, cm^2); then eps_bar (erg, mean
 * photon energy of the whole spectrum above hnu0, as in the grey case).
 * n >= 10 G + 1, else RH_EINVAL.  Errors: rh_last_error(NULL). */
rh_status rh_multigroup_constants(const rh_params* p, const rh_multigroup_params* mg, double* out,
                                  int32_t n);

/* Bytes of device workspace rh_multigroup_setup needs (one grey workspace
 * per group plus the coupled fields), or 0 if p or mg is invalid. */
size_t rh_multigroup_workspace_bytes(const rh_params* p, const rh_multigroup_params* mg);

/* As rh_setup, for the multigroup step: validates p (as rh_setup does) and
 * mg, computes the group constants and carves the caller's workspace (at
 * least rh_multigroup_workspace_bytes).  Errors: rh_last_error(NULL). */
rh_status rh_multigroup_setup(const rh_params* p, const rh_multigroup_params* mg, void* workspace,
                              size_t ws_bytes, void* hip_stream, rh_multigroup** out);

/* Initial fields: E_g = f_g E0, n_HI = (1 - x0) n_H, n_HeI = (1 - x0) n_He,
 * n_HeII = x0 n_He, and (e not NULL) e of temperature T0_K (T_iso_K when
 * isothermal) at those fractions.  Arguments and errors as rh_initial_state. */
rh_status rh_multigroup_initial_state(rh_multigroup* h, const double* nH, double x0, double T0_K,
                                      double E0, double* E, double* e, double* y);

/* One implicit step from t_n to t_n + dt_s of the multigroup system: In:
 * E, e, y hold U^n; out: U^{n+1}.  On RH_ENEWTON, RH_ELINEAR or
 * RH_ENONFINITE they are restored to U^n.  stats (may be NULL) as for
 * rh_implicit_step, except lin_its_total (multigrid iterations over all
 * groups and sweeps), lin_its_max (most preconditioner sweeps of one Newton
 * iteration), lin_cap_hits (Newton iterations whose coupled solve stopped
 * above both its target and its rounding floor) and lin_res_max (largest
 * ratio of the final coupled residual to ||f||, floor stops included);
 * t_ms[1..5] are 0. */
rh_status rh_multigroup_step(rh_multigroup* h, double t_n_s, double dt_s, const double* nH,
                             const double* src, double* E, double* e, double* y,
                             rh_step_stats* stats);

/* Residual of the multigroup step from U^n = (E_n, e_n, y_n) at U = (E, e,
 * y), as rh_multigroup_step evaluates it: fE [G][N], fe [N], fy [3][N]
 * (device, each may be NULL; fe unused when isothermal, fy rows 1-2 without
 * helium) and *norm_out (host) = ||f(U)||. */
rh_status rh_multigroup_residual(rh_multigroup* h, double t_n_s, double dt_s, const double* nH,
                                 const double* src, const double* E_n, const double* e_n,
                                 const double* y_n, const double* E, const double* e,
                                 const double* y, double* fE, double* fe, double* fy,
                                 double* norm_out);

/* Per-kernel GPU timing of the multigroup step (as rh_set_kernel_timing /
 * rh_get_kernel_timing, for every group's handle): the totals are summed
 * over the groups.  Classes 0..19 as for the grey step (each launch covers
 * one group's N cells), 20 the local solves over the species (all groups,
 * one launch), 21 the coupled residuals and operator applications of the
 * FGMRES solve, 22 its vector work (Gram-Schmidt dot products, basis and
 * solution updates, the preconditioner's accumulation). */
rh_status rh_multigroup_set_kernel_timing(rh_multigroup* h, int32_t enable);
rh_status rh_multigroup_get_kernel_timing(rh_multigroup* h, double* ms, int64_t* counts,
                                          int32_t n, int32_t reset);

/* Message of the last failed call on h (NULL: of the last failed
 * rh_multigroup_setup / _constants / _workspace_bytes on this thread). */
const char* rh_multigroup_last_error(const rh_multigroup* h);

/* Release the handle (not the caller's workspace).  NULL is accepted. */
void rh_multigroup_destroy(rh_multigroup* h);

#ifdef __cplusplus
}
#endif

#endif /* RH_H */
