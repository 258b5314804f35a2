// Host-side internals shared by the grey driver (rh_host.cpp) and the
// multigroup driver (rh_groups_host.cpp): the handle and the grey step's
// building blocks the multigroup step reuses per group.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "rh_internal.h"

namespace rh {

// Grey constants of the spectrum (equation grey_definition).
struct Grey {
  double sigma_E, K_Gamma, K_G, eps_bar, hnu0;
};

// Multigrid level plan.
struct Plan {
  int nlev;
  int dims[kMaxLevels][3];
};

}  // namespace rh

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
struct StateBuf {
  double* E;
  double* e;
  double* n;
  double* loc[4];  // BCn, BCe, Bfn, Bfe
};

enum KernelKind {
  KK_SETUP = 0, KK_LOCAL, KK_RESID, KK_FINALIZE, KK_RBGS0, KK_MGRES0, KK_RESTRICT0, KK_PROLONG0,
  KK_COARSE, KK_PCG_DIR, KK_PCG_UPD, KK_PCG_PRE, KK_DEFECT, KK_CAST, KK_RBGS0C, KK_RBGS0D,
  KK_ADVECT, KK_ADVECT_C, KK_BLOCK0, KK_BLOCKINV,
  // multigroup step: local solves over the species, coupled residuals, the
  // FGMRES vector work (timed on the first group's handle)
  KK_LOCALG, KK_GCOUPLED, KK_KRYLOV, KK_COUNT
};

struct rh_handle {
  rh_params p;
  rh::Plan plan;
  rh::Grey g;
  double h, compton;
  long long N;
  hipStream_t stream;
  int device;
  char* ws;
  size_t ws_bytes;
  // fine FP64 fields
  double *En, *en, *nn, *rhsn, *rS, *diag64, *dEa, *dEb;
  double *r64, *pa, *pb, *q64;  // conjugate-gradient vectors
  double* cf64[3];
  StateBuf B;
  double* locA[4];
  double* part;
  // levels
  rh::LevelK<float> L32[rh::kMaxLevels];
  rh::LevelK<double> L64[rh::kMaxLevels];
  // source-centred boxes of the block smoother (levels 0 .. nblk - 1)
  int nblk = 0;                        // levels with boxes this step
  rh::BlockSet<float> B32[rh::kMaxBlockLevels];
  rh::BlockSet<double> B64[rh::kMaxBlockLevels];
  int* bstart[rh::kMaxBlockLevels];               // device: box corners (3 ints per box)
  std::vector<int> bcolour[rh::kMaxBlockLevels];  // colour c: boxes [off[c], off[c+1])
  int* src_count;                      // device: source cells per scan range
  int* src_offset;                     // device: their exclusive prefix sums
  int* src_list;                       // device: source cells in cell order
  int src_groups = 0;
  long long src_chunk = 0;
  int nsrc = 0;                        // source cells of the current step
  double *cA, *cInv;
  float* cInv32;
  double* cInv64;
  double* hred;      // pinned host memory the reductions' second pass writes
  double* hred_dev;  // its device address
  hipEvent_t ev0, ev1;
  // optional per-launch timing (event pairs on the handle's stream)
  static constexpr int kPool = 2048;
  bool timing = false;
  int npool = 0;
  hipEvent_t eva[kPool], evb[kPool];
  int pkind[kPool];
  double kms[KK_COUNT] = {};
  long long kcount[KK_COUNT] = {};
  std::string err;
  // per-phase GPU time of a step: an event is recorded on the stream where
  // the step enters another phase; after each stream synchronisation the
  // completed intervals are folded into pms[phase] (contiguous intervals, so
  // the phases partition the step's GPU time)
  static constexpr int kPhaseEv = 64;
  hipEvent_t pev[kPhaseEv];
  int pph[kPhaseEv];
  int npev = 0, cur_phase = -1;
  bool phases_on = false, phase_events = false;
  double pms[8] = {};
  // profiler range (ROCTx) of the current phase, open while a step runs
  bool mark_on = false;
  int mark_phase = 0;
  roctx_range_id_t mark_id = 0;
  // statistics of the current call
  int lin_its, local_its_max, lin_cap_hits, lin_its_max;
  double last_E_s = 1.0;  // E_s of the last step set up (weight of E in the norms)
  // conjugate-gradient dot products requested from the V-cycle's last sweep
  rh::SweepDots dots{};
  bool dots_wanted = false, dots_done = false;
  double lin_res_max;
  // the coarse operators and box inverses are current (a multigroup step
  // solves each group's system several times per Newton iteration)
  bool keep_coarse = false;
};

namespace rh {

// A named profiler range (ROCTx) over a scope, shown by a marker trace of a
// profiler; with no profiler attached a call costs one indirect branch.
struct MarkerRange {
  roctx_range_id_t id;
  explicit MarkerRange(const char* name) : id(roctxRangeStartA(name)) {}
  ~MarkerRange() { roctxRangeStop(id); }
  MarkerRange(const MarkerRange&) = delete;
  MarkerRange& operator=(const MarkerRange&) = delete;
};

// Per-launch timing: fold the completed event pairs of h into its totals.
void flush_timing(rh_handle* h);

// Brackets one launch on h's stream with an event pair when timing is on.
struct Timed {
  rh_handle* h;
  int slot = -1;
  Timed(rh_handle* hh, int kind) : h(hh) {
    if (!h->timing) return;
    if (h->npool == rh_handle::kPool) {
      (void)hipStreamSynchronize(h->stream);
      flush_timing(h);
    }
    slot = h->npool++;
    h->pkind[slot] = kind;
    (void)hipEventRecord(h->eva[slot], h->stream);
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(h->evb[slot], h->stream);
  }
  Timed(const Timed&) = delete;
  Timed& operator=(const Timed&) = delete;
};

// The per-step scalars of a step on handle h (its grey constants).
StepK handle_step(const rh_handle* h, double t_n, double dt);
// Face coefficients, constant part of f_E and E_s of a step from U^n (the
// handle's copy unless En / nn are given; y1n, y2n: helium of a multigroup
// step), the coarse face coefficients and the source boxes.
rh_status handle_setup_step(rh_handle* h, StepK& k, const double* src, const double* En,
                            const double* nn, const double* y1n, const double* y2n);
// Finalize the reduction slots in mask into h->hred and synchronise the stream.
rh_status handle_reductions(rh_handle* h, unsigned mask);
// Linear solve of the handle's Schur system for the right-hand side h->rS
// with the configured outer iteration and V-cycles (see solve_linear).
rh_status handle_solve(rh_handle* h, const StepK& k, double rmax0, double target_w,
                       double target_2, int max_it, double** x, int* its, double* w, double* l2,
                       bool* reached);
// Unknowns per cell of the grey norm (2 isothermal, else 3).
double handle_nvars(const rh_handle* h);

}  // namespace rh
