// Internal structures of the visual-inertial step library: the per-shape plan
// (index tables built on the host from the frame graph), the workspace carve,
// and the kernel launchers shared by the translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vi_ba.h"

namespace vi {

constexpr int kMaxOutDegree = 18;     // per-source outgoing edges (Gram tile budget)
constexpr int kVisBlock = 256;        // pixels per assembly workgroup
constexpr int kGramChunk = 64;        // pixels staged per Gram MFMA pass
constexpr int kGramRange = 320;       // pixels per Gram workgroup
constexpr int kCholNB = 64;           // Cholesky block size
constexpr int kMaxIters = 64;         // cost trace capacity of vi_ba_solve

// Device status word: first error (vi_status), its detail (e.g. pivot index),
// and the number of committed steps.
struct DevStatus {
  int code;
  int detail;
  int iters;
  int pad;
};

// Host-built description of one frame-graph shape.
struct Plan {
  int N = 0, E = 0, H = 0, W = 0, HW = 0;
  int F = 0;                     // IMU factors (N - 1)
  int n = 0;                     // reduced dimension 15 N
  int npad = 0;                  // n rounded up to kCholNB
  int nblk = 0;                  // npad / kCholNB
  int nkr_vis = 0;               // pixel ranges per source in the assembly
  int nkr_gram = 0;              // pixel ranges per source in the Gram
  int kmax = 0;
  size_t n_pairs = 0;            // gather items of the reduced assembly
  // host copies
  std::vector<int32_t> ii, jj, src_off, src_edges, edge_slot;
  std::vector<int32_t> gram_off, q_off, z_off, zb_off, tiles;
  std::vector<int32_t> pair_off, pair_z, pair_zb;
  // sizes (doubles)
  size_t L_size = 0, gram_size = 0, q_size = 0, z_size = 0, zb_size = 0;
};

// Device pointers into the plan upload (int32 tables).
struct DevPlan {
  const int32_t *ii, *jj, *src_off, *src_edges, *edge_slot;
  const int32_t *gram_off, *q_off, *z_off, *zb_off, *tiles;
  const int32_t *pair_off, *pair_z, *pair_zb;
};

// Workspace carve (device pointers into the caller's workspace).
struct Work {
  double* Rw;        // [N][9]
  double* rel;       // [E][12]  R_ji (9), t_ji (3)
  double* L;         // per source [HW][6 k_i]   E-block in local edge coordinates
  double* Cd;        // [N][HW]  C + eta
  double* wd;        // [N][HW]
  double* hpart;     // [E][nkr_vis][32]
  double* vcost;     // [N * nkr_vis][2]  vision cost / valid count partials
  double* gpart;     // Gram partials
  double* Z;         // per source (k+1)^2 * 36
  double* ZB;        // per source 6 (k+1)
  double* ZV;        // per source 6 (k+1)
  double* Lam;       // [F][225]
  double* Hf;        // [F][900]
  double* gf;        // [F][30]
  double* icost;     // [F]
  double* A;         // [(npad + NB) * npad]  reduced matrix (+ augmented rhs row)
  double* Linv;      // [nblk][NB*NB]
  double* x;         // [npad]
  double* dd;        // [N][HW]
  double* trace;     // [kMaxIters + 1][2]  cost, n_valid
};

size_t workspace_bytes(const Plan& P);
Work carve_workspace(const Plan& P, void* base);

struct OptsDev {
  int n_fixed, use_imu, bias_fixed;
  double lambda, eta, z_min, d_min;
};

struct CamDev {
  double fx, fy, cx, cy;
  int H, W;
  double g[3];
};

// kernel launchers (enqueue on `s`)
void launch_preint(hipStream_t s, int F, const int32_t* off, const double* gyro,
                   const double* accel, const double* dt, const double* bias_hat,
                   vi_imu_noise noise, vi_preint* out, DevStatus* st);
void launch_imu_info(hipStream_t s, int F, const vi_preint* imu, double* Lam, DevStatus* st);
// Stages of one step, for per-stage event timing.
enum Stage { kStVis = 0, kStGram, kStLocal, kStAssemble, kStChol, kStBacksub, kNumStages };
// `marks`, when non-null, is called between stages (used to record timing events).
typedef void (*StageMark)(void* user, int stage_done);
void launch_step(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const CamDev& cam,
                 const OptsDev& o, const vi_state& x, const float* target, const float* weight,
                 const vi_preint* imu, int iter, double* rep_dxi, double* rep_dd, DevStatus* st,
                 StageMark mark = nullptr, void* mark_user = nullptr);
void launch_reset_status(hipStream_t s, DevStatus* st);
size_t step_lds_max(int kmax);
void step_set_attributes(int kmax);
void launch_final_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w,
                       const CamDev& cam, const OptsDev& o, const vi_state& x, const float* target,
                       const float* weight, const vi_preint* imu, int slot, DevStatus* st);

}  // namespace vi
