// Internal structures of the visual-inertial step library: the per-batch plan
// (index tables built on the host from the windows' frame graphs), the
// per-window device descriptors, the workspace carve, and the kernel launchers
// shared by the translation units.
//
// A call solves a batch of independent windows (a single-window call is a
// batch of one).  Keyframes, edges and IMU factors of all windows are numbered
// globally (window after window); per-window quantities (map size, intrinsics,
// the caller's arrays, the reduced system) are reached through the window
// descriptor of the keyframe, edge or factor.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vi_ba.h"

namespace vi {

constexpr int kMaxOutDegree = 18;     // per-source outgoing edges (Gram tile budget)
constexpr int kVisBlock = 256;        // pixels per workgroup of the per-pixel kernels
constexpr int kCholNB = 32;           // Cholesky tile size
constexpr int kCholSmallMaxNpad = 512;  // systems up to this size are solved by one workgroup
constexpr int kPairTicketFlag = 1 << 30;  // Cholesky ticket of tile (j + 1, j) that also factors tile (j + 1, j + 1)
constexpr int kMaxIters = 64;         // cost trace capacity of vi_ba_solve
constexpr int kMaxKeyframes = 640;    // per window: the back-substitution keeps 2 x 15 N doubles in LDS
constexpr int kTraceLen = 2 * (kMaxIters + 1);

// Device status word of one window: first error (vi_status), its detail (e.g.
// pivot index), and the number of committed steps.
struct DevStatus {
  int code;
  int detail;
  int iters;
  int conv;          // 1 once the tolerance stop has frozen the window
};

// Per-window device descriptor.
struct WinDev {
  double fx, fy, cx, cy, g[3];
  double Rbc[9], tbc[3];             // camera-IMU extrinsic (body-from-camera), row-major rotation
  int ext;                           // 1: T_bc is not the identity (vision terms go through it)
  int H, W, HW, N;
  int kf_base, e_base, f_base, F;    // global index of the first keyframe / edge / factor
  int nkr;                           // pixel ranges per source in the fused assembly + Gram
  int n, npad, nblk;                 // reduced system
  int pair_base;                     // offset of this window's pair table
  int flag_off, nflags;              // Cholesky tile flags [(nblk + 1) * nblk]
  int band;                          // tiles (i, j) with i - j > band are zero in S and in L
  int fc_off;                        // offset of the tile envelope (nblk + 1 entries) in chol_fc
  long long pix_base;                // global offset of the first keyframe's first pixel
  long long A_off, Linv_off, x_off;  // reduced system, diagonal-tile inverses, solution
  double* pose;
  double* vel;
  double* bias;
  double* invdepth;                  // FP64 inverse depths, or null when they are FP32:
  float* invdepth32;                 // FP32 inverse depths (mixed precision), or null
  const float* target;
  const float* weight;
  const vi_preint* imu;
  double* rep_dxi;
  double* rep_dd;
  // pose-graph adjustment in Sim(3) (null / 0 for the visual-inertial step)
  double* scale;                     // [N] keyframe scales s (X_w = s R X_c + p), updated in place
  const double* rel_meas;            // [n_rel][8] measured E_ij = T_j^-1 T_i: t (3), q (4), s
  const double* rel_info;            // [n_rel][49] information, (rotation, translation, log-scale) order
  int rel_base, n_rel;               // global index of the window's first relative-pose factor
};

// Host-built description of one batch.
struct Plan {
  int n_win = 0;
  int N = 0, E = 0, F = 0;       // totals over the batch
  int kmax = 0;
  int nkr_max = 0;               // max pixel ranges per source
  int hw_max = 0;
  int nblk_max = 0;
  int range = 320;               // pixels per workgroup of the fused kernel
  long long pix_total = 0;       // sum over keyframes of H*W
  std::vector<WinDev> win;       // pointers filled per call
  // host tables
  std::vector<int32_t> ii, jj;                 // global keyframe indices per global edge
  std::vector<int32_t> win_of_kf, win_of_f;
  std::vector<int32_t> src_off, src_edges;     // CSR of edges by source keyframe
  std::vector<int32_t> gram_off, z_off, zb_off;
  std::vector<int32_t> pair_off, pair_z, pair_zb;
  std::vector<int32_t> chol_tiles;             // ticket -> (window, (i << 16) | j)
  // keyframe order of each window's reduced system: keyframe a (local) has
  // its unknowns at block position kf_pos[kf_base + a]; kf_at is the inverse
  std::vector<int32_t> kf_pos, kf_at;
  // per window, first nonzero tile column of every tile row of S and L (the
  // right-hand-side row last, 0): tiles (i, j < fc[i]) are zero in both
  std::vector<int32_t> chol_fc;
  int pdim = 15;                               // unknowns per keyframe: 15 (visual-inertial) or 7 (Sim(3) graph)
  int R = 0;                                   // relative-pose factors (pose-graph adjustment)
  std::vector<int32_t> rel_ii, rel_jj;         // global keyframe indices per factor
  std::vector<int32_t> rel_z, rel_zb;          // offsets of each factor's four 7x7 blocks in Z and its 14 in ZB/ZV
  int n_tickets = 0;
  int n_bs = 0;                                // back-substitution columns after the tiles in chol_tiles
  size_t flags_size = 0;
  size_t gram_size = 0, z_size = 0, zb_size = 0;
  size_t A_size = 0, Linv_size = 0, x_size = 0;
};

// Device pointers into the plan upload.
struct DevPlan {
  const int32_t *ii, *jj, *win_of_kf, *win_of_f, *src_off, *src_edges;
  const int32_t *gram_off, *z_off, *zb_off;
  const int32_t *pair_off, *pair_z, *pair_zb;
  const int32_t* chol_tiles;
  const int32_t *rel_ii, *rel_jj, *rel_z, *rel_zb;
  const int32_t *kf_pos, *kf_at, *chol_fc;
  const WinDev* win;
};

// Workspace carve (device pointers into the caller's workspace).
struct Work {
  double* Rw;        // [N][9]
  double* rel;       // [E][12]  R_ji (9), t_ji (3)
  double* Cd;        // [pix_total]  C + eta
  double* wd;        // [pix_total]
  double* hpart;     // [E][nkr_max][32]
  double* vcost;     // [N][ncost][2]  vision cost / valid count partials
  double* gpart;     // Gram partials
  double* Z;         // per source (k+1)^2 * 36
  double* ZB;        // per source 6 (k+1)
  double* ZV;        // per source 6 (k+1)
  double* Lam;       // [F][225]
  double* Hf;        // [F][900]
  double* gf;        // [F][30]
  double* icost;     // [F]
  double* A;         // per window [(npad + NB) * npad]  reduced matrix (+ augmented rhs row)
  int32_t* flags;    // Cholesky tile flags of all windows
  int32_t* sync;     // [0] ticket counter, [1] abort flag
  double* Linv;      // per window [nblk][NB*NB]
  double* x;         // per window [npad]
  double* trace;     // [n_win][kTraceLen]  cost, n_valid per slot
  double* rcost;     // [R]  relative-pose factor costs (pose-graph adjustment)
};

struct OptsDev {
  int n_fixed, use_imu, bias_fixed, precision;
  double lambda, eta, z_min, d_min;
  double tol;        // relative cost decrease below which a window stops (0: never)
  int bias_global;   // one bias per window, in the last keyframe's slot (with use_imu)
};

// learned warm-start network (k_wnet.hip)
constexpr int kWCin = 15, kWCinPad = 16, kWC = 32, kWLayers = 4;
constexpr int kWParams = kWC * kWCin * 9 + kWC + 3 * (kWC * kWC * 9 + kWC) + kWC * 9 + 1 + 6 * kWC + 6;
constexpr int kWHQMax = 16, kWWQMax = 24;       // canvas of 4x4-pixel cells (maps up to 64 x 96)
constexpr float kWSd = 0.02f;                   // inverse-depth correction scale of the loss

// partial-sum slots per source in the cost / Hessian partial arrays
inline int cost_slots(const Plan& P) {
  return std::max(P.nkr_max, (P.hw_max + kVisBlock - 1) / kVisBlock);
}

// kernel launchers (enqueue on `s`)
void launch_preint(hipStream_t s, int F, const int32_t* off, const double* gyro,
                   const double* accel, const double* dt, const double* bias_hat,
                   vi_imu_noise noise, vi_preint* out, DevStatus* st);
void launch_imu_info(hipStream_t s, const Plan& P, const DevPlan& D, double* Lam, DevStatus* st);
void launch_predict_kf(hipStream_t s, int n, const double* pose_i, const double* vel_i, const double* bias_i,
                       const vi_preint* imu, const double* g, double tau, double* pose_j, double* vel_j,
                       double* bias_j, int32_t* used);
// Stages of one step, for per-stage event timing.
enum Stage { kStVis = 0, kStLocal, kStAssemble, kStChol, kStBacksub, kNumStages };
// `mark`, when non-null, is called between stages (used to record timing events).
typedef void (*StageMark)(void* user, int stage_done);
void launch_step(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o, int iter,
                 DevStatus* st, StageMark mark = nullptr, void* mark_user = nullptr);
// the first two stages only (autotuning of the assembly tiling)
void launch_tune_stages(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                        StageMark mark, void* mark_user);
void launch_reset_status(hipStream_t s, DevStatus* st, int n);
// dd / db (optional): warm-start corrections (cells [n][HQ][WQ], [n][6]) applied
// to the state first, so that the cost is that of the corrected state
void launch_final_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                       int slot, double* trace = nullptr, const float* dd = nullptr, const float* db = nullptr,
                       int HQ = 0, int WQ = 0, double d_min = 0.0);   // trace: w.trace unless given
void launch_chol(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st);
// the fused vision assembly alone (no inertial workgroups) and the vision cost
// of the current state (vcost in ranges of kVisBlock pixels)
void launch_vis_assembly(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                         DevStatus* st);
void launch_vis_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o);
// pose-graph adjustment in Sim(3) (k_pgba.hip)
size_t pg_local_lds(int kmax);
void pg_set_attributes();
void launch_pg_local(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st);
void launch_pg_relpose(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st, bool jac);
void launch_pg_assemble(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, int n_fixed, double lambda,
                        DevStatus* st);
void launch_pg_backsub(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                       DevStatus* st);
void launch_pg_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, int ncost, int range_px,
                    int slot, double tol, DevStatus* st);
void step_set_attributes(int kmax);
// warm start
void wnet_set_attributes();
// wprep (optional device scratch of wnet_prep_bytes()): the layers' weights are
// converted to their LDS image once per call instead of once per image
void launch_wnet_forward(hipStream_t s, int n, int HQ, int WQ, const int* dims, const float* theta, const float* feat,
                         void* act, float* dd, float* db, void* wprep = nullptr);
size_t wnet_prep_bytes();
void launch_wnet_backward(hipStream_t s, int n, int HQ, int WQ, const int* dims, const float* theta, const void* act,
                          const float* dd, const float* db, const float* lab_dd, const float* lab_db, float nv,
                          float* g_dd, float* g_db, float* loss, float* partial, float* grads);
// inertial-only initialisation (k_iinit.hip): one descriptor per problem, in the workspace
struct IInitDesc {
  int N;
  int pad;
  const double* pose_vis;
  const vi_preint* imu;
  double* vel;
  double* bias;
  double* rot_wg;
  double* log_scale;
  double* cost;
  double* wf;            // whitening scratch [N-1][87]
};
constexpr int kIInitMaxKeyframes = 32;
size_t iinit_lds_bytes(int N);
size_t iinit_whiten_doubles(int N);
void launch_inertial_init(hipStream_t s, int n, const IInitDesc* descs, int max_n_kf, double G, double lambda,
                          int iters, DevStatus* status);

// loop-closure update of a Gaussian map (k_gauss.hip)
size_t reanchor_table_bytes(int n_kf);
// allocation-free variant: the keyframe table in a file-scope device array of
// k_gauss.hip.  reanchor_scratch_init (with `device` current) looks up that
// array's address on the device once; reanchor_scratch returns it (nullptr
// before a successful init).
int reanchor_noalloc_max_keyframes();
hipError_t reanchor_scratch_init(int device);
void* reanchor_scratch(int device);
int64_t reanchor_max_gaussians();
void launch_reanchor(hipStream_t s, int n_kf, const double* pose_pre, const double* pose_post, const double* ds,
                     void* table, int64_t K, const int32_t* anchor, const float* mean_in, const float* cov_in,
                     float* mean_out, float* cov_out, int* n_rej);

void launch_wnet_adamw(hipStream_t s, int P, float* theta, const float* g, float* m, float* v, int t, float lr,
                       float b1, float b2, float eps, float wd);
void launch_warm_features(hipStream_t s, const Plan& P, const DevPlan& D, const OptsDev& o, int HQ, int WQ,
                          float* feat, int* dims, double* saved_d = nullptr,
                          double* saved_b = nullptr);
void launch_warm_apply(hipStream_t s, const Plan& P, const DevPlan& D, int HQ, int WQ, const float* dd,
                       const float* db, double d_min, int apply_bias);
void launch_warm_state(hipStream_t s, const Plan& P, const DevPlan& D, double* saved_d, double* saved_b,
                       const double* trace, int restore);

}  // namespace vi
