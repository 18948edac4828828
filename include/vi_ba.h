/*
 * vi_ba.h - C ABI of the MI355X (gfx950) visual-inertial bundle-adjustment step.
 *
 * The library computes one damped Gauss-Newton (fixed-damping Levenberg-
 * Marquardt) step, or a fixed number of them, of the joint visual-inertial
 * problem of VIGS-SLAM, Sec. 3.1: keyframe poses, per-pixel inverse depths,
 * velocities and gyro/accel biases minimise the sum of the vision energy of
 * Eq. 1 and the inertial energy of Eq. 2-3; the normal equations are reduced
 * by eliminating the (diagonal) inverse-depth block as in Eq. 4 and the
 * reduced pose/velocity/bias system is solved by an FP64 Cholesky.  IMU
 * measurements between consecutive keyframes are preintegrated first
 * (Sec. 3.1, "Inertial Residual").
 *
 * Conventions used throughout:
 *   - pose of keyframe i: world-from-body (R_i, p_i), stored as 7 doubles
 *     (px, py, pz, qx, qy, qz, qw), unit quaternion, Hamilton product;
 *   - the camera frame equals the body frame (identity extrinsics);
 *   - per-keyframe tangent (15): (dtheta, dp, dv, db_g, db_a) with the
 *     right perturbation R <- R Exp(dtheta) and additive world-frame p, v and
 *     additive biases; bias = (b_g, b_a);
 *   - edge (i, j): pixels of source keyframe i, whose inverse depth the edge
 *     uses, are projected into target keyframe j.  Pixel (x, y) is (column,
 *     row) at integer coordinates;
 *   - vision cost of a pixel: w_x r_x^2 + w_y r_y^2 with r = target - projection
 *     (weights are information); a pixel-residual counts only when its inverse
 *     depth is positive and the point lies more than z_min in front of camera j;
 *   - inertial factor (i, i+1) uses the bias of keyframe i; its velocity term
 *     uses the full 6-vector bias; information = blkdiag(cov, diag(cov_bias))^-1;
 *   - cost F = sum_vision w r^2 + sum_imu r^T Lambda r (no 1/2 factor);
 *   - damping: B_rr += lm_lambda * B_rr on every solved pose/velocity/bias
 *     coordinate and C += depth_eta, before elimination, so the step is the
 *     exact solution of the damped full system; 0/0 gives pure Gauss-Newton;
 *   - gauge: the pose coordinates of keyframes 0..n_fixed-1 are not solved.
 *
 * Memory: every array is owned by the caller.  Pointers documented "device"
 * are HIP device pointers on the context's device; "host" pointers are read
 * during the call only.  The library never frees caller memory.  The context
 * owns only its stream handle, index tables uploaded from host inputs, captured
 * graphs and a few bytes of status memory.
 *
 * Errors: every function returns a vi_status and never aborts.  On error the
 * caller's state arrays are unchanged by the failing step (increments are
 * committed only by the last kernel of a step, which is skipped when an earlier
 * kernel raised an error), and vi_last_error() describes the failure.
 * A context must not be used from two threads at once.
 */
#ifndef VI_BA_H
#define VI_BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VI_OK = 0,
  VI_EINVAL = -1,        /* bad argument (checked on the host before any launch) */
  VI_ENOMEM = -2,        /* workspace too small or device allocation failed */
  VI_EDEVICE = -3,       /* HIP runtime error */
  VI_ENOTPD = -4,        /* reduced system not positive definite (pivot <= 0) */
  VI_ENONFINITE = -5,    /* non-finite value in the assembled system or in an inverse depth */
  VI_EUNSUPPORTED = -6   /* option combination not implemented */
} vi_status;

typedef struct vi_ctx vi_ctx;

/* Create a context bound to HIP device `device` and stream `stream` (a
 * hipStream_t, or NULL for the null stream).  Writes the handle to *out. */
vi_status vi_ctx_create(int32_t device, void* stream, vi_ctx** out);
/* Destroy a context (waits for its stream).  NULL is accepted. */
void vi_ctx_destroy(vi_ctx* ctx);
/* Change the stream later calls enqueue on. */
vi_status vi_ctx_set_stream(vi_ctx* ctx, void* stream);
/* Message describing the last failing call on this context ("" if none). */
const char* vi_last_error(const vi_ctx* ctx);
/* Library version string. */
const char* vi_version(void);

typedef struct {
  double fx, fy, cx, cy;     /* pinhole intrinsics, pixels */
  int32_t H, W;              /* inverse-depth map rows and columns */
  double gravity[3];         /* world gravity vector g (Eq. 3), e.g. {0, 0, -9.81} */
  double T_bc[7];            /* camera-IMU extrinsic, body-from-camera (t, q xyzw): the state's poses are the
                                IMU body's (world-from-body), the camera of a keyframe is T_wb T_bc (Sec. 3.1,
                                inertial residual).  A zero quaternion reads as the identity (a zero-initialised
                                struct keeps the camera at the body); otherwise it is normalised.  Not used by
                                the pose-graph adjustment, whose poses are camera poses. */
} vi_camera;

typedef struct {
  double sigma_g;            /* gyro white-noise density, rad/s/sqrt(Hz) */
  double sigma_a;            /* accel white-noise density, m/s^2/sqrt(Hz) */
  double sigma_bgw;          /* gyro bias random walk, rad/s^2/sqrt(Hz) */
  double sigma_baw;          /* accel bias random walk, m/s^3/sqrt(Hz) */
} vi_imu_noise;

/* One preintegrated IMU factor (Sec. 3.1: "relative rotation, position and
 * velocity, their Jacobians and covariance").  154 doubles, row-major. */
typedef struct {
  double dt;                 /* Delta t_ij, seconds */
  double dR[9];              /* Delta R_ij */
  double dv[3];              /* Delta v_ij */
  double dp[3];              /* Delta p_ij */
  double J_rot[9];           /* d(Delta R)/d(b_g), right-perturbation form */
  double J_vel[18];          /* 3x6 d(Delta v)/d(b_g, b_a) */
  double J_pos[18];          /* 3x6 d(Delta p)/d(b_g, b_a) */
  double cov[81];            /* 9x9 covariance, order (rot, pos, vel) as in Eq. 3 */
  double bias_hat[6];        /* bias the factor was integrated at */
  double cov_bias[6];        /* bias random-walk variances over Delta t_ij */
} vi_preint;

/* Preintegrate IMU samples into n_factors factors (Sec. 3.1, following Forster
 * et al.; zero-order hold per sample: Delta R <- Delta R Exp((w - b_g) dt),
 * velocity and position by the constant-acceleration update, white-noise
 * covariance sigma^2/dt per sample).
 *   off      host   [n_factors+1]  CSR: factor f uses samples off[f]..off[f+1]-1;
 *                                  off[0] = 0, non-decreasing, >= 1 sample each
 *   gyro     device [S][3]  angular rate, rad/s, body frame
 *   accel    device [S][3]  specific force, m/s^2, body frame
 *   dt       device [S]     duration each sample is held, s (> 0)
 *   bias_hat device [n_factors][6] (b_g, b_a) linearisation point per factor
 *   out      device [n_factors]
 * Synchronous.  VI_EINVAL for a malformed CSR or a non-positive dt. */
vi_status imu_preintegrate(vi_ctx* ctx, int32_t n_factors, const int32_t* off,
                           const double* gyro, const double* accel, const double* dt,
                           const double* bias_hat, const vi_imu_noise* noise,
                           vi_preint* out);

/* Estimate, updated in place by a step. */
typedef struct {
  int32_t n_kf;              /* N >= 2 keyframes */
  double* pose;              /* device [N][7] (p, q xyzw) */
  double* vel;               /* device [N][3] world frame */
  double* bias;              /* device [N][6] (b_g, b_a) */
  void* invdepth;            /* device [N][H][W] inverse depth: float64, or float32 with vi_opts.invdepth_f32 */
} vi_state;

/* Frame graph: directed co-visible pairs and their correspondence targets
 * (Eq. 1: u*_ij and the confidence w_ij). */
typedef struct {
  int32_t n_edges;           /* E >= 1 */
  const int32_t* ii;         /* host [E] source keyframe (its inverse depth is used) */
  const int32_t* jj;         /* host [E] target keyframe, jj != ii, no duplicate pairs */
  const float* target;       /* device [E][2][H][W] target pixel x (plane 0), y (plane 1) */
  const float* weight;       /* device [E][2][H][W] weights >= 0, per coordinate */
} vi_edges;

/* Arithmetic of the step (vi_opts.precision).
 *  VI_PREC_FP64   every stage in FP64.
 *  VI_PREC_MIXED  per-pixel residuals and Jacobians (Eq. 1), the per-edge
 *                 J^T W J reductions and the Schur Gram of Eq. 4 in FP32 (FP32
 *                 MFMA; partial sums over 64-pixel blocks Kahan-compensated
 *                 across blocks, then handed over in FP64); C and w_d, the
 *                 inertial factors (Eq. 2-3), the reduced system, its Cholesky
 *                 solve, the depth update and the retraction in FP64; IMU
 *                 preintegration is always FP64. */
#define VI_PREC_FP64 0
#define VI_PREC_MIXED 1

/* How the IMU biases are solved (vi_opts.bias_mode; Table 6 (a) and (f)). */
#define VI_BIAS_PER_KF 0     /* one bias per keyframe, random walk between keyframes (Eq. 3) */
#define VI_BIAS_FIXED 1      /* the biases are not solved (kept at their input values) */
#define VI_BIAS_GLOBAL 2     /* one bias shared by every keyframe of the window */

typedef struct {
  int32_t n_fixed;           /* gauge: leading keyframes whose pose is held (>= 1 typical) */
  int32_t use_imu;           /* 0: vision only (velocity and bias are not solved) */
  int32_t bias_mode;         /* VI_BIAS_PER_KF, VI_BIAS_FIXED or VI_BIAS_GLOBAL */
  int32_t precision;         /* VI_PREC_FP64 or VI_PREC_MIXED */
  int32_t invdepth_f32;      /* 1: vi_state.invdepth of every window is float32 [N][H][W] (VI_PREC_MIXED only:
                                the maps are read and written in FP32, the depth update is formed in FP64 and
                                rounded once); 0: float64 */
  int32_t reserved;          /* must be 0 */
  double lm_lambda;          /* Marquardt factor on the pose/vel/bias diagonal (>= 0) */
  double depth_eta;          /* added to the inverse-depth diagonal C (>= 0) */
  double z_min;              /* minimum depth in the target camera, m */
  double d_min;              /* inverse depth is clamped to >= d_min after a step */
} vi_opts;

/* Stages reported by vi_report.stage_ms, in launch order:
 *  0 vision residual/Jacobian assembly fused with the Schur Gram, plus the
 *    inertial factors (one launch)
 *  1 per-source reduced blocks and cost reduction
 *  2 reduced-system assembly   3 Cholesky factor and solves
 *  4 back-substitution and retraction
 *  5 final cost evaluation */
#define VI_NUM_STAGES 6

typedef struct {
  double cost_before;        /* F at the input state of the (last) step */
  double cost_after;         /* F at the output state */
  int64_t n_valid;           /* valid pixel-residuals at the (last) linearisation point */
  int32_t iters_done;        /* steps applied */
  int32_t tile_px;           /* pixels per workgroup the assembly ran with (autotuned or default) */
  double* dxi;               /* optional device [N][15]: increments of the last step */
  double* dd;                /* optional device [N][H][W]: depth increments of the last step */
  double* costs;             /* optional host [iters+1]: F before each step, then final F */
  float* stage_ms;           /* optional host [VI_NUM_STAGES]: when set, the call runs without a
                                graph and returns the GPU time of each stage (HIP events on the
                                library's stream), summed over the steps */
} vi_report;

/* Device workspace (bytes) needed by vi_ba_step / vi_ba_solve for this shape. */
size_t vi_workspace_size(const vi_camera* cam, int32_t n_kf, const vi_edges* edges,
                         const vi_opts* opts);

/* One damped Gauss-Newton step (Eq. 4), in place on *state.
 *   imu        device [N-1] factors for pairs (i, i+1); may be NULL iff !use_imu
 *   workspace  device, >= vi_workspace_size() bytes, 256-byte aligned
 * Synchronous (the report is filled on return). */
vi_status vi_ba_step(vi_ctx* ctx, const vi_camera* cam, vi_state* state, const vi_edges* edges,
                     const vi_preint* imu, const vi_opts* opts, void* workspace,
                     size_t workspace_bytes, vi_report* report);

/* `iters` steps (Sec. 3.1: the local bundle adjustment iterates the LM step),
 * captured once per shape into a HIP graph and replayed.  On error at step t the
 * state holds the result of steps 0..t-1 and report->iters_done = t. */
vi_status vi_ba_solve(vi_ctx* ctx, const vi_camera* cam, vi_state* state, const vi_edges* edges,
                      const vi_preint* imu, const vi_opts* opts, int32_t iters,
                      void* workspace, size_t workspace_bytes, vi_report* report);

/* One independent window of a batch (the same step as vi_ba_solve, per window). */
typedef struct {
  vi_camera cam;             /* intrinsics and map size of this window */
  vi_state state;            /* device arrays, updated in place */
  vi_edges edges;            /* edges within this window (indices local to it) */
  const vi_preint* imu;      /* device [N-1]; may be NULL iff !use_imu */
  vi_report* report;         /* optional host report of this window */
} vi_window;

/* Device workspace (bytes) for vi_ba_solve_batched on these windows. */
size_t vi_workspace_size_batched(int32_t n_windows, const vi_window* windows, const vi_opts* opts);

/* `iters` steps on every window of a batch, all windows in the same launches
 * (one HIP graph per batch shape): each kernel of the step processes every
 * window's keyframes, edges, factors and reduced system.  Windows are
 * independent; a window whose reduced system fails (VI_ENOTPD, VI_ENONFINITE)
 * stops being updated while the others continue, and the first such error is
 * returned.  Per-window costs and counters go to windows[w].report.  When
 * windows[0].report->stage_ms is set the batch runs without a graph and the
 * stage times of the whole batch are returned there. */
vi_status vi_ba_solve_batched(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                              int32_t iters, void* workspace, size_t workspace_bytes);

/* Autotuning of the pixels-per-workgroup of the fused assembly.  When enabled,
 * the first call for a new batch shape times each candidate tiling on the
 * actual inputs (eagerly, before graph capture) and keeps the fastest for that
 * shape in the context; later calls reuse it.  Off by default (320 pixels). */
vi_status vi_ctx_set_autotune(vi_ctx* ctx, int32_t enable);

/* Tolerance stop of the Gauss-Newton iterations (Sec. 3.1 iterates the damped
 * step; the paper gives no stopping rule, so this one is the library's).  With
 * rel_tol > 0, every later vi_ba_solve, vi_ba_solve_batched and
 * vi_ba_solve_warm call on this context freezes a window before its step t
 * (t >= 1) when F_{t-1} - F_t <= rel_tol * F_{t-1}, F_t being the cost at the
 * state that step t would linearise (so also when the cost went up or is not
 * finite).  A frozen window takes no further step and its later assembly and
 * one-workgroup Cholesky work is skipped, while the other windows of a batch
 * go on; report->iters_done counts the steps applied, report->costs[t] stays
 * at the frozen value, report->cost_after is F at the state left behind.  The
 * same `iters` launches are made (one graph per shape and tolerance), so the
 * time saved is that of the skipped work.  0 (the default) never stops.
 * Errors: VI_EINVAL for a null context or rel_tol outside [0, 1). */
vi_status vi_ctx_set_tolerance(vi_ctx* ctx, double rel_tol);

/* ---------------------------------------------------------------------------
 * Learned warm start.  The paper's step has no learned initialisation; this
 * is an addition: a small convolutional network proposes inverse-depth and
 * bias corrections of a window before Gauss-Newton, and plain Gauss-Newton
 * remains the arbiter (a caller keeps the corrected state only if its cost is
 * lower than that of the plain initial state).
 *
 * Network (parameters: FP32 vector of vi_warm_param_count() floats, layout
 * W1 [32][15][3][3], b1 [32], W2..W4 [32][32][3][3] with b2..b4 [32],
 * Wd [1][32][3][3], bd [1], Wb [6][32], bb [6]): four 3x3 convolutions with 32
 * channels and ReLU over a keyframe's 15 input planes on a grid of 4 x 4-pixel
 * cells; a 3x3 convolution to one plane gives the per-cell inverse-depth
 * correction dd; the mean of the last layer over the cells, times Wb plus bb,
 * gives the keyframe's bias correction db (gyro, accel).  BF16 activations
 * and MFMA operands, FP32 accumulation, FP32 weights and optimiser state.
 *
 * Images: every keyframe of the given windows, window after window; all share
 * a canvas of hq x wq cells (hq <= 16, wq <= 24) and image k occupies its own
 * grid dims[k] = (ceil(H/4), ceil(W/4)) in the top-left corner. */
int32_t vi_warm_param_count(void);

/* Device workspace (bytes) of vi_warm_gradients for n_img images. */
size_t vi_warm_workspace_size(int32_t n_img, int32_t hq, int32_t wq);

/* Input planes of every keyframe at the windows' current state (device
 * feat [n_img][15][hq][wq] FP32, dims [n_img][2] int32):
 *   0, 1  confidence-weighted mean x / y residual (Eq. 1) over the cell's
 *         pixels and the keyframe's outgoing edges, px
 *   2     mean confidence of those pixel-residuals
 *   3     mean inverse depth of the cell
 *   4-12  inertial residual (Eq. 3) of the factor (i, i+1): rotation x 100,
 *         position x 10, velocity x 10 (zero for the last keyframe)
 *   13    depth-only Gauss-Newton step of the cell (poses held):
 *         -sum(w J_d r) / (h + 1e-6) / 0.2 with J_d = dr/dd (Eq. 1) and
 *         h = sum w J_d^2 over the cell's pixel-residuals
 *   14    log(1 + h / n_cell)
 * Synchronous. */
vi_status vi_warm_features(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                           int32_t hq, int32_t wq, float* feat, int32_t* dims);

/* Inference: dd [n_img][hq][wq] and db [n_img][6] (device FP32). */
vi_status vi_warm_forward(vi_ctx* ctx, int32_t n_img, int32_t hq, int32_t wq, const int32_t* dims,
                          const float* params, const float* feat, float* dd, float* db);

/* Training loss and its gradient (grads: device [vi_warm_param_count()]):
 *   L = sum_{img, valid cell} ((dd - label_dd) / 0.02)^2 / n_valid_cells
 *     + sum_img sum_6 ((db - label_db) / s_b)^2 / n_img,
 *   s_b = (0.005, 0.005, 0.005, 0.05, 0.05, 0.05);
 * label_dd [n_img][hq][wq], label_db [n_img][6] (device FP32); *loss on the
 * host.  Gradient partials are reduced over the images in a fixed order
 * (deterministic).  Synchronous. */
vi_status vi_warm_gradients(vi_ctx* ctx, int32_t n_img, int32_t hq, int32_t wq, const int32_t* dims,
                            const float* params, const float* feat, const float* label_dd, const float* label_db,
                            float n_valid_cells, void* workspace, size_t workspace_bytes, float* grads,
                            float* loss);

/* One AdamW step (t = 1, 2, ...; decoupled weight decay) on device params,
 * first and second moments m, v. */
vi_status vi_warm_adamw(vi_ctx* ctx, float* params, const float* grads, float* m, float* v, int32_t t, float lr,
                        float beta1, float beta2, float eps, float weight_decay);

/* Apply corrections in place: inverse depth d <- max(d + up(dd), opts->d_min),
 * up = bilinear upsampling of the keyframe's cell grid (cell centres at
 * 4 c + 1.5, clamped at the borders); bias b <- b + db when the step solves
 * the biases (opts->use_imu set and opts->bias_fixed clear), otherwise the
 * biases are left as they are. */
vi_status vi_warm_apply(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts, int32_t hq,
                        int32_t wq, const float* dd, const float* db);

/* Device workspace (bytes) of vi_warm_start for these windows: the solver's
 * workspace of the same batch followed by the warm start's buffers (input
 * planes, corrections, a copy of the inverse depths and biases).  0 on
 * invalid input. */
size_t vi_warm_start_workspace_size(int32_t n_windows, const vi_window* windows, const vi_opts* opts);

/* The whole warm start with plain Gauss-Newton as the arbiter, on the device in
 * one call: the cost F (Eq. 1 and 3 terms, as reported by vi_ba_solve) at the
 * windows' initial state; a copy of every inverse depth and bias; input
 * planes, network (params as for vi_warm_forward) and corrections as
 * vi_warm_features / vi_warm_forward / vi_warm_apply, on a canvas of the
 * largest cell grid of the windows (maps up to 64 x 96 pixels); F at the
 * corrected state; and every window whose corrected F is not below its
 * initial F (or is not finite) put back to its initial inverse depths and
 * biases.  Poses and velocities are never changed, nor are the biases when
 * opts leaves them unsolved (use_imu clear or bias_fixed set).  Per window:
 * accepted[w] (host, optional) = 1 if the corrections were kept; the
 * window's report (optional) gets cost_before = initial F, cost_after = F of
 * the state left behind, iters_done = 0, and costs[0..1] = the initial and
 * the corrected F (costs, when set, must hold 2 entries).  workspace: device,
 * 256-byte aligned, at least vi_warm_start_workspace_size bytes.
 * Synchronous.  Errors: VI_EINVAL (arguments, maps too large), VI_ENOMEM
 * (workspace too small), VI_EDEVICE. */
vi_status vi_warm_start(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                        const float* params, void* workspace, size_t workspace_bytes, int32_t* accepted);

/* vi_warm_start followed by iters (>= 0) Gauss-Newton steps, as one HIP
 * graph (captured on the first call of a shape and replayed after), so that
 * the warm start costs no extra host round trip.  Reports and errors as for
 * vi_ba_solve_batched over the steps that follow the warm start (iters = 0:
 * as vi_warm_start); accepted as for vi_warm_start.  workspace: at least
 * vi_warm_start_workspace_size bytes. */
vi_status vi_ba_solve_warm(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                           const float* params, int32_t iters, void* workspace, size_t workspace_bytes,
                           int32_t* accepted);


/* Initial state of new keyframes from IMU preintegration (Sec. 3.1, frontend
 * tracking: the pose of a new keyframe is initialised by preintegration,
 * falling back to the previous keyframe's pose when the trace of the factor's
 * covariance exceeds a threshold; the experiments use 1e-4).  For each of n
 * predictions k, with the state (R_i, p_i, v_i, b_i) of the previous keyframe
 * and the factor imu[k] preintegrated from it to the new keyframe:
 *   if tr(cov) + sum(cov_bias) <= tau (the trace of Sigma^iner):
 *     dR~ = dR Exp(J_rot (b_g - bh_g)), dv~ = dv + J_vel (b - bh), dp~ = dp + J_pos (b - bh)
 *     R_j = R_i dR~, v_j = v_i + g dt + R_i dv~, p_j = p_i + v_i dt + g dt^2 / 2 + R_i dp~, b_j = b_i
 *     (the state at which the inertial residual of Eq. 3 is zero), used_imu[k] = 1;
 *   otherwise (also when the trace is not a number): the new keyframe takes the
 *     previous keyframe's pose, velocity and bias, used_imu[k] = 0.
 *   pose_prev, vel_prev, bias_prev  device [n][7], [n][3], [n][6]
 *   imu                             device [n] factors from the previous keyframe to the new one
 *   gravity                         host [3], world frame (e.g. 0, 0, -9.81)
 *   tau                             threshold >= 0 (1e-4 in the paper's experiments)
 *   pose_new, vel_new, bias_new     device, same shapes; each equal to its input (in
 *                                   place) or not overlapping any input
 *   used_imu                        optional device [n] int32
 * Asynchronous on the context's stream.  VI_EINVAL for n < 0, null arrays, a
 * negative or NaN tau, or a partly overlapping output. */
vi_status vi_predict_keyframe(vi_ctx* ctx, int32_t n, const double* pose_prev, const double* vel_prev,
                              const double* bias_prev, const vi_preint* imu, const double* gravity, double tau,
                              double* pose_new, double* vel_new, double* bias_new, int32_t* used_imu);

/* ---------------------------------------------------------------------------
 * IMU initialisation, stage 2: inertial-only optimisation (Sec. 3.2, "Stage 2:
 * Inertial-Only Optimization", and the IMU-initialisation paragraph of the
 * implementation details).  The visual poses (R_i, p_i^vis) of the first
 * keyframes, known up to scale, are held fixed; positions and velocities are
 * e^s p_i^vis and e^s v_i^vis with a global log-scale s, gravity is
 * g = R_wg (0, 0, G), and R_wg, s, every v_i^vis and every bias b_i minimise
 * the inertial energy (Eq. 2, residuals as in Eq. 3 with these substitutions,
 * information as for the step).  R_wg is perturbed on the right about the
 * first two axes of the gravity frame (a turn about gravity is not
 * observable); damping as for the step (H_rr += lm_lambda H_rr on all 3 + 9N
 * unknowns); a fixed number of Gauss-Newton iterations. */
typedef struct {
  int32_t n_kf;              /* 2 <= N <= 32 keyframes */
  const double* pose_vis;    /* device [N][7] visual poses (p^vis, q xyzw), fixed */
  const vi_preint* imu;      /* device [N-1] factors (i, i+1) */
  double* vel_vis;           /* device [N][3] velocities in the visual scale: initial guess in, estimate out */
  double* bias;              /* device [N][6] (b_g, b_a): in / out */
  double* rot_wg;            /* device [4] quaternion (x, y, z, w) of R_wg: in / out */
  double* log_scale;         /* device [1] s: in / out */
  double* cost;              /* optional device [iters + 1]: cost before each iteration and at the end */
} vi_inertial_init;

/* Device workspace (bytes) of vi_inertial_init_solve for these problems; 0 on
 * invalid input. */
size_t vi_inertial_init_workspace_size(int32_t n_problems, const vi_inertial_init* problems);

/* `iters` (>= 0) iterations on every problem (host array of n_problems
 * descriptors), one workgroup per problem in one launch.  gravity_z: G of
 * g_I = (0, 0, G) (e.g. -9.81).  Synchronous.  Errors: VI_EINVAL (arguments),
 * VI_ENOMEM (workspace too small), VI_ENOTPD (a non-positive-definite factor
 * covariance or normal matrix), VI_ENONFINITE (non-finite cost); on error the
 * state of the failing problem is left as it was. */
vi_status vi_inertial_init_solve(vi_ctx* ctx, int32_t n_problems, const vi_inertial_init* problems,
                                 double gravity_z, double lm_lambda, int32_t iters, void* workspace,
                                 size_t workspace_bytes);

/* ---------------------------------------------------------------------------
 * Loop-closure update of a Gaussian map (Sec. 3.3, "Loop Closure Gaussian
 * Update", Eq. 7-8).  After pose-graph bundle adjustment each keyframe k has
 * its pose before (R-, t-) and after (R+, t+) the correction and a scale
 * change ds_k.  A Gaussian created from keyframe k gets
 *   mean  <- R+ (ds_k (R-)^T (mean - t-)) + t+              (Eq. 7)
 *   Sigma <- R+ (ds_k^2 (R-)^T Sigma R-) (R+)^T              (Eq. 8)
 * and keeps its opacity and colour (not touched here).  Poses are camera-to-
 * world (t, q xyzw) as 7 doubles, the quaternion normalised before use.  The
 * update is evaluated as the per-keyframe similarity x -> A x + b with
 * A = ds_k R+ (R-)^T and b = t+ - A t-, folded in FP64 and applied in FP32. */
typedef struct {
  int64_t n;                 /* number of Gaussians K >= 0 */
  const int32_t* anchor;     /* device [K]: keyframe each Gaussian was created from */
  const float* mean_in;      /* device [K][3] world-frame means */
  const float* cov_in;       /* device [K][6] (xx, xy, xz, yy, yz, zz), or NULL: means only */
  float* mean_out;           /* device [K][3]; equal to mean_in (in place) or not overlapping it */
  float* cov_out;            /* device [K][6]; NULL iff cov_in is NULL; in place or disjoint */
} vi_gaussians;

/* Device workspace (bytes) of vi_gaussian_reanchor for n_kf keyframes (48 per
 * keyframe, rounded up to 256). */
size_t vi_reanchor_workspace_size(int32_t n_kf);

/* Apply Eq. 7-8 to every Gaussian of *g.
 *   pose_pre, pose_post  device [n_kf][7] poses before / after the correction
 *   scale_change         device [n_kf] ds_k
 *   workspace            device, 16-byte aligned, >= vi_reanchor_workspace_size(n_kf)
 *   n_rejected           optional device int32: set to the number of Gaussians left
 *                        unchanged (copied to the outputs as they are) because their
 *                        anchor is outside 0..n_kf-1 or their keyframe's update is not
 *                        valid (ds_k not positive and finite, a pose not finite, a zero
 *                        quaternion)
 * Asynchronous on the context's stream; the workspace and outputs must not be
 * reused before the stream reaches this work.  Vector (16-byte) memory access
 * is used when all arrays are 16-byte aligned, element access otherwise.
 * Errors (host checks, nothing launched): VI_EINVAL (n_kf < 1, K < 0, null
 * arrays, cov_in / cov_out not both given, an output that partly overlaps its
 * input), VI_ENOMEM (workspace too small), VI_EDEVICE. */
vi_status vi_gaussian_reanchor(vi_ctx* ctx, int32_t n_kf, const double* pose_pre, const double* pose_post,
                               const double* scale_change, const vi_gaussians* g, void* workspace,
                               size_t workspace_bytes, int32_t* n_rejected);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid it): vi_gaussian_reanchor
 * without a workspace.  The per-keyframe table lives in a fixed device array
 * of the library (48 B per keyframe, at most 16384 keyframes = 768 KiB per
 * GPU, held until the process ends); the call allocates nothing.  Same
 * arguments, results, stream semantics and errors as vi_gaussian_reanchor,
 * plus VI_EINVAL when n_kf exceeds 16384.  All calls on one GPU share that
 * array: calls that can overlap on the same GPU (different streams or
 * contexts without ordering between them) race and must not be issued;
 * calls on one context's stream run in order and are safe. */
vi_status vi_gaussian_reanchor_noalloc(vi_ctx* ctx, int32_t n_kf, const double* pose_pre, const double* pose_post,
                                       const double* scale_change, const vi_gaussians* g, int32_t* n_rejected);

/* ---------------------------------------------------------------------------
 * Loop closure: pose-graph bundle adjustment in Sim(3) (Sec. 3.1, "Loop
 * Closure: Pose Graph Bundle Adjustment", Eq. 5).  Minimises the vision
 * energy of Eq. 1 over the loop pairs E* plus relative-pose terms over the
 * pose graph E+,
 *   sum_{E*} sum_u w_x r_x^2 + w_y r_y^2 + sum_{E+} r_ij^T Lambda_ij r_ij,
 *   r_ij = Log(T~_ij E_ij^-1),  E_ij = T_j^-1 T_i,
 * over the keyframes' similarities T_i = (s_i, R_i, p_i) (camera to world,
 * X_w = s_i R_i X_c + p_i; E_ij takes camera i coordinates to camera j
 * coordinates, so the vision term of pair (i, j) reads X_j = E_ij X_i) and
 * the inverse depths of the loop pairs' source keyframes.  The paper writes
 * the same residual with world-to-camera poses, log(T~_ij T_i T_j^-1).
 * Sim(3) tangent vectors are ordered (rotation phi, translation rho,
 * log-scale sigma), the Lie-algebra matrix being [[sigma I + [phi]x, rho],
 * [0, 0]].  7 unknowns per keyframe: R <- R Exp(dtheta), p <- p + dp,
 * s <- s exp(dsigma); inverse depths as for the step (d <- max(d + dd,
 * d_min)).  Damping as for the step (lm_lambda on the pose diagonal,
 * depth_eta on C); the first opts->n_fixed keyframes are held entirely (the
 * seven gauge freedoms of Sim(3) with n_fixed = 1).  opts->use_imu and
 * opts->bias_fixed are ignored; opts->precision selects FP64 or FP32 vision
 * assembly as for the step (the reduced system and its Cholesky are FP64).
 * --------------------------------------------------------------------------- */
typedef struct {
  int32_t n_rel;             /* relative-pose factors (edges of E+) */
  const int32_t* ii;         /* host [n_rel] keyframe i */
  const int32_t* jj;         /* host [n_rel] keyframe j (!= i) */
  const double* meas;        /* device [n_rel][8]: measured E_ij = T_j^-1 T_i as t (3), q (x y z w), s > 0 */
  const double* info;        /* device [n_rel][49]: Lambda_ij = (Sigma^rel_ij)^-1, row-major, symmetric
                                positive semi-definite, (rotation, translation, log-scale) order */
} vi_rel_poses;

/* Device workspace (bytes) of vi_pgba_solve for this problem shape (0 on
 * invalid input). */
size_t vi_pgba_workspace_size(const vi_camera* cam, int32_t n_kf, const vi_edges* loops, const vi_rel_poses* rel,
                              const vi_opts* opts);

/* iters damped Gauss-Newton steps in place.
 *   cam                  intrinsics and map size (gravity unused)
 *   pose                 device [n_kf][7] (p, q x y z w), in / out
 *   scale                device [n_kf] s > 0, in / out
 *   invdepth             device [n_kf][H][W] FP64, in / out (only the loop
 *                        pairs' sources change)
 *   loops                loop pairs E* (ii, jj host; target, weight device
 *                        [E*][2][H][W] FP32, as vi_edges), at least one pair,
 *                        at most 18 per source keyframe
 *   rel                  pose-graph edges E+ (n_rel >= 0)
 *   report               optional: costs before each step and final,
 *                        n_valid, iters_done; dxi (device [n_kf][7]) and dd
 *                        (device [n_kf][H][W]) of the last step when set
 * Synchronous.  Errors as vi_ba_solve (VI_EINVAL on host checks, VI_ENOTPD,
 * VI_ENONFINITE, VI_EDEVICE); on error the failing step leaves the state as
 * it was.  The tolerance stop of vi_ctx_set_tolerance applies. */
vi_status vi_pgba_solve(vi_ctx* ctx, const vi_camera* cam, int32_t n_kf, double* pose, double* scale,
                        double* invdepth, const vi_edges* loops, const vi_rel_poses* rel, const vi_opts* opts,
                        int32_t iters, void* workspace, size_t workspace_bytes, vi_report* report);

#ifdef __cplusplus
}
#endif

#endif /* VI_BA_H */
