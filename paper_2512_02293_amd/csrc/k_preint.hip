// IMU preintegration between consecutive keyframes (Sec. 3.1, "Inertial
// Residual": relative rotation, velocity and position, their bias Jacobians
// and covariance, following Forster et al.) and the per-factor information
// matrix used by the inertial residual of Eq. 2-3.
//
// One 192-thread workgroup per factor.  The sample loop is inherently serial;
// the threads share each sample's work in two phases: T = A cov (one entry per
// thread) beside the new mean and bias Jacobians, then the 45 lower-triangle
// entries of cov = T A^T + Q, using the block structure of the transition A of
// the (rot, vel, pos) error state.
#include "vi_internal.h"
#include "vi_math.h"

namespace vi {

namespace {

__device__ __forceinline__ void set_status(DevStatus* st, int code, int detail) {
  if (atomicCAS(&st->code, 0, code) == 0) st->detail = detail;
}

// row r of M1 = dR [a]x (column m of [a]x is a x e_m)
__device__ __forceinline__ void m1_row(const double* dR, const double* a, int r, double* m1) {
  const double d0 = dR[r * 3 + 0], d1 = dR[r * 3 + 1], d2 = dR[r * 3 + 2];
  m1[0] = d1 * a[2] - d2 * a[1];
  m1[1] = d2 * a[0] - d0 * a[2];
  m1[2] = d0 * a[1] - d1 * a[0];
}

// Three waves per factor: in phase 1 the 81 entries of T = A cov take one
// lane each (waves 0 and 1) while wave 2 updates the mean and the bias
// Jacobians; phase 2 and the per-sample precomputation run on wave 0.
constexpr int kPreintThreads = 192;

// LDS layout of one factor's running state
struct PreintLds {
  double dR[9], dv[3], dp[3], JR[9], Jvg[9], Jva[9], Jpg[9], Jpa[9];
  double nR[9], nv[3], np_[3], nJR[9], nJvg[9], nJva[9], nJpg[9], nJpa[9];
  double M1[9];                          // per-sample: dR [a]x
  double pdRk[64][9], pJrk[64][9], pa[64][3], ph[64];   // 64 samples: Exp(w h), Jr(w h), a, h
  double T[81], cov[81];
};

__global__ void __launch_bounds__(kPreintThreads) k_preint(int F, const int32_t* __restrict__ off,
                                               const double* __restrict__ gyro,
                                               const double* __restrict__ accel,
                                               const double* __restrict__ dt,
                                               const double* __restrict__ bias_hat,
                                               vi_imu_noise noise, vi_preint* __restrict__ out,
                                               DevStatus* st) {
  __shared__ PreintLds S;
  const int f = blockIdx.x;
  const int l = threadIdx.x;
  if (f >= F) return;
  const int s0 = off[f], s1 = off[f + 1];
  const double bg0 = bias_hat[f * 6 + 0], bg1 = bias_hat[f * 6 + 1], bg2 = bias_hat[f * 6 + 2];
  const double ba0 = bias_hat[f * 6 + 3], ba1 = bias_hat[f * 6 + 4], ba2 = bias_hat[f * 6 + 5];
  const double sg2 = noise.sigma_g * noise.sigma_g, sa2 = noise.sigma_a * noise.sigma_a;

  if (l < 9) {
    S.dR[l] = (l % 4 == 0) ? 1.0 : 0.0;
    S.JR[l] = 0.0; S.Jvg[l] = 0.0; S.Jva[l] = 0.0; S.Jpg[l] = 0.0; S.Jpa[l] = 0.0;
  }
  if (l < 3) { S.dv[l] = 0.0; S.dp[l] = 0.0; }
  for (int e = l; e < 81; e += kPreintThreads) S.cov[e] = 0.0;
  double total = 0.0;
  __syncthreads();

  for (int sb = s0; sb < s1; sb += 64) {
    // per-sample quantities that do not depend on the running state, one lane each
    const int nb = min(64, s1 - sb);
    if (l < nb) {
      const int s = sb + l;
      const double h = dt[s];
      if (!(h > 0.0) || !isfinite(h)) set_status(st, VI_EINVAL, s);
      const double w[3] = {(gyro[s * 3 + 0] - bg0) * h, (gyro[s * 3 + 1] - bg1) * h, (gyro[s * 3 + 2] - bg2) * h};
      so3_exp(w, S.pdRk[l]);
      so3_jr(w, S.pJrk[l]);
      S.pa[l][0] = accel[s * 3 + 0] - ba0;
      S.pa[l][1] = accel[s * 3 + 1] - ba1;
      S.pa[l][2] = accel[s * 3 + 2] - ba2;
      S.ph[l] = h;
    }
    __syncthreads();
    for (int u = 0; u < nb; ++u) {
      const double h = S.ph[u];
      const double hh = h * h;
      total += h;
      const double* dRk = S.pdRk[u];
      const double* Jrk = S.pJrk[u];
      const double* a = S.pa[u];
      // The transition of the (rot, vel, pos) error state is block lower
      // triangular: A = [[dRk^T, 0, 0], [-M1 h, I, 0], [-M1 h^2 / 2, I h, I]]
      // with M1 = dR [a]x; only its non-trivial terms are multiplied.
      // phase 1: T = A cov; the new mean and bias Jacobians (old values on the right); M1 for phase 2
      if (l < 81) {
        const int e = l;
        const int r = e / 9, c = e % 9, br = r / 3, rr = r % 3;
        double v = 0.0;
        if (br == 0) {
          for (int m = 0; m < 3; ++m) v += dRk[m * 3 + rr] * S.cov[m * 9 + c];
        } else {
          double m1[3];
          m1_row(S.dR, a, rr, m1);
          const double f0 = br == 1 ? -h : -0.5 * hh;
          for (int m = 0; m < 3; ++m) v += (f0 * m1[m]) * S.cov[m * 9 + c];
          if (br == 1) {
            v += S.cov[(3 + rr) * 9 + c];
          } else {
            v += h * S.cov[(3 + rr) * 9 + c];
            v += S.cov[(6 + rr) * 9 + c];
          }
        }
        S.T[e] = v;
      }
      const int lj = l - 128;                    // wave 2
      if (lj >= 0 && lj < 9) {
        const int r = lj / 3, c = lj % 3;
        double m1[3];
        m1_row(S.dR, a, r, m1);
        S.M1[lj] = m1[c];
        double mj = 0.0;
        for (int m = 0; m < 3; ++m) mj += m1[m] * S.JR[m * 3 + c];
        S.nJpa[lj] = S.Jpa[lj] + S.Jva[lj] * h - 0.5 * S.dR[lj] * hh;
        S.nJpg[lj] = S.Jpg[lj] + S.Jvg[lj] * h - 0.5 * mj * hh;
        S.nJva[lj] = S.Jva[lj] - S.dR[lj] * h;
        S.nJvg[lj] = S.Jvg[lj] - mj * h;
        double v = 0.0, w = 0.0;
        for (int m = 0; m < 3; ++m) {
          v += dRk[m * 3 + r] * S.JR[m * 3 + c];     // dRk^T J^rot
          w += S.dR[r * 3 + m] * dRk[m * 3 + c];     // dR dRk
        }
        S.nJR[lj] = v - Jrk[lj] * h;
        S.nR[lj] = w;
      } else if (lj >= 16 && lj < 19) {
        const int i = lj - 16;
        const double ra = S.dR[i * 3 + 0] * a[0] + S.dR[i * 3 + 1] * a[1] + S.dR[i * 3 + 2] * a[2];
        S.np_[i] = S.dp[i] + S.dv[i] * h + 0.5 * ra * hh;
        S.nv[i] = S.dv[i] + ra * h;
      }
      __syncthreads();
      // phase 2: cov = T A^T + Q (lower triangle, mirrored; Q = Bg (sg^2/h) Bg^T +
      // Ba (sa^2/h) Ba^T with Bg = [Jr h; 0; 0], Ba = [0; dR h; dR h^2 / 2], dR dR^T = I);
      // commit the mean and the Jacobians
      if (l < 45) {
        int r = 0;
        while ((r + 1) * (r + 2) / 2 <= l) ++r;
        const int c = l - r * (r + 1) / 2;
        const int bc = c / 3, cc = c % 3, br = r / 3, rr = r % 3;
        const double* Tr = S.T + r * 9;
        double v = 0.0;
        if (bc == 0) {
          for (int m = 0; m < 3; ++m) v += Tr[m] * dRk[m * 3 + cc];
        } else {
          const double f0 = bc == 1 ? -h : -0.5 * hh;
          for (int m = 0; m < 3; ++m) v += Tr[m] * (f0 * S.M1[cc * 3 + m]);
          if (bc == 1) {
            v += Tr[3 + cc];
          } else {
            v += Tr[3 + cc] * h;
            v += Tr[6 + cc];
          }
        }
        double q = 0.0;
        if (br == 0 && bc == 0) {
          double jj = 0.0;
          for (int m = 0; m < 3; ++m) jj += Jrk[rr * 3 + m] * Jrk[cc * 3 + m];
          q = sg2 * h * jj;
        } else if (br >= 1 && bc >= 1 && rr == cc) {
          const double fr = (br == 1) ? h : 0.5 * hh;
          const double fc = (bc == 1) ? h : 0.5 * hh;
          q = sa2 / h * fr * fc;
        }
        S.cov[r * 9 + c] = v + q;
        S.cov[c * 9 + r] = v + q;
      } else if (l < 54) {
        const int i = l - 45;
        S.dR[i] = S.nR[i]; S.JR[i] = S.nJR[i];
        S.Jvg[i] = S.nJvg[i]; S.Jva[i] = S.nJva[i]; S.Jpg[i] = S.nJpg[i]; S.Jpa[i] = S.nJpa[i];
      } else if (l < 57) {
        S.dp[l - 54] = S.np_[l - 54];
        S.dv[l - 54] = S.nv[l - 54];
      }
      __syncthreads();
    }
  }

  vi_preint* o = out + f;
  if (l == 0) o->dt = total;
  if (l < 9) {
    o->dR[l] = S.dR[l];
    o->J_rot[l] = S.JR[l];
    const int r = l / 3, c = l % 3;
    o->J_vel[r * 6 + c] = S.Jvg[l];
    o->J_vel[r * 6 + 3 + c] = S.Jva[l];
    o->J_pos[r * 6 + c] = S.Jpg[l];
    o->J_pos[r * 6 + 3 + c] = S.Jpa[l];
  }
  if (l < 3) { o->dv[l] = S.dv[l]; o->dp[l] = S.dp[l]; }
  // internal (rot, vel, pos) -> residual order (rot, pos, vel)
  for (int e = l; e < 81; e += kPreintThreads) {
    const int r = e / 9, c = e % 9;
    const int pr = (r < 3) ? r : (r < 6 ? r + 3 : r - 3);
    const int pc = (c < 3) ? c : (c < 6 ? c + 3 : c - 3);
    o->cov[e] = S.cov[pr * 9 + pc];
  }
  if (l < 6) {
    o->bias_hat[l] = bias_hat[f * 6 + l];
    const double sw = (l < 3) ? noise.sigma_bgw : noise.sigma_baw;
    o->cov_bias[l] = sw * sw * total;
  }
}

// Lambda = blkdiag(cov^-1, diag(1 / cov_bias)) per factor.  Every lane forms
// the Cholesky factor of the 9x9 covariance in registers (packed lower
// triangle; no lane waits on another), then lane c < 9 forms column c of its
// inverse by forward substitution; Lambda's 9x9 block is L^-T L^-1.
__device__ __forceinline__ constexpr int tri9(int i, int j) { return i * (i + 1) / 2 + j; }

__global__ void __launch_bounds__(64) k_imu_info(int F, DevPlan D, double* __restrict__ Lam, DevStatus* stall) {
  __shared__ double Li[81];     // L^-1
  const int f = blockIdx.x;
  const int l = threadIdx.x;
  if (f >= F) return;
  const int w = D.win_of_f[f];
  const WinDev& W = D.win[w];
  const vi_preint* P = W.imu + (f - W.f_base);
  DevStatus* st = stall + w;
  double L[45];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j)
      if (j <= i) L[tri9(i, j)] = P->cov[i * 9 + j];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double d = L[tri9(k, k)];
#pragma unroll
    for (int m = 0; m < 9; ++m)
      if (m < k) d -= L[tri9(k, m)] * L[tri9(k, m)];
    if (!(d > 0.0)) { ok = false; d = 1.0; }
    d = sqrt(d);
    L[tri9(k, k)] = d;
#pragma unroll
    for (int i = 0; i < 9; ++i)
      if (i > k) {
        double v = L[tri9(i, k)];
#pragma unroll
        for (int m = 0; m < 9; ++m)
          if (m < k) v -= L[tri9(i, m)] * L[tri9(k, m)];
        L[tri9(i, k)] = v / d;
      }
  }
  if (!ok && l == 0) set_status(st, VI_ENOTPD, -1 - (f - W.f_base));
  if (l < 9) {
    // column l of L^-1: x_r = 0 above the diagonal, (e_l - sum_m L_rm x_m) / L_rr from it on
    double x[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      double v = (r == l) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < 9; ++m)
        if (m < r && m >= l) v -= L[tri9(r, m)] * x[m];
      x[r] = (r < l) ? 0.0 : v / L[tri9(r, r)];
      Li[r * 9 + l] = x[r];
    }
  }
  __syncthreads();
  double* o = Lam + (size_t)f * 225;
  for (int e = l; e < 225; e += 64) {
    const int r = e / 15, c = e % 15;
    double v = 0.0;
    if (r < 9 && c < 9) {
      // (L^-T L^-1)[r][c] = sum_m Li[m][r] Li[m][c]
      for (int m = 0; m < 9; ++m) v += Li[m * 9 + r] * Li[m * 9 + c];
    } else if (r == c) {
      v = 1.0 / P->cov_bias[r - 9];
    }
    o[e] = v;
  }
}

// Initial state of a new keyframe j from the state of keyframe i and the
// factor preintegrated from i to j (Sec. 3.1, frontend tracking): the state
// that zeroes the inertial residual of Eq. 3 (deltas corrected to the bias b_i
// to first order), unless tr(Sigma^iner) (the 9x9 preintegration covariance
// and the 6 bias random-walk variances) is above tau or not finite, in which
// case keyframe j takes keyframe i's state.  One lane per prediction.
__global__ void k_predict_kf(int n, const double* pose_i, const double* vel_i, const double* bias_i,
                             const vi_preint* __restrict__ imu, double gx, double gy, double gz, double tau,
                             double* pose_j, double* vel_j, double* bias_j, int32_t* used) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const vi_preint* P = imu + k;
  double tr = 0.0;
  for (int i = 0; i < 9; ++i) tr += P->cov[10 * i];
  for (int i = 0; i < 6; ++i) tr += P->cov_bias[i];
  double q[7], v[3], b[6];
  for (int i = 0; i < 7; ++i) q[i] = pose_i[7 * k + i];
  for (int i = 0; i < 3; ++i) v[i] = vel_i[3 * k + i];
  for (int i = 0; i < 6; ++i) b[i] = bias_i[6 * k + i];
  const bool use = tr <= tau;
  if (use) {
    double db[6], w[3], E[9], dRc[9], Ri[9], Rj[9], dv[3], dp[3], Rdv[3], Rdp[3];
    for (int i = 0; i < 6; ++i) db[i] = b[i] - P->bias_hat[i];
    m3_vec(P->J_rot, db, w);
    so3_exp(w, E);
    m3_mul(P->dR, E, dRc);
    for (int r = 0; r < 3; ++r) {
      double sv = P->dv[r], sp = P->dp[r];
      for (int c = 0; c < 6; ++c) {
        sv += P->J_vel[6 * r + c] * db[c];
        sp += P->J_pos[6 * r + c] * db[c];
      }
      dv[r] = sv;
      dp[r] = sp;
    }
    quat_to_rot(q + 3, Ri);
    m3_mul(Ri, dRc, Rj);
    m3_vec(Ri, dv, Rdv);
    m3_vec(Ri, dp, Rdp);
    const double g[3] = {gx, gy, gz}, dt = P->dt;
    double pn[3], vn[3];
    for (int r = 0; r < 3; ++r) {
      vn[r] = v[r] + g[r] * dt + Rdv[r];
      pn[r] = q[r] + v[r] * dt + 0.5 * g[r] * dt * dt + Rdp[r];
    }
    rot_to_quat(Rj, q + 3);
    for (int r = 0; r < 3; ++r) {
      q[r] = pn[r];
      v[r] = vn[r];
    }
  }
  for (int i = 0; i < 7; ++i) pose_j[7 * k + i] = q[i];
  for (int i = 0; i < 3; ++i) vel_j[3 * k + i] = v[i];
  for (int i = 0; i < 6; ++i) bias_j[6 * k + i] = b[i];
  if (used) used[k] = use ? 1 : 0;
}

}  // namespace

void launch_preint(hipStream_t s, int F, const int32_t* off, const double* gyro, const double* accel,
                   const double* dt, const double* bias_hat, vi_imu_noise noise, vi_preint* out,
                   DevStatus* st) {
  if (F <= 0) return;
  hipLaunchKernelGGL(k_preint, dim3(F), dim3(kPreintThreads), 0, s, F, off, gyro, accel, dt, bias_hat, noise, out, st);
}

void launch_predict_kf(hipStream_t s, int n, const double* pose_i, const double* vel_i, const double* bias_i,
                       const vi_preint* imu, const double* g, double tau, double* pose_j, double* vel_j,
                       double* bias_j, int32_t* used) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_predict_kf, dim3((n + 63) / 64), dim3(64), 0, s, n, pose_i, vel_i, bias_i, imu, g[0], g[1],
                     g[2], tau, pose_j, vel_j, bias_j, used);
}

void launch_imu_info(hipStream_t s, const Plan& P, const DevPlan& D, double* Lam, DevStatus* st) {
  if (P.F <= 0) return;
  hipLaunchKernelGGL(k_imu_info, dim3(P.F), dim3(64), 0, s, P.F, D, Lam, st);
}

}  // namespace vi
