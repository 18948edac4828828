// IMU initialisation, stage 2: inertial-only optimisation (Sec. 3.2, "Stage 2:
// Inertial-Only Optimization", and the IMU-initialisation paragraph of the
// implementation details).
//
// The visual poses (R_i, p_i^vis) are fixed; positions and velocities are
// e^s p_i^vis and e^s v_i^vis with a global log-scale s; gravity is
// g = R_wg (0, 0, G).  Unknowns: R_wg (perturbed on the right about the first
// two axes of the gravity frame; a turn about gravity leaves g alone), s, and
// (v_i^vis, b_i) per keyframe: 3 + 9 N.  The objective is the inertial energy
// of Eq. 2 over the factors (i, i+1), each residual as in Eq. 3.
//
// One 256-thread workgroup solves one problem, every iteration in the same
// launch, everything in LDS:
//   * per factor (one lane each): residual and the 15 x 21 Jacobian with
//     respect to (phi_x, phi_y, s, keyframe i, keyframe i+1), whitened by the
//     inverse Cholesky factor of the factor covariance (so H = J^T J);
//   * the normal matrix is an arrowhead of 9 x 9 blocks: block-tridiagonal over
//     the keyframes (a factor couples only i and i+1) with a 3-row border (the
//     globals touch every factor); the damped blocks are assembled one entry per
//     lane (15-term dot products in a fixed order);
//   * block Cholesky along the keyframes (each step: the Schur update of the
//     next diagonal and border blocks by the previous column, the 9 x 9 pivot
//     factor in one lane's registers, the column solve), then the 3 x 3 border
//     pivot, forward and back substitution.
// The workgroup is latency-bound (about 3 barriers per keyframe per
// iteration); problems of a batch run in parallel workgroups.
#include "vi_internal.h"
#include "vi_math.h"

namespace vi {
namespace {

constexpr int kIIThreads = 256;
constexpr int kJC = 21;          // Jacobian columns of one factor
constexpr int kWF = 87;          // whitening record per factor: L^-1 (9 x 9, row-major) + 1/sqrt(cov_bias) (6)

struct IILds {
  double *R, *pv, *v, *b, *Rwg, *s, *J, *r, *cf, *D, *S, *B, *C, *x;
  int* flag;
};

__host__ __device__ inline size_t iinit_lds_doubles(int N) {
  const int F = N - 1;
  return (size_t)9 * N + 3 * N + 3 * N + 6 * N + 9 + 2 + (size_t)15 * kJC * F + 15 * F + F + 1 + 81 * N +
         81 * (size_t)(N > 1 ? N - 1 : 1) + 27 * N + 9 + 3 + 9 * N + 2;
}

__device__ inline IILds carve(double* sh, int N) {
  const int F = N - 1;
  IILds L;
  double* p = sh;
  L.R = p; p += 9 * N;
  L.pv = p; p += 3 * N;
  L.v = p; p += 3 * N;
  L.b = p; p += 6 * N;
  L.Rwg = p; p += 9;
  L.s = p; p += 2;
  L.J = p; p += 15 * kJC * F;
  L.r = p; p += 15 * F;
  L.cf = p; p += F + 1;
  L.D = p; p += 81 * N;
  L.S = p; p += 81 * (N > 1 ? N - 1 : 1);
  L.B = p; p += 27 * N;
  L.C = p; p += 9;
  L.x = p; p += 3 + 9 * N;
  L.flag = (int*)p;
  return L;
}

// residual and whitened Jacobian of factor f -> L.r[15 f..], L.J[315 f..]; returns r^T Lambda r
__device__ double linearize_factor(const IInitDesc& d, const IILds& L, int f, double G) {
  const vi_preint* P = d.imu + f;
  const int i = f, j = f + 1;
  const double es = exp(L.s[0]);
  const double* Ri = L.R + 9 * i;
  const double* Rj = L.R + 9 * j;
  double* J = L.J + 15 * kJC * f;
  double* r = L.r + 15 * f;
  const double dt = P->dt;
  double db[6];
  for (int m = 0; m < 6; ++m) db[m] = L.b[6 * i + m] - P->bias_hat[m];
  // rotation: Log((dR Exp(J_rot db_g))^T R_i^T R_j)
  double w[3], E[9], dRc[9], A[9], M[9], rr[3];
  m3_vec(P->J_rot, db, w);
  so3_exp(w, E);
  m3_mul(P->dR, E, dRc);
  m3_tmul(Ri, Rj, A);
  m3_tmul(dRc, A, M);
  so3_log(M, rr);
  // gravity and its derivatives along phi_x, phi_y: dg/dphi_x = -G R_wg e_y, dg/dphi_y = G R_wg e_x
  double g[3], dgx[3], dgy[3];
  for (int m = 0; m < 3; ++m) {
    g[m] = G * L.Rwg[3 * m + 2];
    dgx[m] = -G * L.Rwg[3 * m + 1];
    dgy[m] = G * L.Rwg[3 * m + 0];
  }
  double yp[3], yv[3], sp[3], sv[3];
  for (int m = 0; m < 3; ++m) {
    sp[m] = L.pv[3 * j + m] - L.pv[3 * i + m] - L.v[3 * i + m] * dt;
    sv[m] = L.v[3 * j + m] - L.v[3 * i + m];
    yp[m] = es * sp[m] - 0.5 * g[m] * dt * dt;
    yv[m] = es * sv[m] - g[m] * dt;
  }
  double Ryp[3], Ryv[3], Rsp[3], Rsv[3], Rgx[3], Rgy[3];
  m3_tvec(Ri, yp, Ryp);
  m3_tvec(Ri, yv, Ryv);
  m3_tvec(Ri, sp, Rsp);
  m3_tvec(Ri, sv, Rsv);
  m3_tvec(Ri, dgx, Rgx);
  m3_tvec(Ri, dgy, Rgy);
  for (int m = 0; m < 3; ++m) {
    double cp = P->dp[m], cv = P->dv[m];
    for (int c = 0; c < 6; ++c) {
      cp += P->J_pos[6 * m + c] * db[c];
      cv += P->J_vel[6 * m + c] * db[c];
    }
    r[m] = rr[m];
    r[3 + m] = Ryp[m] - cp;
    r[6 + m] = Ryv[m] - cv;
  }
  for (int m = 0; m < 6; ++m) r[9 + m] = L.b[6 * j + m] - L.b[6 * i + m];

  for (int e = 0; e < 15 * kJC; ++e) J[e] = 0.0;
  // d r_rot / d b_g,i = -Jr^-1(r_rot) Exp(r_rot)^T Jr(J_rot db_g) J_rot
  {
    double Jri[9], Er[9], Jw[9], T1[9], T2[9], T3[9];
    so3_jr_inv(rr, Jri);
    so3_exp(rr, Er);
    so3_jr(w, Jw);
    m3_tmul(Er, Jw, T1);
    m3_mul(T1, P->J_rot, T2);
    m3_mul(Jri, T2, T3);
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) J[kJC * a + 6 + c] = -T3[3 * a + c];
  }
  for (int a = 0; a < 3; ++a) {
    double* jp = J + kJC * (3 + a);
    double* jv = J + kJC * (6 + a);
    jp[0] = -0.5 * dt * dt * Rgx[a];
    jp[1] = -0.5 * dt * dt * Rgy[a];
    jp[2] = es * Rsp[a];
    jv[0] = -dt * Rgx[a];
    jv[1] = -dt * Rgy[a];
    jv[2] = es * Rsv[a];
    for (int c = 0; c < 3; ++c) {
      jp[3 + c] = -es * dt * Ri[3 * c + a];   // (R_i^T)_{a c}
      jv[3 + c] = -es * Ri[3 * c + a];
      jv[12 + c] = es * Ri[3 * c + a];
    }
    for (int c = 0; c < 6; ++c) {
      jp[6 + c] = -P->J_pos[6 * a + c];
      jv[6 + c] = -P->J_vel[6 * a + c];
    }
  }
  for (int a = 0; a < 6; ++a) {
    J[kJC * (9 + a) + 6 + a] = -1.0;
    J[kJC * (9 + a) + 15 + a] = 1.0;
  }
  // whiten: rows 0..8 by L^-1 of the 9x9 covariance, rows 9..14 by 1/sqrt(cov_bias)
  const double* wf = d.wf + (size_t)kWF * f;
  double Li[45];
  for (int a = 0, e = 0; a < 9; ++a)
    for (int c = 0; c <= a; ++c, ++e) Li[e] = wf[9 * a + c];
  double cost = 0.0;
  for (int c = 0; c <= kJC; ++c) {          // column kJC is the residual
    double x[9], y[9];
    for (int a = 0; a < 9; ++a) x[a] = c < kJC ? J[kJC * a + c] : r[a];
    for (int a = 0, e = 0; a < 9; ++a) {
      double s = 0.0;
      for (int m = 0; m <= a; ++m, ++e) s += Li[e] * x[m];
      y[a] = s;
    }
    for (int a = 0; a < 9; ++a) {
      if (c < kJC) J[kJC * a + c] = y[a];
      else r[a] = y[a];
    }
    for (int a = 9; a < 15; ++a) {
      if (c < kJC) J[kJC * a + c] *= wf[81 + a - 9];
      else r[a] *= wf[81 + a - 9];
    }
  }
  for (int a = 0; a < 15; ++a) cost += r[a] * r[a];
  return cost;
}

// 15-term dot product of columns p and q of factor f's whitened Jacobian (q = kJC: the residual)
__device__ __forceinline__ double jdot(const IILds& L, int f, int p, int q) {
  const double* J = L.J + 15 * kJC * f;
  const double* r = L.r + 15 * f;
  double s = 0.0;
  for (int a = 0; a < 15; ++a) s += J[kJC * a + p] * (q == kJC ? r[a] : J[kJC * a + q]);
  return s;
}

// in-place Cholesky (lower) of a 9x9 block in LDS, in one lane's registers; false if a pivot is not positive
__device__ bool chol9(double* D) {
  double a[81];
#pragma unroll
  for (int e = 0; e < 81; ++e) a[e] = D[e];
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    double dsum = a[9 * c + c];
#pragma unroll
    for (int m = 0; m < c; ++m) dsum -= a[9 * c + m] * a[9 * c + m];
    ok = ok && dsum > 0.0;
    const double lc = sqrt(dsum > 0.0 ? dsum : 1.0);
    a[9 * c + c] = lc;
    const double inv = 1.0 / lc;
#pragma unroll
    for (int rw = c + 1; rw < 9; ++rw) {
      double s = a[9 * rw + c];
#pragma unroll
      for (int m = 0; m < c; ++m) s -= a[9 * rw + m] * a[9 * c + m];
      a[9 * rw + c] = s * inv;
    }
  }
#pragma unroll
  for (int e = 0; e < 81; ++e) D[e] = a[e];
  return ok;
}

__global__ void __launch_bounds__(kIIThreads) k_inertial_init(const IInitDesc* __restrict__ descs, double G,
                                                              double lambda, int iters, DevStatus* status) {
  const IInitDesc d = descs[blockIdx.x];
  const int N = d.N, F = N - 1, t = threadIdx.x;
  extern __shared__ double sh[];
  const IILds L = carve(sh, N);

  // ---- set-up: fixed poses, state, whitening of every factor
  for (int k = t; k < N; k += kIIThreads) {
    quat_to_rot(d.pose_vis + 7 * k + 3, L.R + 9 * k);
    for (int m = 0; m < 3; ++m) L.pv[3 * k + m] = d.pose_vis[7 * k + m];
    for (int m = 0; m < 3; ++m) L.v[3 * k + m] = d.vel[3 * k + m];
    for (int m = 0; m < 6; ++m) L.b[6 * k + m] = d.bias[6 * k + m];
  }
  if (t == 0) {
    quat_to_rot(d.rot_wg, L.Rwg);
    L.s[0] = d.log_scale[0];
    L.flag[0] = 0;
  }
  __syncthreads();
  for (int f = t; f < F; f += kIIThreads) {
    // the diagonal-block area serves as scratch: factor the 9x9 covariance there
    const vi_preint* P = d.imu + f;
    double* a = L.D + 81 * f;
    for (int e = 0; e < 81; ++e) a[e] = P->cov[e];
    bool ok = chol9(a);
    // L^-1 (lower) by forward substitution against the columns of the identity
    double* wf = d.wf + (size_t)kWF * f;
    for (int c = 0; c < 9; ++c) {
      for (int rw = 0; rw < c; ++rw) wf[9 * rw + c] = 0.0;
      for (int rw = c; rw < 9; ++rw) {
        double s = rw == c ? 1.0 : 0.0;
        for (int m = c; m < rw; ++m) s -= a[9 * rw + m] * wf[9 * m + c];
        wf[9 * rw + c] = s / a[9 * rw + rw];
      }
    }
    for (int m = 0; m < 6; ++m) {
      const double cb = P->cov_bias[m];
      ok = ok && cb > 0.0;
      wf[81 + m] = cb > 0.0 ? 1.0 / sqrt(cb) : 0.0;
    }
    if (!ok) atomicOr(L.flag, 1);
  }
  __syncthreads();
  if (L.flag[0]) {
    if (t == 0) { status[blockIdx.x].code = VI_ENOTPD; status[blockIdx.x].detail = -1; }
    return;
  }

  double* xG = L.x;                    // [3] border unknowns (phi_x, phi_y, s)
  double* xK = L.x + 3;                // [N][9] (v, b_g, b_a) per keyframe
  for (int it = 0; it <= iters; ++it) {
    // ---- residuals and whitened Jacobians
    for (int f = t; f < F; f += kIIThreads) L.cf[f] = linearize_factor(d, L, f, G);
    __syncthreads();
    if (t == 0) {
      double c = 0.0;
      for (int f = 0; f < F; ++f) c += L.cf[f];
      if (d.cost) d.cost[it] = c;
      if (!isfinite(c)) L.flag[0] = 2;
    }
    __syncthreads();
    if (it == iters || L.flag[0]) break;
    // ---- damped normal equations: D_k (9x9), S_k (K_{k+1} x K_k), B_k (3 x 9), C (3x3), right-hand side
    const int nD = 81 * N, nS = 81 * F, nB = 27 * N, nC = 9, nR = 3 + 9 * N;
    for (int e = t; e < nD + nS + nB + nC + nR; e += kIIThreads) {
      if (e < nD) {
        const int k = e / 81, p = (e % 81) / 9, q = e % 9;
        double h = 0.0;
        if (k < F) h += jdot(L, k, 3 + p, 3 + q);
        if (k > 0) h += jdot(L, k - 1, 12 + p, 12 + q);
        if (p == q) h *= 1.0 + lambda;
        L.D[e] = h;
      } else if (e < nD + nS) {
        const int u = e - nD, k = u / 81, p = (u % 81) / 9, q = u % 9;
        L.S[u] = jdot(L, k, 12 + p, 3 + q);
      } else if (e < nD + nS + nB) {
        const int u = e - nD - nS, k = u / 27, p = (u % 27) / 9, q = u % 9;
        double h = 0.0;
        if (k < F) h += jdot(L, k, p, 3 + q);
        if (k > 0) h += jdot(L, k - 1, p, 12 + q);
        L.B[u] = h;
      } else if (e < nD + nS + nB + nC) {
        const int u = e - nD - nS - nB, p = u / 3, q = u % 3;
        double h = 0.0;
        for (int f = 0; f < F; ++f) h += jdot(L, f, p, q);
        if (p == q) h *= 1.0 + lambda;
        L.C[u] = h;
      } else {
        const int u = e - nD - nS - nB - nC;
        double h = 0.0;
        if (u < 3) {
          for (int f = 0; f < F; ++f) h += jdot(L, f, u, kJC);
        } else {
          const int k = (u - 3) / 9, p = (u - 3) % 9;
          if (k < F) h += jdot(L, k, 3 + p, kJC);
          if (k > 0) h += jdot(L, k - 1, 12 + p, kJC);
        }
        L.x[u] = -h;
      }
    }
    __syncthreads();
    // ---- block Cholesky along the keyframes with the border; forward substitution
    for (int k = 0; k < N; ++k) {
      if (k > 0) {
        // Schur update by column k-1 (S_{k-1} = L_{k,k-1}, B_{k-1} = L_{G,k-1}, x_{k-1} = y_{k-1})
        const double* Sp = L.S + 81 * (k - 1);
        const double* Bp = L.B + 27 * (k - 1);
        const double* yp = xK + 9 * (k - 1);
        for (int e = t; e < 81 + 27 + 9 + 9 + 3; e += kIIThreads) {
          if (e < 81) {
            const int p = e / 9, q = e % 9;
            double s = 0.0;
            for (int m = 0; m < 9; ++m) s += Sp[9 * p + m] * Sp[9 * q + m];
            L.D[81 * k + e] -= s;
          } else if (e < 108) {
            const int u = e - 81, p = u / 9, q = u % 9;
            double s = 0.0;
            for (int m = 0; m < 9; ++m) s += Bp[9 * p + m] * Sp[9 * q + m];
            L.B[27 * k + u] -= s;
          } else if (e < 117) {
            const int p = e - 108;
            double s = 0.0;
            for (int m = 0; m < 9; ++m) s += Sp[9 * p + m] * yp[m];
            xK[9 * k + p] -= s;
          } else if (e < 126) {
            const int u = e - 117, p = u / 3, q = u % 3;
            double s = 0.0;
            for (int m = 0; m < 9; ++m) s += Bp[9 * p + m] * Bp[9 * q + m];
            L.C[u] -= s;
          } else {
            const int p = e - 126;
            double s = 0.0;
            for (int m = 0; m < 9; ++m) s += Bp[9 * p + m] * yp[m];
            xG[p] -= s;
          }
        }
        __syncthreads();
      }
      if (t == 0) {
        double* Dk = L.D + 81 * k;
        if (!chol9(Dk)) {
          L.flag[0] = 3;
        } else {
          double* y = xK + 9 * k;
          for (int a = 0; a < 9; ++a) {
            double s = y[a];
            for (int m = 0; m < a; ++m) s -= Dk[9 * a + m] * y[m];
            y[a] = s / Dk[9 * a + a];
          }
        }
      }
      __syncthreads();
      if (L.flag[0]) break;
      // column solve: rows of S_k and B_k times L_kk^-T
      if (t < 12) {
        const double* Dk = L.D + 81 * k;
        double* row = t < 9 ? (k < F ? L.S + 81 * k + 9 * t : nullptr) : L.B + 27 * k + 9 * (t - 9);
        if (row) {
          for (int a = 0; a < 9; ++a) {
            double s = row[a];
            for (int m = 0; m < a; ++m) s -= row[m] * Dk[9 * a + m];
            row[a] = s / Dk[9 * a + a];
          }
        }
      }
      __syncthreads();
    }
    if (L.flag[0]) break;
    // border: the last column's update, the 3x3 pivot, then back substitution
    if (t == 0) {
      const double* Bp = L.B + 27 * (N - 1);
      const double* yp = xK + 9 * (N - 1);
      double C[9], y[3];
      for (int p = 0; p < 3; ++p) {
        double s = xG[p];
        for (int m = 0; m < 9; ++m) s -= Bp[9 * p + m] * yp[m];
        y[p] = s;
        for (int q = 0; q < 3; ++q) {
          double c = L.C[3 * p + q];
          for (int m = 0; m < 9; ++m) c -= Bp[9 * p + m] * Bp[9 * q + m];
          C[3 * p + q] = c;
        }
      }
      bool ok = true;
      for (int c = 0; c < 3; ++c) {
        double dsum = C[3 * c + c];
        for (int m = 0; m < c; ++m) dsum -= C[3 * c + m] * C[3 * c + m];
        ok = ok && dsum > 0.0;
        C[3 * c + c] = sqrt(dsum > 0.0 ? dsum : 1.0);
        for (int rw = c + 1; rw < 3; ++rw) {
          double s = C[3 * rw + c];
          for (int m = 0; m < c; ++m) s -= C[3 * rw + m] * C[3 * c + m];
          C[3 * rw + c] = s / C[3 * c + c];
        }
      }
      if (!ok) {
        L.flag[0] = 4;
      } else {
        for (int a = 0; a < 3; ++a) {
          double s = y[a];
          for (int m = 0; m < a; ++m) s -= C[3 * a + m] * y[m];
          y[a] = s / C[3 * a + a];
        }
        for (int a = 2; a >= 0; --a) {
          double s = y[a];
          for (int m = a + 1; m < 3; ++m) s -= C[3 * m + a] * y[m];
          y[a] = s / C[3 * a + a];
        }
        for (int a = 0; a < 3; ++a) xG[a] = y[a];
        // x_k = L_kk^-T (y_k - L_{k+1,k}^T x_{k+1} - L_{G,k}^T x_G), k = N-1 .. 0
        for (int k = N - 1; k >= 0; --k) {
          const double* Dk = L.D + 81 * k;
          double z[9];
          for (int m = 0; m < 9; ++m) {
            double s = xK[9 * k + m];
            if (k < F)
              for (int p = 0; p < 9; ++p) s -= L.S[81 * k + 9 * p + m] * xK[9 * (k + 1) + p];
            for (int p = 0; p < 3; ++p) s -= L.B[27 * k + 9 * p + m] * xG[p];
            z[m] = s;
          }
          for (int a = 8; a >= 0; --a) {
            double s = z[a];
            for (int m = a + 1; m < 9; ++m) s -= Dk[9 * m + a] * z[m];
            z[a] = s / Dk[9 * a + a];
          }
          for (int m = 0; m < 9; ++m) xK[9 * k + m] = z[m];
        }
      }
    }
    __syncthreads();
    if (L.flag[0]) break;
    // ---- retraction
    for (int k = t; k < N; k += kIIThreads) {
      for (int m = 0; m < 3; ++m) L.v[3 * k + m] += xK[9 * k + m];
      for (int m = 0; m < 6; ++m) L.b[6 * k + m] += xK[9 * k + 3 + m];
    }
    if (t == 0) {
      const double w[3] = {xG[0], xG[1], 0.0};
      double E[9], Rn[9];
      so3_exp(w, E);
      m3_mul(L.Rwg, E, Rn);
      for (int e = 0; e < 9; ++e) L.Rwg[e] = Rn[e];
      L.s[0] += xG[2];
    }
    __syncthreads();
  }
  __syncthreads();
  const int fl = L.flag[0];
  if (fl) {
    if (t == 0) {
      status[blockIdx.x].code = fl == 2 ? VI_ENONFINITE : VI_ENOTPD;
      status[blockIdx.x].detail = fl;
    }
    return;
  }
  for (int k = t; k < N; k += kIIThreads) {
    for (int m = 0; m < 3; ++m) d.vel[3 * k + m] = L.v[3 * k + m];
    for (int m = 0; m < 6; ++m) d.bias[6 * k + m] = L.b[6 * k + m];
  }
  if (t == 0) {
    rot_to_quat(L.Rwg, d.rot_wg);
    d.log_scale[0] = L.s[0];
    status[blockIdx.x].iters = iters;
  }
}

}  // namespace

size_t iinit_lds_bytes(int N) { return iinit_lds_doubles(N) * sizeof(double); }

size_t iinit_whiten_doubles(int N) { return (size_t)kWF * (N > 1 ? N - 1 : 0); }

void launch_inertial_init(hipStream_t s, int n, const IInitDesc* descs, int max_n_kf, double G, double lambda,
                          int iters, DevStatus* status) {
  if (n <= 0) return;
  const size_t lds = iinit_lds_bytes(max_n_kf);
  (void)hipFuncSetAttribute((const void*)k_inertial_init, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_inertial_init, dim3(n), dim3(kIIThreads), lds, s, descs, G, lambda, iters, status);
}

}  // namespace vi
