// Loop closure by pose-graph bundle adjustment in Sim(3) (Sec. 3.1, "Loop
// Closure: Pose Graph Bundle Adjustment", Eq. 5): the kernels of one damped
// Gauss-Newton step besides the fused vision assembly, which is shared with
// the visual-inertial step (k_vis_gram in k_step.hip; with keyframe scales its
// relative transforms are the similarities E_ij = T_j^-1 T_i).
//
// Keyframe pose T = (s, R, p), X_w = s R X_c + p; 7 unknowns per keyframe
// (dtheta, dp, dsigma): R <- R Exp(dtheta), p <- p + dp, s <- s e^dsigma.
//
// Vision terms in local edge coordinates.  The fused assembly works with the
// perturbation (phi, rho) of camera-j coordinates, P <- P + phi x P + d rho
// (P = d X_j); a scaling of camera-j coordinates moves no projection.  The
// keyframe unknowns map into it by the 6x7 matrices (t = t_ji, R_ji the
// rotation part of E_ij, R_j and s_j of the target keyframe)
//   M_i = [[R_ji, 0, 0], [[t]x R_ji, R_j^T / s_j, -t]],
//   M_j = [[-I, 0, 0], [0, -R_j^T / s_j, 0]],
// so a source's contribution to the reduced system is Z = G X G^T with
// X = blockdiag(H_e) - Q as for the visual-inertial step and G built from
// these maps (7x7 blocks).
//
// Relative-pose terms r_ij = Log(T~_ij E_ij^-1) with information Lambda_ij:
// a right perturbation T <- T Exp(xi) moves r by -Jr^-1(r) Ad(E_ij) xi_i and
// by Jr^-1(r) xi_j; the keyframe update is xi = (dtheta, R^T dp / s, dsigma)
// to first order.  Sim(3) vectors are ordered (phi, rho, sigma).  The
// logarithm takes phi = Log(R), sigma = ln s and rho = V^-1 t with
// V = int_0^1 e^(sigma u) Exp(u phi) du (8-point Gauss-Legendre quadrature of
// the entire integrand); Jr^-1 is the Bernoulli series in ad up to ad^10.
#include "vi_internal.h"
#include "vi_math.h"

namespace vi {

namespace {

__device__ __forceinline__ void set_status_pg(DevStatus* st, int code, int detail) {
  if (atomicCAS(&st->code, 0, code) == 0) st->detail = detail;
}

// 6x7 local maps of edge e (row-major): rel = (s_i/s_j R_ji, t_ji), Rj = R_j / s_j
__device__ __forceinline__ void pg_maps(const double* rel, const double* Rj, double sij, double* Mi, double* Mj) {
  const double* t = rel + 9;
  double Rji[9], tx[9];
  for (int q = 0; q < 9; ++q) Rji[q] = rel[q] / sij;
  skew(t, tx);
  for (int q = 0; q < 42; ++q) { Mi[q] = 0.0; Mj[q] = 0.0; }
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      Mi[r * 7 + c] = Rji[r * 3 + c];
      double v = 0.0;
      for (int m = 0; m < 3; ++m) v += tx[r * 3 + m] * Rji[m * 3 + c];
      Mi[(3 + r) * 7 + c] = v;
      Mi[(3 + r) * 7 + 3 + c] = Rj[c * 3 + r];        // (R_j / s_j)^T
      Mj[(3 + r) * 7 + 3 + c] = -Rj[c * 3 + r];
    }
    Mi[(3 + r) * 7 + 6] = -t[r];
    Mj[r * 7 + r] = -1.0;
  }
}

// Sum of n partials p[0], p[stride], ... in a fixed order
__device__ __forceinline__ double sum_part(const double* __restrict__ p, size_t stride, int n) {
  double s = 0.0;
  for (int r = 0; r < n; ++r) s += p[(size_t)r * stride];
  return s;
}

// ---------------------------------------------------------------------------
// per-source 7x7 blocks of the reduced system: Z = G X G^T, the diagonal of
// the vision Hessian part G blockdiag(H) G^T (for the damping) and the
// right-hand side G (g - y), from the partial sums of the fused assembly.
// One 256-thread workgroup per source.  Block row / column 0 is the source,
// s + 1 the target of its edge s; Z at Z + z_off[src] as [(k+1)^2][7][7].
// ---------------------------------------------------------------------------
constexpr int kPgThreads = 256;

__global__ void __launch_bounds__(kPgThreads) k_local_pg(int nkr_max, DevPlan D, const double* __restrict__ Rw,
                                                         const double* __restrict__ rel,
                                                         const double* __restrict__ hpart,
                                                         const double* __restrict__ gpart, double* __restrict__ Z,
                                                         double* __restrict__ ZB, double* __restrict__ ZV,
                                                         const DevStatus* __restrict__ st) {
  extern __shared__ double sm[];
  const int src = blockIdx.x;
  const int w = D.win_of_kf[src];
  if (st[w].conv) return;
  const WinDev& W = D.win[w];
  const int nkr = W.nkr;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int tid = threadIdx.x;
  const int K1 = k + 1;
  double* Zs = Z + D.z_off[src];
  double* ZBs = ZB + D.zb_off[src];
  double* ZVs = ZV + D.zb_off[src];
  if (k == 0) {
    for (int i = tid; i < 49; i += kPgThreads) Zs[i] = 0.0;
    for (int i = tid; i < 7; i += kPgThreads) { ZBs[i] = 0.0; ZVs[i] = 0.0; }
    return;
  }
  const int ncol = 6 * k, nq = ncol + 1;
  const int T = (ncol + 16) / 16;
  const int ntiles = T * (T + 1) / 2;
  double* Qs = sm;                  // [nq][nq] symmetric
  double* Hs = Qs + nq * nq;        // [k][36]
  double* gs = Hs + 36 * k;         // [k][6]   g - y
  double* Mi = gs + 6 * k;          // [k][42]
  double* Mj = Mi + 42 * k;         // [k][42]
  double* Wt = Mj + 42 * k;         // [k][42]  W_t = sum_s M_i,s^T X_st (7x6)
  const double* gp = gpart + D.gram_off[src];
  const size_t gstride = (size_t)ntiles * 256;
  for (int i = tid; i < ntiles * 256; i += kPgThreads) {
    const int t = i >> 8, e = i & 255;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const int a = 16 * I + (e >> 4), b = 16 * J + (e & 15);
    if (a < nq && b < nq && a >= b) {
      const double v = sum_part(gp + i, gstride, nkr);
      Qs[a * nq + b] = v;
      Qs[b * nq + a] = v;
    }
  }
  for (int i = tid; i < 36 * k; i += kPgThreads) {
    const int s = i / 36, rc = i % 36, r = rc / 6, c = rc % 6;
    const int a = min(r, c), b = max(r, c);
    const int qq = a * 6 - a * (a - 1) / 2 + (b - a);
    Hs[i] = sum_part(hpart + (size_t)(e0 + s) * nkr_max * 32 + qq, 32, nkr);
  }
  for (int i = tid; i < 6 * k; i += kPgThreads)
    gs[i] = sum_part(hpart + (size_t)(e0 + i / 6) * nkr_max * 32 + 21 + i % 6, 32, nkr);
  for (int s = tid; s < k; s += kPgThreads) {
    const int e = D.src_edges[e0 + s];
    const int ls = src - W.kf_base, lj = D.jj[e] - W.kf_base;
    pg_maps(rel + (size_t)e * 12, Rw + (size_t)D.jj[e] * 9, W.scale[ls] / W.scale[lj], Mi + 42 * s, Mj + 42 * s);
  }
  __syncthreads();
  for (int i = tid; i < 6 * k; i += kPgThreads) gs[i] -= Qs[ncol * nq + i];
  auto X = [&](int s, int t, int m, int n) { return (s == t ? Hs[s * 36 + m * 6 + n] : 0.0) - Qs[(6 * s + m) * nq + 6 * t + n]; };
  // W_t[a][n] = sum_s sum_m M_i,s[m][a] X_st[m][n]
  for (int i = tid; i < 42 * k; i += kPgThreads) {
    const int t = i / 42, a = (i % 42) / 6, n = i % 6;
    double v = 0.0;
    for (int s = 0; s < k; ++s)
      for (int m = 0; m < 6; ++m) v += Mi[42 * s + m * 7 + a] * X(s, t, m, n);
    Wt[i] = v;
  }
  __syncthreads();
  // Z blocks
  for (int i = tid; i < K1 * K1 * 49; i += kPgThreads) {
    const int blk = i / 49, a = (i % 49) / 7, b = i % 7;
    const int A = blk / K1, B = blk % K1;
    double v = 0.0;
    if (A == 0 && B == 0) {
      for (int t = 0; t < k; ++t)
        for (int n = 0; n < 6; ++n) v += Wt[42 * t + a * 6 + n] * Mi[42 * t + n * 7 + b];
    } else if (A == 0) {
      const int t = B - 1;
      for (int n = 0; n < 6; ++n) v += Wt[42 * t + a * 6 + n] * Mj[42 * t + n * 7 + b];
    } else if (B == 0) {
      const int t = A - 1;
      for (int n = 0; n < 6; ++n) v += Wt[42 * t + b * 6 + n] * Mj[42 * t + n * 7 + a];
    } else {
      const int s = A - 1, t = B - 1;
      for (int m = 0; m < 6; ++m) {
        const double ma = Mj[42 * s + m * 7 + a];
        if (ma == 0.0) continue;
        double u = 0.0;
        for (int n = 0; n < 6; ++n) u += X(s, t, m, n) * Mj[42 * t + n * 7 + b];
        v += ma * u;
      }
    }
    Zs[i] = v;
  }
  // diagonal of G blockdiag(H) G^T and G (g - y)
  for (int i = tid; i < 7 * K1; i += kPgThreads) {
    const int A = i / 7, a = i % 7;
    double zb = 0.0, zv = 0.0;
    const int s0 = A == 0 ? 0 : A - 1, s1 = A == 0 ? k : A;
    for (int s = s0; s < s1; ++s) {
      const double* M = (A == 0 ? Mi : Mj) + 42 * s;
      for (int m = 0; m < 6; ++m) {
        double hm = 0.0;
        for (int n = 0; n < 6; ++n) hm += Hs[s * 36 + m * 6 + n] * M[n * 7 + a];
        zb += M[m * 7 + a] * hm;
        zv += M[m * 7 + a] * gs[s * 6 + m];
      }
    }
    ZBs[i] = zb;
    ZVs[i] = zv;
  }
}

// ---------------------------------------------------------------------------
// Sim(3) helpers (FP64)
// ---------------------------------------------------------------------------
struct Sim3 {
  double s, R[9], t[3];
};

__device__ inline void sim3_pose(const double* pose, double s, Sim3& T) {
  T.s = s;
  quat_to_rot(pose + 3, T.R);
  for (int k = 0; k < 3; ++k) T.t[k] = pose[k];
}

// A B (similarities compose: s_A s_B, R_A R_B, s_A R_A t_B + t_A)
__device__ inline void sim3_mul(const Sim3& A, const Sim3& B, Sim3& C) {
  C.s = A.s * B.s;
  m3_mul(A.R, B.R, C.R);
  double u[3];
  m3_vec(A.R, B.t, u);
  for (int k = 0; k < 3; ++k) C.t[k] = A.s * u[k] + A.t[k];
}

__device__ inline void sim3_inv(const Sim3& A, Sim3& B) {
  B.s = 1.0 / A.s;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) B.R[r * 3 + c] = A.R[c * 3 + r];
  double u[3];
  m3_tvec(A.R, A.t, u);
  for (int k = 0; k < 3; ++k) B.t[k] = -u[k] / A.s;
}

// r = (phi, rho, sigma) = Log(T)
__device__ inline void sim3_log(const Sim3& T, double* r) {
  double phi[3];
  so3_log(T.R, phi);
  const double sg = log(T.s);
  // V = int_0^1 e^(sg u) Exp(u phi) du by 8-point Gauss-Legendre on [0, 1]
  const double xg[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
  const double wg[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
  double V[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < 8; ++q) {
    const double x = q < 4 ? -xg[3 - q] : xg[q - 4];
    const double w = q < 4 ? wg[3 - q] : wg[q - 4];
    const double u = 0.5 * (x + 1.0);
    double up[3] = {u * phi[0], u * phi[1], u * phi[2]}, E[9];
    so3_exp(up, E);
    const double f = 0.5 * w * exp(sg * u);
    for (int k = 0; k < 9; ++k) V[k] += f * E[k];
  }
  // rho = V^-1 t (3x3 by cofactors)
  const double a = V[0], b = V[1], c = V[2], d = V[3], e = V[4], f = V[5], g = V[6], h = V[7], i = V[8];
  const double A0 = e * i - f * h, A1 = -(d * i - f * g), A2 = d * h - e * g;
  const double det = a * A0 + b * A1 + c * A2;
  const double inv[9] = {A0 / det, -(b * i - c * h) / det, (b * f - c * e) / det,
                         A1 / det, (a * i - c * g) / det, -(a * f - c * d) / det,
                         A2 / det, -(a * h - b * g) / det, (a * e - b * d) / det};
  double rho[3];
  m3_vec(inv, T.t, rho);
  for (int k = 0; k < 3; ++k) { r[k] = phi[k]; r[3 + k] = rho[k]; }
  r[6] = sg;
}

// 7x7 ad of x = (phi, rho, sigma): [[phi]x, 0, 0], [[rho]x, [phi]x + sigma I, -rho], [0, 0, 0]
__device__ inline void sim3_ad(const double* x, double* A) {
  double P[9], Rh[9];
  skew(x, P);
  skew(x + 3, Rh);
  for (int q = 0; q < 49; ++q) A[q] = 0.0;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      A[r * 7 + c] = P[r * 3 + c];
      A[(3 + r) * 7 + c] = Rh[r * 3 + c];
      A[(3 + r) * 7 + 3 + c] = P[r * 3 + c] + (r == c ? x[6] : 0.0);
    }
    A[(3 + r) * 7 + 6] = -x[3 + r];
  }
}

__device__ inline void mat7_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) {
      double v = 0.0;
      for (int m = 0; m < 7; ++m) v += A[r * 7 + m] * B[m * 7 + c];
      C[r * 7 + c] = v;
    }
}

// Jr^-1(x) = I + ad/2 + ad^2/12 - ad^4/720 + ad^6/30240 - ad^8/1209600 + ad^10/47900160
__device__ inline void sim3_jr_inv(const double* x, double* J) {
  double ad[49], P2[49], Pk[49], T[49];
  sim3_ad(x, ad);
  mat7_mul(ad, ad, P2);
  for (int q = 0; q < 49; ++q) J[q] = (q % 8 == 0 ? 1.0 : 0.0) + 0.5 * ad[q] + P2[q] / 12.0;
  const double cf[4] = {-1.0 / 720.0, 1.0 / 30240.0, -1.0 / 1209600.0, 1.0 / 47900160.0};
  for (int q = 0; q < 49; ++q) Pk[q] = P2[q];
  for (int m = 0; m < 4; ++m) {
    mat7_mul(Pk, P2, T);
    for (int q = 0; q < 49; ++q) { Pk[q] = T[q]; J[q] += cf[m] * Pk[q]; }
  }
}

// one relative-pose factor: its residual and, when Ji is set, its Jacobians
// with respect to the two keyframes (the caller weights them by Lambda)
__device__ void relpose_factor(const WinDev& W, int i, int j, const double* meas, double* r, double* Ji,
                               double* Jj) {
  Sim3 Ti, Tj, Tji, E, Ei, Tm, M;
  sim3_pose(W.pose + (size_t)i * 7, W.scale[i], Ti);
  sim3_pose(W.pose + (size_t)j * 7, W.scale[j], Tj);
  sim3_inv(Tj, Tji);
  sim3_mul(Tji, Ti, E);                    // E_ij = T_j^-1 T_i
  sim3_inv(E, Ei);
  Tm.s = meas[7];
  quat_to_rot(meas + 3, Tm.R);
  for (int k = 0; k < 3; ++k) Tm.t[k] = meas[k];
  sim3_mul(Tm, Ei, M);
  sim3_log(M, r);
  if (!Ji) return;
  double Jinv[49], Ad[49], tx[9], tmp[49];
  sim3_jr_inv(r, Jinv);
  // Ad(E) = [[R, 0, 0], [[t]x R, s R, -t], [0, 0, 1]]
  skew(E.t, tx);
  for (int q = 0; q < 49; ++q) Ad[q] = 0.0;
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      Ad[a * 7 + b] = E.R[a * 3 + b];
      double v = 0.0;
      for (int m = 0; m < 3; ++m) v += tx[a * 3 + m] * E.R[m * 3 + b];
      Ad[(3 + a) * 7 + b] = v;
      Ad[(3 + a) * 7 + 3 + b] = E.s * E.R[a * 3 + b];
    }
    Ad[(3 + a) * 7 + 6] = -E.t[a];
  }
  Ad[48] = 1.0;
  mat7_mul(Jinv, Ad, tmp);
  // K = blockdiag(I, R^T / s, 1) of each keyframe applied on the right
  for (int a = 0; a < 7; ++a) {
    for (int c = 0; c < 7; ++c) {
      double vi, vj;
      if (c < 3 || c == 6) {
        vi = -tmp[a * 7 + c];
        vj = Jinv[a * 7 + c];
      } else {
        vi = 0.0;
        vj = 0.0;
        for (int m = 0; m < 3; ++m) {
          vi -= tmp[a * 7 + 3 + m] * Ti.R[(c - 3) * 3 + m] / Ti.s;     // (R^T / s)[m][c-3] = R[c-3][m] / s
          vj += Jinv[a * 7 + 3 + m] * Tj.R[(c - 3) * 3 + m] / Tj.s;
        }
      }
      Ji[a * 7 + c] = vi;
      Jj[a * 7 + c] = vj;
    }
  }
}

// One thread per factor: the four 7x7 blocks of J^T Lambda J into Z at
// rel_z[f] ((i,i), (i,j), (j,i), (j,j)), their diagonals and the right-hand
// side -J^T Lambda r into ZB / ZV at rel_zb[f] (i, then j), the cost.
__global__ void __launch_bounds__(64) k_relpose(int R, DevPlan D, double* __restrict__ Z, double* __restrict__ ZB,
                                                double* __restrict__ ZV, double* __restrict__ rcost,
                                                DevStatus* __restrict__ st, int want_jac) {
  const int f = blockIdx.x * 64 + threadIdx.x;
  if (f >= R) return;
  const int gi = D.rel_ii[f], gj = D.rel_jj[f];
  const int w = D.win_of_kf[gi];
  if (want_jac && st[w].conv) return;
  const WinDev& W = D.win[w];
  const int lf = f - W.rel_base;
  const double* meas = W.rel_meas + (size_t)lf * 8;
  const double* L = W.rel_info + (size_t)lf * 49;
  double r[7], Ji[49], Jj[49];
  relpose_factor(W, gi - W.kf_base, gj - W.kf_base, meas, r, want_jac ? Ji : nullptr, want_jac ? Jj : nullptr);
  double Lr[7], c = 0.0;
  for (int a = 0; a < 7; ++a) {
    double v = 0.0;
    for (int b = 0; b < 7; ++b) v += L[a * 7 + b] * r[b];
    Lr[a] = v;
    c += r[a] * v;
  }
  rcost[f] = c;
  if (!want_jac) return;
  double* Zf = Z + D.rel_z[f];
  double* ZBf = ZB + D.rel_zb[f];
  double* ZVf = ZV + D.rel_zb[f];
  const double* J[2] = {Ji, Jj};
  for (int A = 0; A < 2; ++A) {
    // J_A^T Lambda (7x7)
    double JL[49];
    for (int a = 0; a < 7; ++a)
      for (int b = 0; b < 7; ++b) {
        double v = 0.0;
        for (int m = 0; m < 7; ++m) v += J[A][m * 7 + a] * L[m * 7 + b];
        JL[a * 7 + b] = v;
      }
    for (int a = 0; a < 7; ++a) {
      double g = 0.0;
      for (int m = 0; m < 7; ++m) g += J[A][m * 7 + a] * Lr[m];
      ZVf[7 * A + a] = -g;
    }
    for (int B = 0; B < 2; ++B) {
      double* blk = Zf + (A * 2 + B) * 49;
      for (int a = 0; a < 7; ++a)
        for (int b = 0; b < 7; ++b) {
          double v = 0.0;
          for (int m = 0; m < 7; ++m) v += JL[a * 7 + m] * J[B][m * 7 + b];
          blk[a * 7 + b] = v;
          if (A == B && a == b) ZBf[7 * A + a] = v;
        }
    }
    if (!isfinite(c)) set_status_pg(st + w, VI_ENONFINITE, -3);
  }
}

// reduced system of each window (blockIdx.y), as k_assemble with 7 unknowns
// per keyframe: the pair lists gather the per-source and per-factor blocks
__device__ __forceinline__ bool pg_active(int a, int n_fixed) { return a >= n_fixed; }

__global__ void k_assemble_pg(int n_fixed, double lambda, DevPlan D, const double* __restrict__ Z,
                              const double* __restrict__ ZB, const double* __restrict__ ZV, double* __restrict__ A,
                              int* __restrict__ flags, int* __restrict__ sync, DevStatus* st) {
  const int w = blockIdx.y;
  const WinDev& W = D.win[w];
  const int N = W.N, n = W.n, npad = W.npad;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)(npad + kCholNB) * npad;
  if (idx < (size_t)W.nflags) flags[W.flag_off + idx] = 0;
  if (w == 0 && idx < 4) sync[idx] = 0;
  if (idx >= total) return;
  const int r = (int)(idx / npad), c = (int)(idx % npad);
  // systems on the tile dataflow read only the lower tiles inside the
  // envelope of S (and the right-hand-side row): the other entries are not
  // formed
  if (npad > kCholSmallMaxNpad && r < npad) {
    const int ti = r / kCholNB, tj = c / kCholNB;
    if (tj > ti || tj < D.chol_fc[W.fc_off + ti]) return;
  }
  const int* poff = D.pair_off + W.pair_base;
  double val = 0.0;
  if (r < n && c < n) {
    // block positions -> keyframes (the window's order of the reduced system)
    const int a = D.kf_at[W.kf_base + r / 7], ra = r % 7, b = D.kf_at[W.kf_base + c / 7], cb = c % 7;
    if (pg_active(a, n_fixed) && pg_active(b, n_fixed)) {
      double bd = 0.0;
      const int p0 = poff[a * N + b], p1 = poff[a * N + b + 1];
      for (int it = p0; it < p1; ++it) {
        val += Z[D.pair_z[it] + ra * 7 + cb];
        if (r == c) bd += ZB[D.pair_zb[it] + ra];
      }
      if (r == c) val += lambda * bd;
    } else {
      val = (r == c) ? 1.0 : 0.0;
    }
    if (!isfinite(val)) set_status_pg(st + w, VI_ENONFINITE, 7 * a + ra);
  } else if (r < npad) {
    val = (r == c) ? 1.0 : 0.0;
  } else if (r == npad && c < n) {
    const int b = D.kf_at[W.kf_base + c / 7], cb = c % 7;
    if (pg_active(b, n_fixed)) {
      const int p0 = poff[b * N + b], p1 = poff[b * N + b + 1];
      for (int it = p0; it < p1; ++it) val += ZV[D.pair_zb[it] + cb];
    }
    if (!isfinite(val)) set_status_pg(st + w, VI_ENONFINITE, n + 7 * b + cb);
  }
  A[W.A_off + idx] = val;
}

// back-substitution dd = C^-1 (w_d - L_p . u), u = M_i x_i + M_j x_j per edge
// (7 unknowns per keyframe), and the retraction R <- R Exp(dtheta),
// p <- p + dp, s <- s e^dsigma (workgroups blockIdx.y >= N: window blockIdx.y - N)
template <typename R>
__global__ void __launch_bounds__(256) k_backsub_pg(double z_min, double d_min, int N, DevPlan D,
                                                    const double* __restrict__ Rw, const double* __restrict__ rel,
                                                    const double* __restrict__ Cd, const double* __restrict__ wd,
                                                    const double* __restrict__ x, DevStatus* st) {
  __shared__ double u[kMaxOutDegree * 6];
  __shared__ R rel_s[kMaxOutDegree * 12];
  const int tid = threadIdx.x;
  if ((int)blockIdx.y >= N) {
    const int w = blockIdx.y - N;
    if (blockIdx.x != 0 || st[w].code != 0 || st[w].conv != 0) return;
    const WinDev& W = D.win[w];
    const double* xw = x + W.x_off;
    for (int t = tid; t < W.N; t += 256) {
      const double* dx = xw + (size_t)D.kf_pos[W.kf_base + t] * 7;
      double* q = W.pose + (size_t)t * 7;
      quat_retract(q + 3, dx);
      for (int k = 0; k < 3; ++k) q[k] += dx[3 + k];
      W.scale[t] *= exp(dx[6]);
      if (W.rep_dxi)
        for (int k = 0; k < 7; ++k) W.rep_dxi[(size_t)t * 7 + k] = dx[k];
    }
    if (tid == 0) st[w].iters += 1;
    return;
  }
  const int src = blockIdx.y;
  const int w = D.win_of_kf[src];
  const WinDev W = D.win[w];
  const int HW = W.HW;
  if (st[w].code != 0 || st[w].conv != 0 || (int)blockIdx.x * 256 >= HW) return;
  const int ls = src - W.kf_base;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const double* xw = x + W.x_off;
  for (int i = tid; i < 12 * k; i += 256) rel_s[i] = (R)rel[(size_t)D.src_edges[e0 + i / 12] * 12 + i % 12];
  if (tid < k) {
    const int e = D.src_edges[e0 + tid];
    const int lj = D.jj[e] - W.kf_base;
    double Mi[42], Mj[42];
    pg_maps(rel + (size_t)e * 12, Rw + (size_t)D.jj[e] * 9, W.scale[ls] / W.scale[lj], Mi, Mj);
    const double* xi = xw + (size_t)D.kf_pos[src] * 7;
    const double* xj = xw + (size_t)D.kf_pos[D.jj[e]] * 7;
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
      for (int m = 0; m < 7; ++m) v += Mi[c * 7 + m] * xi[m] + Mj[c * 7 + m] * xj[m];
      u[tid * 6 + c] = v;
    }
  }
  __syncthreads();
  const int p = blockIdx.x * 256 + tid;
  if (p >= HW) return;
  const size_t pl = (size_t)ls * HW + p;
  const size_t pi = W.pix_base + pl;
  const double cd = Cd[pi];
  double* dep = W.invdepth + pl;
  const double d = *dep;
  double ddv = 0.0;
  if (cd > 0.0 && k > 0) {
    // E^T x at this pixel: sum over edges of L_e,p . u_e, L = J_loc^T W J_d
    const R qx = (R)(((double)(p % W.W) - W.cx) / W.fx);
    const R qy = (R)(((double)(p / W.W) - W.cy) / W.fy);
    const R fx = (R)W.fx, fy = (R)W.fy;
    R et = (R)0;
    for (int s = 0; s < k; ++s) {
      const size_t t = (size_t)(D.src_edges[e0 + s] - W.e_base) * 2 * HW + p;
      const R* Rt = rel_s + s * 12;
      const R dd = (R)d;
      const R Px = Rt[0] * qx + Rt[1] * qy + Rt[2] + Rt[9] * dd;
      const R Py = Rt[3] * qx + Rt[4] * qy + Rt[5] + Rt[10] * dd;
      const R Pz = Rt[6] * qx + Rt[7] * qy + Rt[8] + Rt[11] * dd;
      if (!(dd > (R)0 && Pz > (R)z_min * dd)) continue;
      const R iz = (R)1 / Pz;
      const R xp = Px * iz, yp = Py * iz, dz = dd * iz;
      const R wx = (R)W.weight[t], wy = (R)W.weight[t + HW];
      const R Jdx = -fx * iz * (Rt[9] - xp * Rt[11]);
      const R Jdy = -fy * iz * (Rt[10] - yp * Rt[11]);
      const R Jx[6] = {fx * xp * yp, -fx * ((R)1 + xp * xp), fx * yp, -fx * dz, (R)0, fx * xp * dz};
      const R Jy[6] = {fy * ((R)1 + yp * yp), -fy * xp * yp, -fy * xp, (R)0, -fy * dz, fy * yp * dz};
      const R ax = wx * Jdx, ay = wy * Jdy;
#pragma unroll
      for (int c = 0; c < 6; ++c) et += (ax * Jx[c] + ay * Jy[c]) * (R)u[s * 6 + c];
    }
    ddv = (double)(((R)wd[pi] - et) / (R)cd);
  }
  *dep = fmax(d + ddv, d_min);
  if (W.rep_dd) W.rep_dd[pl] = ddv;
}

// per-window cost: the vision partials of every keyframe (ranges of range_px
// pixels) and the relative-pose costs, in a fixed order, into trace slot `slot`;
// with tol > 0 and slot > 0 the window freezes once F_{slot-1} - F_slot <= tol F_{slot-1}
__global__ void __launch_bounds__(256) k_pg_cost(int ncost, int range_px, DevPlan D, const double* __restrict__ vcost,
                                                 const double* __restrict__ rcost, double* __restrict__ trace,
                                                 int slot, double tol, DevStatus* st) {
  __shared__ double s0[256], s1[256];
  const int w = blockIdx.x;
  const WinDev& W = D.win[w];
  const int t = threadIdx.x;
  const int nk = (W.HW + range_px - 1) / range_px;
  double c = 0.0, n = 0.0;
  for (int i = t; i < W.N * nk; i += 256) {
    const size_t b = ((size_t)(W.kf_base + i / nk) * ncost + i % nk) * 2;
    c += vcost[b];
    n += vcost[b + 1];
  }
  for (int i = t; i < W.n_rel; i += 256) c += rcost[W.rel_base + i];
  s0[t] = c;
  s1[t] = n;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if (t < q) { s0[t] += s0[t + q]; s1[t] += s1[t + q]; }
    __syncthreads();
  }
  if (t == 0) {
    trace[(size_t)w * kTraceLen + 2 * slot] = s0[0];
    trace[(size_t)w * kTraceLen + 2 * slot + 1] = s1[0];
    if (st && tol > 0.0 && slot > 0) {
      const double prev = trace[(size_t)w * kTraceLen + 2 * (slot - 1)];
      if (!(prev - s0[0] > tol * prev)) st[w].conv = 1;
    }
  }
}

}  // namespace

size_t pg_local_lds(int kmax) {
  const size_t k = kmax, nq = 6 * k + 1;
  return sizeof(double) * (nq * nq + 36 * k + 6 * k + 3 * 42 * k);
}

void pg_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_local_pg, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)pg_local_lds(kMaxOutDegree));
}

void launch_pg_local(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st) {
  hipLaunchKernelGGL(k_local_pg, dim3(P.N), dim3(kPgThreads), pg_local_lds(P.kmax), s, P.nkr_max, D, w.Rw, w.rel,
                     w.hpart, w.gpart, w.Z, w.ZB, w.ZV, st);
}

void launch_pg_relpose(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st, bool jac) {
  if (P.R > 0)
    hipLaunchKernelGGL(k_relpose, dim3((P.R + 63) / 64), dim3(64), 0, s, P.R, D, w.Z, w.ZB, w.ZV, w.rcost, st,
                       jac ? 1 : 0);
}

void launch_pg_assemble(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, int n_fixed, double lambda,
                        DevStatus* st) {
  size_t total_max = 0;
  for (const WinDev& W : P.win) total_max = std::max(total_max, (size_t)(W.npad + kCholNB) * W.npad);
  hipLaunchKernelGGL(k_assemble_pg, dim3((unsigned)((total_max + 255) / 256), P.n_win), dim3(256), 0, s, n_fixed,
                     lambda, D, w.Z, w.ZB, w.ZV, w.A, w.flags, w.sync, st);
}

void launch_pg_backsub(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                       DevStatus* st) {
  if (o.precision == VI_PREC_MIXED)
    hipLaunchKernelGGL(k_backsub_pg<float>, dim3((P.hw_max + 255) / 256, P.N + P.n_win), dim3(256), 0, s, o.z_min,
                       o.d_min, P.N, D, w.Rw, w.rel, w.Cd, w.wd, w.x, st);
  else
    hipLaunchKernelGGL(k_backsub_pg<double>, dim3((P.hw_max + 255) / 256, P.N + P.n_win), dim3(256), 0, s, o.z_min,
                       o.d_min, P.N, D, w.Rw, w.rel, w.Cd, w.wd, w.x, st);
}

void launch_pg_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, int ncost, int range_px,
                    int slot, double tol, DevStatus* st) {
  hipLaunchKernelGGL(k_pg_cost, dim3(P.n_win), dim3(256), 0, s, ncost, range_px, D, w.vcost, w.rcost, w.trace, slot,
                     tol, st);
}

}  // namespace vi
