// One damped Gauss-Newton step of the joint visual-inertial problem
// (Sec. 3.1): vision residual and Jacobian per (edge, pixel) (Eq. 1), per-edge
// J^T W J reduction, inertial factors (Eq. 2-3), elimination of the diagonal
// inverse-depth block (Eq. 4), assembly of the reduced pose/velocity/bias
// system, back-substitution of the depth increments and retraction.  The
// Cholesky solve of the reduced system lives in k_chol.hip.
//
// Local edge coordinates.  For an edge e = (i -> j) and a source pixel with
// scaled point P = R_ji q + t_ji d (q = K^-1 [x y 1]^T), a perturbation of the
// relative transform in camera j, P <- P + phi x P + d rho, gives a 2x6 local
// Jacobian J_loc per pixel.  Keyframe perturbations map into it by two 6x6
// matrices that depend on the edge only:
//   eps = M_i (dtheta_i, dp_i) + M_j (dtheta_j, dp_j),
//   M_i = [[R_ji, 0], [[t_ji]x R_ji, R_j^T]],   M_j = [[-I, 0], [0, -R_j^T]].
// The per-pixel work is therefore done in 6-dimensional local coordinates
// (21 Hessian entries instead of 78), and the 6x6 maps are applied once per
// edge when the reduced system is assembled.
#include <algorithm>

#include "vi_internal.h"
#include "vi_math.h"

namespace vi {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void set_status(DevStatus* st, int code, int detail) {
  if (atomicCAS(&st->code, 0, code) == 0) st->detail = detail;
}

// ---------------------------------------------------------------------------
// wave-wide reduce-scatter of 32 doubles: afterwards lane l holds the sum over
// the 64 lanes of element (l >> 1).  32 exchanges instead of 32 * 6.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double reduce_scatter32(double (&v)[32], int lane) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const bool up = lane & 32;
    const double send = up ? v[i] : v[i + 16];
    const double keep = up ? v[i + 16] : v[i];
    v[i] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool up = lane & 16;
    const double send = up ? v[i] : v[i + 8];
    const double keep = up ? v[i + 8] : v[i];
    v[i] = keep + __shfl_xor(send, 16);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool up = lane & 8;
    const double send = up ? v[i] : v[i + 4];
    const double keep = up ? v[i + 4] : v[i];
    v[i] = keep + __shfl_xor(send, 8);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool up = lane & 4;
    const double send = up ? v[i] : v[i + 2];
    const double keep = up ? v[i + 2] : v[i];
    v[i] = keep + __shfl_xor(send, 4);
  }
  {
    const bool up = lane & 2;
    const double send = up ? v[0] : v[1];
    const double keep = up ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 2);
  }
  return v[0] + __shfl_xor(v[0], 1);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ void imu_factor_block(int f, const CamDev& cam, const double* __restrict__ pose,
                                 const double* __restrict__ vel, const double* __restrict__ bias,
                                 const vi_preint* __restrict__ imu, const double* __restrict__ Lam,
                                 double* __restrict__ Hf, double* __restrict__ gf, double* __restrict__ icost,
                                 double* sm);

// relative transform of edge (i -> j): R_ji = R_j^T R_i, t_ji = R_j^T (p_i - p_j)
__device__ __forceinline__ void edge_rel(const double* __restrict__ pose, int i, int j, double* o) {
  double Ri[9], Rj[9], Rji[9], dp[3], tji[3];
  quat_to_rot(pose + (size_t)i * 7 + 3, Ri);
  quat_to_rot(pose + (size_t)j * 7 + 3, Rj);
  m3_tmul(Rj, Ri, Rji);
  for (int k = 0; k < 3; ++k) dp[k] = pose[(size_t)i * 7 + k] - pose[(size_t)j * 7 + k];
  m3_tvec(Rj, dp, tji);
  for (int k = 0; k < 9; ++k) o[k] = Rji[k];
  for (int k = 0; k < 3; ++k) o[9 + k] = tji[k];
}

// ---------------------------------------------------------------------------
// vision assembly: one workgroup per (source keyframe, 256-pixel range), one
// lane per pixel, loop over the source's outgoing edges.  Per pixel: C, w_d and
// the 6 local E-entries per edge; per edge: the local 6x6 Hessian (21) and
// gradient (6), reduced over the wave by reduce_scatter32 into LDS.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_vis_assemble(
    CamDev cam, OptsDev o, DevPlan D, int N, int nkr, const double* __restrict__ pose,
    const double* __restrict__ vel, const double* __restrict__ bias, const double* __restrict__ invdepth,
    const float* __restrict__ target, const float* __restrict__ weight, int F, const vi_preint* __restrict__ imu,
    const double* __restrict__ Lam, double* __restrict__ Rw, double* __restrict__ rel, double* __restrict__ L,
    double* __restrict__ Cd, double* __restrict__ wd, double* __restrict__ hpart, double* __restrict__ vcost,
    double* __restrict__ Hf, double* __restrict__ gf, double* __restrict__ icost) {
  extern __shared__ double sm[];
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if ((int)blockIdx.y >= N) {
    // inertial factors ride along as extra workgroups
    const int f = ((int)blockIdx.y - N) * nkr + (int)blockIdx.x;
    if (f < F && o.use_imu) imu_factor_block(f, cam, pose, vel, bias, imu, Lam, Hf, gf, icost, sm);
    return;
  }
  const int src = blockIdx.y, kr = blockIdx.x;
  const int HW = cam.H * cam.W;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  double* rel_s = sm;              // [k][12]
  double* acc = sm + k * 12;       // [4][k][32]
  if (tid < k) {
    const int e = D.src_edges[e0 + tid];
    edge_rel(pose, src, D.jj[e], rel_s + tid * 12);
    if (kr == 0)
      for (int q = 0; q < 12; ++q) rel[(size_t)e * 12 + q] = rel_s[tid * 12 + q];
  }
  if (kr == 0 && tid == 0) {
    double R[9];
    quat_to_rot(pose + (size_t)src * 7 + 3, R);
    for (int q = 0; q < 9; ++q) Rw[(size_t)src * 9 + q] = R[q];
  }
  for (int i = tid; i < 4 * k * 32; i += 256) acc[i] = 0.0;
  __syncthreads();

  const int p = kr * kVisBlock + tid;
  const bool inpx = p < HW;
  const int pc = inpx ? p : 0;
  const double qx = ((double)(pc % cam.W) - cam.cx) / cam.fx;
  const double qy = ((double)(pc / cam.W) - cam.cy) / cam.fy;
  const double d = invdepth[(size_t)src * HW + pc];
  const int ncol = 6 * k;
  double* Lp = L + (size_t)HW * 6 * e0 + (size_t)pc * ncol;
  double C = 0.0, wdv = 0.0, cost = 0.0, nval = 0.0;

  for (int s = 0; s < k; ++s) {
    const int e = D.src_edges[e0 + s];
    const double* Rt = rel_s + s * 12;
    const double Px = Rt[0] * qx + Rt[1] * qy + Rt[2] + Rt[9] * d;
    const double Py = Rt[3] * qx + Rt[4] * qy + Rt[5] + Rt[10] * d;
    const double Pz = Rt[6] * qx + Rt[7] * qy + Rt[8] + Rt[11] * d;
    const bool valid = inpx && d > 0.0 && Pz > o.z_min * d;
    const size_t toff = (size_t)e * 2 * HW + pc;
    const double tx = target[toff], ty = target[toff + HW];
    const double wx = valid ? (double)weight[toff] : 0.0;
    const double wy = valid ? (double)weight[toff + HW] : 0.0;
    double Jx[6], Jy[6], Jdx = 0.0, Jdy = 0.0, rx = 0.0, ry = 0.0;
    if (valid) {
      const double iz = 1.0 / Pz;
      const double xp = Px * iz, yp = Py * iz, dz = d * iz;
      rx = tx - (cam.fx * xp + cam.cx);
      ry = ty - (cam.fy * yp + cam.cy);
      Jx[0] = cam.fx * xp * yp;  Jx[1] = -cam.fx * (1.0 + xp * xp); Jx[2] = cam.fx * yp;
      Jx[3] = -cam.fx * dz;      Jx[4] = 0.0;                       Jx[5] = cam.fx * xp * dz;
      Jy[0] = cam.fy * (1.0 + yp * yp); Jy[1] = -cam.fy * xp * yp;  Jy[2] = -cam.fy * xp;
      Jy[3] = 0.0;               Jy[4] = -cam.fy * dz;              Jy[5] = cam.fy * yp * dz;
      Jdx = -cam.fx * iz * (Rt[9] - xp * Rt[11]);
      Jdy = -cam.fy * iz * (Rt[10] - yp * Rt[11]);
      nval += 1.0;
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) { Jx[c] = 0.0; Jy[c] = 0.0; }
    }
    C += wx * Jdx * Jdx + wy * Jdy * Jdy;
    wdv -= wx * Jdx * rx + wy * Jdy * ry;
    cost += wx * rx * rx + wy * ry * ry;
    const double ax = wx * Jdx, ay = wy * Jdy;
    if (inpx) {
#pragma unroll
      for (int c = 0; c < 6; ++c) Lp[6 * s + c] = ax * Jx[c] + ay * Jy[c];
    }
    double v[32];
    int q = 0;
    const double bx = wx * rx, by = wy * ry;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double px = wx * Jx[a], py = wy * Jy[a];
#pragma unroll
      for (int b = a; b < 6; ++b) v[q++] = px * Jx[b] + py * Jy[b];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) v[21 + a] = -(Jx[a] * bx + Jy[a] * by);
#pragma unroll
    for (int a = 27; a < 32; ++a) v[a] = 0.0;
    const double tot = reduce_scatter32(v, lane);
    if ((lane & 1) == 0 && (lane >> 1) < 27) acc[(wave * k + s) * 32 + (lane >> 1)] += tot;
  }
  if (inpx) {
    Cd[(size_t)src * HW + p] = C + o.eta;
    wd[(size_t)src * HW + p] = wdv;
  }
  cost = wave_sum(cost);
  nval = wave_sum(nval);
  if (lane == 0) { red[0][wave] = cost; red[1][wave] = nval; }
  __syncthreads();
  if (tid == 0) {
    const size_t b = ((size_t)src * nkr + kr) * 2;
    vcost[b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    vcost[b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
  for (int i = tid; i < k * 27; i += 256) {
    const int s = i / 27, c = i % 27;
    const double t = acc[(0 * k + s) * 32 + c] + acc[(1 * k + s) * 32 + c] + acc[(2 * k + s) * 32 + c] +
                     acc[(3 * k + s) * 32 + c];
    hpart[((size_t)(e0 + s) * nkr + kr) * 32 + c] = t;
  }
}

// ---------------------------------------------------------------------------
// inertial factors (Eq. 3): residual, 15x30 Jacobian, H = J^T Lambda J,
// g = -J^T Lambda r, cost r^T Lambda r.  One 64-lane workgroup per factor.
// ---------------------------------------------------------------------------
__device__ void imu_residual_jacobian(const double* pose, const double* vel, const double* bias,
                                      const vi_preint* P, const double* g, int i, double* r, double* J) {
  const int j = i + 1;
  double Ri[9], Rj[9];
  quat_to_rot(pose + (size_t)i * 7 + 3, Ri);
  quat_to_rot(pose + (size_t)j * 7 + 3, Rj);
  const double* pi = pose + (size_t)i * 7;
  const double* pj = pose + (size_t)j * 7;
  const double* vi = vel + (size_t)i * 3;
  const double* vj = vel + (size_t)j * 3;
  const double* bi = bias + (size_t)i * 6;
  const double* bj = bias + (size_t)j * 6;
  const double dt = P->dt;
  double db[6];
  for (int k = 0; k < 6; ++k) db[k] = bi[k] - P->bias_hat[k];
  double phi[3], Eb[9], dRc[9], RiRj[9], M[9], rr[3];
  m3_vec(P->J_rot, db, phi);
  so3_exp(phi, Eb);
  m3_mul(P->dR, Eb, dRc);
  m3_tmul(Ri, Rj, RiRj);
  m3_tmul(dRc, RiRj, M);
  so3_log(M, rr);
  double yp[3], yv[3], Ryp[3], Ryv[3];
  for (int k = 0; k < 3; ++k) {
    yp[k] = pj[k] - pi[k] - vi[k] * dt - 0.5 * g[k] * dt * dt;
    yv[k] = vj[k] - vi[k] - g[k] * dt;
  }
  m3_tvec(Ri, yp, Ryp);
  m3_tvec(Ri, yv, Ryv);
  for (int k = 0; k < 3; ++k) {
    double cp = P->dp[k], cv = P->dv[k];
    for (int m = 0; m < 6; ++m) {
      cp += P->J_pos[k * 6 + m] * db[m];
      cv += P->J_vel[k * 6 + m] * db[m];
    }
    r[k] = rr[k];
    r[3 + k] = Ryp[k] - cp;
    r[6 + k] = Ryv[k] - cv;
    r[9 + k] = bj[k] - bi[k];
    r[12 + k] = bj[3 + k] - bi[3 + k];
  }
  if (J == nullptr) return;
  double Jri[9], Jrp[9], Er[9], T1[9], T2[9], T3[9];
  so3_jr_inv(rr, Jri);
  so3_jr(phi, Jrp);
  so3_exp(rr, Er);
  // rotation rows
  double RjRi[9];
  m3_tmul(Rj, Ri, RjRi);
  m3_mul(Jri, RjRi, T1);
  m3_tmul(Er, Jrp, T2);           // Exp(r)^T Jr(phi)
  m3_mul(T2, P->J_rot, T3);
  m3_mul(Jri, T3, T2);            // Jr^-1(r) Exp(r)^T Jr(phi) J^rot
  double Syp[9], Syv[9];
  skew(Ryp, Syp);
  skew(Ryv, Syv);
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      J[(0 + a) * 30 + 0 + b] = -T1[a * 3 + b];
      J[(0 + a) * 30 + 9 + b] = -T2[a * 3 + b];
      J[(0 + a) * 30 + 15 + b] = Jri[a * 3 + b];
      const double RiT = Ri[b * 3 + a];
      J[(3 + a) * 30 + 0 + b] = Syp[a * 3 + b];
      J[(3 + a) * 30 + 3 + b] = -RiT;
      J[(3 + a) * 30 + 6 + b] = -RiT * dt;
      J[(3 + a) * 30 + 18 + b] = RiT;
      J[(6 + a) * 30 + 0 + b] = Syv[a * 3 + b];
      J[(6 + a) * 30 + 6 + b] = -RiT;
      J[(6 + a) * 30 + 21 + b] = RiT;
    }
    for (int m = 0; m < 6; ++m) {
      J[(3 + a) * 30 + 9 + m] = -P->J_pos[a * 6 + m];
      J[(6 + a) * 30 + 9 + m] = -P->J_vel[a * 6 + m];
    }
  }
  for (int a = 0; a < 6; ++a) {
    J[(9 + a) * 30 + 9 + a] = -1.0;
    J[(9 + a) * 30 + 24 + a] = 1.0;
  }
}

// One inertial factor per 256-thread workgroup (runs as extra workgroups of the
// vision-assembly launch).  LDS: J (450), T (450), Lambda (225), r (15).
__device__ void imu_factor_block(int f, const CamDev& cam, const double* __restrict__ pose,
                                 const double* __restrict__ vel, const double* __restrict__ bias,
                                 const vi_preint* __restrict__ imu, const double* __restrict__ Lam,
                                 double* __restrict__ Hf, double* __restrict__ gf, double* __restrict__ icost,
                                 double* sm) {
  double* J = sm;
  double* T = J + 450;
  double* Lm = T + 450;
  double* r = Lm + 225;
  const int l = threadIdx.x;
  for (int e = l; e < 450; e += 256) J[e] = 0.0;
  for (int e = l; e < 225; e += 256) Lm[e] = Lam[(size_t)f * 225 + e];
  __syncthreads();
  if (l == 0) imu_residual_jacobian(pose, vel, bias, imu + f, cam.g, f, r, J);
  __syncthreads();
  for (int e = l; e < 450; e += 256) {
    const int a = e / 15, b = e % 15;
    double v = 0.0;
    for (int m = 0; m < 15; ++m) v += J[m * 30 + a] * Lm[m * 15 + b];
    T[a * 15 + b] = v;
  }
  __syncthreads();
  for (int e = l; e < 900; e += 256) {
    const int a = e / 30, c = e % 30;
    double v = 0.0;
    for (int m = 0; m < 15; ++m) v += T[a * 15 + m] * J[m * 30 + c];
    Hf[(size_t)f * 900 + e] = v;
  }
  if (l < 30) {
    double v = 0.0;
    for (int m = 0; m < 15; ++m) v += T[l * 15 + m] * r[m];
    gf[(size_t)f * 30 + l] = -v;
  }
  if (l == 0) {
    double c = 0.0;
    for (int a = 0; a < 15; ++a) {
      double u = 0.0;
      for (int b = 0; b < 15; ++b) u += Lm[a * 15 + b] * r[b];
      c += r[a] * u;
    }
    icost[f] = c;
  }
}

// ---------------------------------------------------------------------------
// Schur Gram per source keyframe on FP64 MFMA:
//   Q' = sum_p [L_p; w_d,p] [L_p; w_d,p]^T / Cd_p     ((6k+1) x (6k+1))
// where L_p stacks the 6 local E-entries of the k outgoing edges.  Row 6k gives
// sum_p L_p w_d,p / Cd_p.  Lower-triangular 16x16 tiles; 64 pixels are staged
// in LDS per pass; each wave owns every fourth tile.
// MFMA f64 16x16x4 operand layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[l/16 + 4 r][l%16] in element r.
// ---------------------------------------------------------------------------
constexpr int kMaxTilesPerWave = 8;

__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

__global__ void __launch_bounds__(256) k_gram(int HW, int nkr, DevPlan D, const double* __restrict__ L,
                                              const double* __restrict__ Cd, const double* __restrict__ wd,
                                              double* __restrict__ gpart) {
  extern __shared__ double sm[];
  const int src = blockIdx.y, kr = blockIdx.x;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  if (k == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ncol = 6 * k;
  const int T = (ncol + 16) / 16;
  const int LDW = 16 * T;
  const int ntiles = T * (T + 1) / 2;
  double* tile = sm;                 // [64][LDW]
  double* invcd = sm + 64 * LDW;     // [64]
  const int p_beg = kr * kGramRange;
  const int p_end = min(HW, p_beg + kGramRange);
  const double* Ls = L + (size_t)HW * 6 * e0;
  double4_t acc[kMaxTilesPerWave];
  int tI[kMaxTilesPerWave], tJ[kMaxTilesPerWave];
#pragma unroll
  for (int u = 0; u < kMaxTilesPerWave; ++u) {
    acc[u] = double4_t{0.0, 0.0, 0.0, 0.0};
    const int t = wave + 4 * u;
    int I = 0, J = 0;
    if (t < ntiles) tile_ij(t, I, J);
    tI[u] = I;
    tJ[u] = J;
  }
  for (int c0 = p_beg; c0 < p_end; c0 += kGramChunk) {
    for (int idx = tid; idx < 64 * LDW; idx += 256) {
      const int pp = idx / LDW, c = idx - pp * LDW;
      const int p = c0 + pp;
      double v = 0.0;
      if (p < p_end) {
        if (c < ncol) v = Ls[(size_t)p * ncol + c];
        else if (c == ncol) v = wd[(size_t)src * HW + p];
      }
      tile[idx] = v;
    }
    if (tid < 64) {
      const int p = c0 + tid;
      const double cd = (p < p_end) ? Cd[(size_t)src * HW + p] : 0.0;
      invcd[tid] = (cd > 0.0) ? 1.0 / cd : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxTilesPerWave; ++u) {
      if (wave + 4 * u < ntiles) {
        const int ca = 16 * tI[u] + (lane & 15);
        const int cb = 16 * tJ[u] + (lane & 15);
#pragma unroll 4
        for (int kk = 0; kk < kGramChunk / 4; ++kk) {
          const int row = kk * 4 + (lane >> 4);
          const double a = tile[row * LDW + ca];
          const double b = tile[row * LDW + cb] * invcd[row];
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  double* out = gpart + D.gram_off[src] + (size_t)kr * ntiles * 256;
#pragma unroll
  for (int u = 0; u < kMaxTilesPerWave; ++u) {
    const int t = wave + 4 * u;
    if (t < ntiles) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = (lane >> 4) + 4 * r, n = lane & 15;
        out[(size_t)t * 256 + m * 16 + n] = acc[u][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// per-source local blocks.  With X = blockdiag(H_e) - Q (6k x 6k, local edge
// coordinates) and the map G (6(k+1) x 6k) whose column block s holds M_i,s^T
// (row block 0: the source) and M_j,s^T (row block s+1: its target):
//   Z  = G X G^T                   the source's contribution to S (6x6 blocks)
//   ZB = diag(G blockdiag(H) G^T)  the B part of its diagonal (for damping)
//   ZV = G (g - y)                 its contribution to w_xi - E C^-1 w_d
// Block by block: W_t = sum_s M_i,s^T X_st;  Z_00 = sum_t W_t M_i,t;
// Z_0,t+1 = W_t M_j,t;  Z_s+1,t+1 = M_j,s^T X_st M_j,t.  The Gram partials
// of every pixel range are summed straight into LDS first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double Mi_at(const double* Rt, const double* Rj, int r, int c) {
  // M_i = [[R_ji, 0], [[t]x R_ji, R_j^T]]
  if (r < 3) return (c < 3) ? Rt[r * 3 + c] : 0.0;
  const int rr = r - 3;
  if (c >= 3) return Rj[(c - 3) * 3 + rr];       // R_j^T[rr][c-3]
  const double* t = Rt + 9;
  double tx[9];
  skew(t, tx);
  return tx[rr * 3 + 0] * Rt[0 * 3 + c] + tx[rr * 3 + 1] * Rt[1 * 3 + c] + tx[rr * 3 + 2] * Rt[2 * 3 + c];
}

__device__ __forceinline__ double Mj_at(const double* Rj, int r, int c) {
  // M_j = [[-I, 0], [0, -R_j^T]]
  if (r < 3) return (c == r) ? -1.0 : 0.0;
  if (c < 3) return 0.0;
  return -Rj[(c - 3) * 3 + (r - 3)];
}

__device__ void cost_reduce_block(int nv, const double* __restrict__ vcost, int F,
                                  const double* __restrict__ icost, int use_imu, double* __restrict__ trace,
                                  int slot, double* s0) {
  double* s1 = s0 + 256;
  const int t = threadIdx.x;
  double c = 0.0, n = 0.0;
  for (int i = t; i < nv; i += 256) { c += vcost[2 * i]; n += vcost[2 * i + 1]; }
  if (use_imu)
    for (int i = t; i < F; i += 256) c += icost[i];
  s0[t] = c;
  s1[t] = n;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) { s0[t] += s0[t + w]; s1[t] += s1[t + w]; }
    __syncthreads();
  }
  if (t == 0) { trace[2 * slot] = s0[0]; trace[2 * slot + 1] = s1[0]; }
}

__global__ void __launch_bounds__(256) k_local(int N, int nkr_vis, int nkr_gram, DevPlan D,
                                               const double* __restrict__ Rw, const double* __restrict__ rel,
                                               const double* __restrict__ hpart,
                                               const double* __restrict__ gpart, double* __restrict__ Z,
                                               double* __restrict__ ZB, double* __restrict__ ZV,
                                               const double* __restrict__ vcost, int F,
                                               const double* __restrict__ icost, int use_imu,
                                               double* __restrict__ trace, int slot) {
  extern __shared__ double sm[];
  if ((int)blockIdx.x == N) {
    cost_reduce_block(N * nkr_vis, vcost, F, icost, use_imu, trace, slot, sm);
    return;
  }
  const int src = blockIdx.x;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int tid = threadIdx.x;
  const int K1 = k + 1;
  double* Zs = Z + D.z_off[src];
  double* ZBs = ZB + D.zb_off[src];
  double* ZVs = ZV + D.zb_off[src];
  if (k == 0) {
    for (int i = tid; i < 36; i += 256) Zs[i] = 0.0;
    for (int i = tid; i < 6; i += 256) { ZBs[i] = 0.0; ZVs[i] = 0.0; }
    return;
  }
  const int ncol = 6 * k, nq = ncol + 1;
  const int T = (ncol + 16) / 16;
  const int ntiles = T * (T + 1) / 2;
  double* Qs = sm;                  // [nq][nq] symmetric
  double* Mi = Qs + nq * nq;        // [k][36]
  double* Mj = Mi + 36 * k;         // [k][36]
  double* Hs = Mj + 36 * k;         // [k][36] full symmetric
  double* gs = Hs + 36 * k;         // [k][6]   g - y
  double* Wt = gs + 6 * k;          // [k][36]
  // Gram partials -> Q (lower tiles hold the data; mirror into both triangles)
  const double* gp = gpart + D.gram_off[src];
  for (int i = tid; i < ntiles * 256; i += 256) {
    const int t = i >> 8, e = i & 255;
    double v = 0.0;
    for (int r = 0; r < nkr_gram; ++r) v += gp[((size_t)r * ntiles + t) * 256 + e];
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const int a = 16 * I + (e >> 4), b = 16 * J + (e & 15);
    if (a < nq && b < nq) {
      Qs[a * nq + b] = v;
      Qs[b * nq + a] = v;
    }
  }
  for (int i = tid; i < k * 36; i += 256) {
    const int s = i / 36, rc = i % 36, r = rc / 6, c = rc % 6;
    const int e = D.src_edges[e0 + s];
    const double* Rt = rel + (size_t)e * 12;
    const double* Rj = Rw + (size_t)D.jj[e] * 9;
    Mi[i] = Mi_at(Rt, Rj, r, c);
    Mj[i] = Mj_at(Rj, r, c);
    const int a = min(r, c), b = max(r, c);
    const int q = a * 6 - a * (a - 1) / 2 + (b - a);
    double h = 0.0;
    const double* hp = hpart + (size_t)(e0 + s) * nkr_vis * 32 + q;
    for (int t = 0; t < nkr_vis; ++t) h += hp[(size_t)t * 32];
    Hs[i] = h;
  }
  __syncthreads();
  for (int i = tid; i < k * 6; i += 256) {
    const int s = i / 6, c = i % 6;
    double g = 0.0;
    const double* hp = hpart + (size_t)(e0 + s) * nkr_vis * 32 + 21 + c;
    for (int t = 0; t < nkr_vis; ++t) g += hp[(size_t)t * 32];
    gs[i] = g - Qs[ncol * nq + 6 * s + c];
  }
  // W_t = sum_s M_i,s^T X_st,  X_st = delta_st H_s - Q_st
  for (int i = tid; i < k * 36; i += 256) {
    const int t = i / 36, a = (i % 36) / 6, b = i % 6;
    double v = 0.0;
    for (int s = 0; s < k; ++s)
      for (int m = 0; m < 6; ++m) {
        double x = -Qs[(6 * s + m) * nq + 6 * t + b];
        if (s == t) x += Hs[s * 36 + m * 6 + b];
        v += Mi[s * 36 + m * 6 + a] * x;
      }
    Wt[i] = v;
  }
  __syncthreads();
  // Z_s+1,t+1 = M_j,s^T X_st M_j,t for all s, t
  for (int i = tid; i < k * k * 36; i += 256) {
    const int st = i / 36, s = st / k, t = st % k, a = (i % 36) / 6, b = i % 6;
    double v = 0.0;
    for (int m = 0; m < 6; ++m) {
      double u = 0.0;
      for (int nn = 0; nn < 6; ++nn) {
        double x = -Qs[(6 * s + m) * nq + 6 * t + nn];
        if (s == t) x += Hs[s * 36 + m * 6 + nn];
        u += x * Mj[t * 36 + nn * 6 + b];
      }
      v += Mj[s * 36 + m * 6 + a] * u;
    }
    Zs[(size_t)((s + 1) * K1 + t + 1) * 36 + a * 6 + b] = v;
  }
  // Z_0,t+1 = W_t M_j,t and its transpose; Z_00 = sum_t W_t M_i,t
  for (int i = tid; i < k * 36; i += 256) {
    const int t = i / 36, a = (i % 36) / 6, b = i % 6;
    double v = 0.0;
    for (int m = 0; m < 6; ++m) v += Wt[t * 36 + a * 6 + m] * Mj[t * 36 + m * 6 + b];
    Zs[(size_t)(0 * K1 + t + 1) * 36 + a * 6 + b] = v;
    Zs[(size_t)((t + 1) * K1 + 0) * 36 + b * 6 + a] = v;
  }
  for (int i = tid; i < 36; i += 256) {
    const int a = i / 6, b = i % 6;
    double v = 0.0;
    for (int t = 0; t < k; ++t)
      for (int m = 0; m < 6; ++m) v += Wt[t * 36 + a * 6 + m] * Mi[t * 36 + m * 6 + b];
    Zs[a * 6 + b] = v;
  }
  for (int i = tid; i < 6 * K1; i += 256) {
    const int ra = i / 6, a = i % 6;
    double zb = 0.0, zv = 0.0;
    const int s_lo = (ra == 0) ? 0 : ra - 1;
    const int s_hi = (ra == 0) ? k : ra;
    for (int s = s_lo; s < s_hi; ++s) {
      const double* M = (ra == 0) ? Mi + s * 36 : Mj + s * 36;
      for (int m = 0; m < 6; ++m) {
        double hm = 0.0;
        for (int nn = 0; nn < 6; ++nn) hm += Hs[s * 36 + m * 6 + nn] * M[nn * 6 + a];
        zb += M[m * 6 + a] * hm;
        zv += M[m * 6 + a] * gs[s * 6 + m];
      }
    }
    ZBs[i] = zb;
    ZVs[i] = zv;
  }
}

// ---------------------------------------------------------------------------
// reduced system: one lane per entry of the (npad + NB) x npad matrix whose
// leading n x n block is S (damped, gauge/inactive rows replaced by identity),
// whose row npad is the right-hand side s (so the Cholesky forward pass
// produces L^-1 s in that row), and whose padding is the identity.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool coord_active(const OptsDev& o, int a, int ra) {
  if (ra < 6) return a >= o.n_fixed;
  if (!o.use_imu) return false;
  if (o.bias_fixed && ra >= 9) return false;
  return true;
}

__global__ void k_assemble(int N, int n, int npad, OptsDev o, DevPlan D, const double* __restrict__ Z,
                           const double* __restrict__ ZB, const double* __restrict__ ZV,
                           const double* __restrict__ Hf, const double* __restrict__ gf,
                           double* __restrict__ A, DevStatus* st) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)(npad + kCholNB) * npad;
  if (idx >= total) return;
  const int r = (int)(idx / npad), c = (int)(idx % npad);
  double val = 0.0;
  if (r < n && c < n) {
    const int a = r / 15, ra = r % 15, b = c / 15, cb = c % 15;
    if (coord_active(o, a, ra) && coord_active(o, b, cb)) {
      double bd = 0.0;
      if (ra < 6 && cb < 6) {
        const int p0 = D.pair_off[a * N + b], p1 = D.pair_off[a * N + b + 1];
        for (int it = p0; it < p1; ++it) {
          val += Z[D.pair_z[it] + ra * 6 + cb];
          if (r == c) bd += ZB[D.pair_zb[it] + ra];
        }
      }
      if (o.use_imu) {
        double vi = 0.0;
        if (a == b) {
          if (a > 0) vi += Hf[(size_t)(a - 1) * 900 + (15 + ra) * 30 + 15 + cb];
          if (a < N - 1) vi += Hf[(size_t)a * 900 + ra * 30 + cb];
        } else if (b == a + 1) {
          vi += Hf[(size_t)a * 900 + ra * 30 + 15 + cb];
        } else if (a == b + 1) {
          vi += Hf[(size_t)b * 900 + (15 + ra) * 30 + cb];
        }
        val += vi;
        if (r == c) bd += vi;
      }
      if (r == c) val += o.lambda * bd;
    } else {
      val = (r == c) ? 1.0 : 0.0;
    }
    if (!isfinite(val)) set_status(st, VI_ENONFINITE, r);
  } else if (r < npad) {
    val = (r == c) ? 1.0 : 0.0;
  } else if (r == npad && c < n) {
    const int b = c / 15, cb = c % 15;
    if (coord_active(o, b, cb)) {
      if (cb < 6) {
        const int p0 = D.pair_off[b * N + b], p1 = D.pair_off[b * N + b + 1];
        for (int it = p0; it < p1; ++it) val += ZV[D.pair_zb[it] + cb];
      }
      if (o.use_imu) {
        if (b > 0) val += gf[(size_t)(b - 1) * 30 + 15 + cb];
        if (b < N - 1) val += gf[(size_t)b * 30 + cb];
      }
    }
    if (!isfinite(val)) set_status(st, VI_ENONFINITE, n + c);
  }
  A[idx] = val;
}

// cost trace: trace[slot] = (vision + inertial cost, valid pixel-residuals)
__global__ void __launch_bounds__(256) k_cost_reduce(int nv, const double* __restrict__ vcost, int F,
                                                     const double* __restrict__ icost, int use_imu,
                                                     double* __restrict__ trace, int slot) {
  __shared__ double s0[512];
  cost_reduce_block(nv, vcost, F, icost, use_imu, trace, slot, s0);
}

// ---------------------------------------------------------------------------
// back-substitution (Eq. 4: dd = C^-1 (w_d - E^T dxi)) and retraction.  The
// E^T dxi term is L_p . u with u_e = M_i,e dxi_i + M_j,e dxi_j (pose parts),
// the local increment of each edge.  Blocks with blockIdx.y == N retract the
// keyframe states.  Nothing is written if an earlier kernel raised an error.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_backsub_retract(
    CamDev cam, OptsDev o, int N, DevPlan D, const double* __restrict__ Rw, const double* __restrict__ rel,
    const double* __restrict__ L, const double* __restrict__ Cd, const double* __restrict__ wd,
    const double* __restrict__ x, double* __restrict__ pose, double* __restrict__ vel,
    double* __restrict__ bias, double* __restrict__ invdepth, double* __restrict__ dd_out,
    double* __restrict__ rep_dxi, DevStatus* st) {
  extern __shared__ double sm[];
  if (st->code != 0) return;
  const int tid = threadIdx.x;
  const int HW = cam.H * cam.W;
  if ((int)blockIdx.y == N) {
    if (blockIdx.x != 0) return;
    for (int t = tid; t < N; t += 256) {
      const double* dx = x + (size_t)t * 15;
      double* q = pose + (size_t)t * 7;
      quat_retract(q + 3, dx);
      for (int k = 0; k < 3; ++k) {
        q[k] += dx[3 + k];
        vel[(size_t)t * 3 + k] += dx[6 + k];
      }
      for (int k = 0; k < 6; ++k) bias[(size_t)t * 6 + k] += dx[9 + k];
      if (rep_dxi)
        for (int k = 0; k < 15; ++k) rep_dxi[(size_t)t * 15 + k] = dx[k];
    }
    if (tid == 0) st->iters += 1;
    return;
  }
  const int src = blockIdx.y;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  double* u = sm;    // [k][6]
  for (int i = tid; i < 6 * k; i += 256) {
    const int s = i / 6, c = i % 6;
    const int e = D.src_edges[e0 + s];
    const double* Rt = rel + (size_t)e * 12;
    const double* Rj = Rw + (size_t)D.jj[e] * 9;
    const double* xi = x + (size_t)src * 15;
    const double* xj = x + (size_t)D.jj[e] * 15;
    double v = 0.0;
    for (int m = 0; m < 6; ++m) v += Mi_at(Rt, Rj, c, m) * xi[m] + Mj_at(Rj, c, m) * xj[m];
    u[i] = v;
  }
  __syncthreads();
  const int p = blockIdx.x * 256 + tid;
  if (p >= HW) return;
  const size_t pi = (size_t)src * HW + p;
  const double cd = Cd[pi];
  double ddv = 0.0;
  if (cd > 0.0 && k > 0) {
    const double* Lp = L + (size_t)HW * 6 * e0 + (size_t)p * 6 * k;
    double et = 0.0;
    for (int i = 0; i < 6 * k; ++i) et += Lp[i] * u[i];
    ddv = (wd[pi] - et) / cd;
  }
  const double dnew = fmax(invdepth[pi] + ddv, o.d_min);
  invdepth[pi] = dnew;
  dd_out[pi] = ddv;
}

__global__ void k_reset_status(DevStatus* st) {
  if (threadIdx.x == 0) { st->code = 0; st->detail = 0; st->iters = 0; st->pad = 0; }
}

// ---------------------------------------------------------------------------
// cost at the current state (residuals only)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_vis_cost(CamDev cam, OptsDev o, DevPlan D, int nkr,
                                                  const double* __restrict__ pose,
                                                  const double* __restrict__ invdepth,
                                                  const float* __restrict__ target,
                                                  const float* __restrict__ weight, double* __restrict__ vcost) {
  __shared__ double red[2][4];
  __shared__ double rel[kMaxOutDegree * 12];
  const int src = blockIdx.y, kr = blockIdx.x;
  const int HW = cam.H * cam.W;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < k) edge_rel(pose, src, D.jj[D.src_edges[e0 + tid]], rel + tid * 12);
  __syncthreads();
  const int p = kr * kVisBlock + tid;
  const bool inpx = p < HW;
  const int pc = inpx ? p : 0;
  const double qx = ((double)(pc % cam.W) - cam.cx) / cam.fx;
  const double qy = ((double)(pc / cam.W) - cam.cy) / cam.fy;
  const double d = invdepth[(size_t)src * HW + pc];
  double cost = 0.0, nval = 0.0;
  for (int s = 0; s < k; ++s) {
    const int e = D.src_edges[e0 + s];
    const double* Rt = rel + s * 12;
    const double Px = Rt[0] * qx + Rt[1] * qy + Rt[2] + Rt[9] * d;
    const double Py = Rt[3] * qx + Rt[4] * qy + Rt[5] + Rt[10] * d;
    const double Pz = Rt[6] * qx + Rt[7] * qy + Rt[8] + Rt[11] * d;
    const bool valid = inpx && d > 0.0 && Pz > o.z_min * d;
    if (valid) {
      const size_t toff = (size_t)e * 2 * HW + pc;
      const double iz = 1.0 / Pz;
      const double rx = target[toff] - (cam.fx * Px * iz + cam.cx);
      const double ry = target[toff + HW] - (cam.fy * Py * iz + cam.cy);
      cost += (double)weight[toff] * rx * rx + (double)weight[toff + HW] * ry * ry;
      nval += 1.0;
    }
  }
  cost = wave_sum(cost);
  nval = wave_sum(nval);
  if (lane == 0) { red[0][wave] = cost; red[1][wave] = nval; }
  __syncthreads();
  if (tid == 0) {
    const size_t b = ((size_t)src * nkr + kr) * 2;
    vcost[b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    vcost[b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ void k_imu_cost(int F, CamDev cam, const double* __restrict__ pose, const double* __restrict__ vel,
                           const double* __restrict__ bias, const vi_preint* __restrict__ imu,
                           const double* __restrict__ Lam, double* __restrict__ icost) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  double r[15];
  imu_residual_jacobian(pose, vel, bias, imu + f, cam.g, f, r, nullptr);
  const double* Lm = Lam + (size_t)f * 225;
  double c = 0.0;
  for (int a = 0; a < 15; ++a) {
    double u = 0.0;
    for (int b = 0; b < 15; ++b) u += Lm[a * 15 + b] * r[b];
    c += r[a] * u;
  }
  icost[f] = c;
}

}  // namespace

void launch_chol(hipStream_t s, const Plan& P, const Work& w, DevStatus* st);

static size_t vis_lds(int kmax) {
  const size_t vis = (size_t)kmax * 12 + 4 * (size_t)kmax * 32;
  const size_t imu = 450 + 450 + 225 + 15;
  return sizeof(double) * std::max(vis, imu);
}
static size_t gram_lds(int kmax) {
  const int T = (6 * kmax + 16) / 16;
  return sizeof(double) * (64 * 16 * (size_t)T + 64);
}
static size_t local_lds(int kmax) {
  const size_t k = kmax, nq = 6 * k + 1;
  return sizeof(double) * std::max<size_t>(nq * nq + 4 * 36 * k + 6 * k, 512);
}

void launch_reset_status(hipStream_t s, DevStatus* st) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, st);
}

void chol_set_attributes();

void step_set_attributes(int kmax) {
  chol_set_attributes();
  (void)hipFuncSetAttribute((const void*)k_vis_assemble, hipFuncAttributeMaxDynamicSharedMemorySize, (int)vis_lds(kmax));
  (void)hipFuncSetAttribute((const void*)k_gram, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gram_lds(kmax));
  (void)hipFuncSetAttribute((const void*)k_local, hipFuncAttributeMaxDynamicSharedMemorySize, (int)local_lds(kmax));
}

void launch_step(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const CamDev& cam,
                 const OptsDev& o, const vi_state& x, const float* target, const float* weight,
                 const vi_preint* imu, int iter, double* rep_dxi, double* rep_dd, DevStatus* st,
                 StageMark mark, void* mark_user) {
  const int N = P.N;
  auto done = [&](int stage) { if (mark) mark(mark_user, stage); };
  const int F = (o.use_imu && P.F > 0) ? P.F : 0;
  const int imu_rows = (F + P.nkr_vis - 1) / P.nkr_vis;
  hipLaunchKernelGGL(k_vis_assemble, dim3(P.nkr_vis, N + imu_rows), dim3(256), vis_lds(P.kmax), s, cam, o, D, N,
                     P.nkr_vis, x.pose, x.vel, x.bias, x.invdepth, target, weight, F, imu, w.Lam, w.Rw, w.rel,
                     w.L, w.Cd, w.wd, w.hpart, w.vcost, w.Hf, w.gf, w.icost);
  done(kStVis);
  hipLaunchKernelGGL(k_gram, dim3(P.nkr_gram, N), dim3(256), gram_lds(P.kmax), s, P.HW, P.nkr_gram, D, w.L,
                     w.Cd, w.wd, w.gpart);
  done(kStGram);
  hipLaunchKernelGGL(k_local, dim3(N + 1), dim3(256), local_lds(P.kmax), s, N, P.nkr_vis, P.nkr_gram, D, w.Rw,
                     w.rel, w.hpart, w.gpart, w.Z, w.ZB, w.ZV, w.vcost, F, w.icost, o.use_imu, w.trace, iter);
  done(kStLocal);
  const size_t total = (size_t)(P.npad + kCholNB) * P.npad;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, N, P.n, P.npad, o, D,
                     w.Z, w.ZB, w.ZV, w.Hf, w.gf, w.A, st);
  done(kStAssemble);
  launch_chol(s, P, w, st);
  done(kStChol);
  hipLaunchKernelGGL(k_backsub_retract, dim3((P.HW + 255) / 256, N + 1), dim3(256),
                     sizeof(double) * 6 * P.kmax, s, cam, o, N, D, w.Rw, w.rel, w.L, w.Cd, w.wd, w.x, x.pose,
                     x.vel, x.bias, x.invdepth, rep_dd ? rep_dd : w.dd, rep_dxi, st);
  done(kStBacksub);
}

void launch_final_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const CamDev& cam,
                       const OptsDev& o, const vi_state& x, const float* target, const float* weight,
                       const vi_preint* imu, int slot, DevStatus* st) {
  (void)st;
  const int N = P.N;
  hipLaunchKernelGGL(k_vis_cost, dim3(P.nkr_vis, N), dim3(256), 0, s, cam, o, D, P.nkr_vis, x.pose, x.invdepth,
                     target, weight, w.vcost);
  if (o.use_imu && P.F > 0)
    hipLaunchKernelGGL(k_imu_cost, dim3((P.F + 63) / 64), dim3(64), 0, s, P.F, cam, x.pose, x.vel, x.bias, imu,
                       w.Lam, w.icost);
  hipLaunchKernelGGL(k_cost_reduce, dim3(1), dim3(256), 0, s, N * P.nkr_vis, w.vcost, P.F, w.icost, o.use_imu,
                     w.trace, slot);
}

size_t step_lds_max(int kmax) {
  return std::max(std::max(vis_lds(kmax), gram_lds(kmax)), local_lds(kmax));
}

}  // namespace vi
