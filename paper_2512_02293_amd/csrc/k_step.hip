// One damped Gauss-Newton step of the joint visual-inertial problem
// (Sec. 3.1), for a batch of independent windows: vision residual and
// Jacobian per (edge, pixel) (Eq. 1), per-edge J^T W J reduction, inertial
// factors (Eq. 2-3), elimination of the diagonal inverse-depth block (Eq. 4),
// assembly of each window's reduced pose/velocity/bias system,
// back-substitution of the depth increments and retraction.  The Cholesky
// solve of the reduced systems lives in k_chol.hip.
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

// ---------------------------------------------------------------------------
// wave-wide reduce of 16 doubles: afterwards lane l holds the sum over the 64
// lanes of element (l >> 2).  Halving steps keep the upper half of the
// remaining elements in the lanes whose deciding bit is set: bit 5 and bit 4
// through the gfx950 lane-swap instructions (which move exactly the halves
// that the two partners need, so no selects), bit 3 and bit 2 through DPP row
// mirrors (involutions that flip the deciding bit and only bits decided
// later); bits 1 and 0 finish with a quad-permute butterfly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double swap_sum32(double a, double b) {
  // lanes < 32: a(l) + a(l + 32);  lanes >= 32: b(l - 32) + b(l)
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double swap_sum16(double a, double b) {
  // even 16-lane rows: a(l) + a(l + 16);  odd rows: b(l - 16) + b(l)
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141;
constexpr int kDppQuadXor2 = 0x4E, kDppQuadXor1 = 0xB1;   // quad_perm [2,3,0,1], [1,0,3,2]

__device__ __forceinline__ double reduce16(double (&v)[16], int lane) {
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = swap_sum32(v[i], v[i + 8]);
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = swap_sum16(v[i], v[i + 4]);
  {
    const bool up = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double send = up ? v[i] : v[i + 2];
      const double keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp_d<kDppRowMirror>(send);
    }
  }
  {
    const bool up = lane & 4;
    const double send = up ? v[0] : v[1];
    const double keep = up ? v[1] : v[0];
    v[0] = keep + dpp_d<kDppRowHalfMirror>(send);
  }
  double r = v[0] + dpp_d<kDppQuadXor2>(v[0]);
  return r + dpp_d<kDppQuadXor1>(r);
}

// the same reduction on 32-bit values
__device__ __forceinline__ float swap_sum32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(a), __float_as_int(b), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ float swap_sum16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(a), __float_as_int(b), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float reduce16(float (&v)[16], int lane) {
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = swap_sum32(v[i], v[i + 8]);
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = swap_sum16(v[i], v[i + 4]);
  {
    const bool up = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = up ? v[i] : v[i + 2];
      const float keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp_f<kDppRowMirror>(send);
    }
  }
  {
    const bool up = lane & 4;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + dpp_f<kDppRowHalfMirror>(send);
  }
  float r = v[0] + dpp_f<kDppQuadXor2>(v[0]);
  return r + dpp_f<kDppQuadXor1>(r);
}

// Running sum of per-block partial sums.  FP64: plain.  FP32: Kahan-
// compensated (s holds the sum, c the running compensation), so the error
// does not grow with the number of blocks.
template <typename R>
struct BlockSum {
  R s = (R)0, c = (R)0;
  __device__ __forceinline__ void add(R v) {
    if constexpr (sizeof(R) == 8) {
      s += v;
    } else {
      const R y = v - c;
      const R t = s + y;
      c = (t - s) - y;
      s = t;
    }
  }
  __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// relative transform of edge (i -> j) of one window, the map that takes
// camera i coordinates to camera j coordinates: R_ji = R_j^T R_i,
// t_ji = R_j^T (p_i - p_j); with keyframe scales (Sim(3) poses of the
// pose-graph adjustment, X_w = s R X + p) o[0..8] = (s_i / s_j) R_ji and
// t_ji = R_j^T (p_i - p_j) / s_j.  i, j index the window's pose array.
// inverse depth i of a window (FP64, or FP32 when the caller keeps FP32 maps)
__device__ __forceinline__ double dep_load(const WinDev& W, size_t i) {
  return W.invdepth32 ? (double)W.invdepth32[i] : W.invdepth[i];
}
__device__ __forceinline__ void dep_store(const WinDev& W, size_t i, double v) {
  if (W.invdepth32)
    W.invdepth32[i] = (float)v;
  else
    W.invdepth[i] = v;
}

// Camera of keyframe a (window index): with the camera-IMU extrinsic the
// state's pose is the body's and the camera is T_wb T_bc, R_c = R_b R_bc,
// p_c = p_b + R_b t_bc (Sec. 3.1, inertial residual).
__device__ __forceinline__ void cam_pose(const WinDev& W, int a, double* Rc, double* pc) {
  const double* pose = W.pose + (size_t)a * 7;
  if (!W.ext) {
    quat_to_rot(pose + 3, Rc);
    for (int k = 0; k < 3; ++k) pc[k] = pose[k];
    return;
  }
  double Rb[9], u[3];
  quat_to_rot(pose + 3, Rb);
  m3_mul(Rb, W.Rbc, Rc);
  m3_vec(Rb, W.tbc, u);
  for (int k = 0; k < 3; ++k) pc[k] = pose[k] + u[k];
}

__device__ __forceinline__ void edge_rel(const WinDev& W, int i, int j, double* o) {
  double Ri[9], Rj[9], Rji[9], pi[3], pj[3], dp[3], tji[3];
  cam_pose(W, i, Ri, pi);
  cam_pose(W, j, Rj, pj);
  m3_tmul(Rj, Ri, Rji);
  for (int k = 0; k < 3; ++k) dp[k] = pi[k] - pj[k];
  m3_tvec(Rj, dp, tji);
  const double sij = W.scale ? W.scale[i] / W.scale[j] : 1.0;
  const double isj = W.scale ? 1.0 / W.scale[j] : 1.0;
  for (int k = 0; k < 9; ++k) o[k] = sij * Rji[k];
  for (int k = 0; k < 3; ++k) o[9 + k] = isj * tji[k];
}

// ---------------------------------------------------------------------------
// Linearisation of one (source pixel, edge) pair in local edge coordinates:
// residual r = target - projection, the 2x6 local Jacobian rows Jx, Jy, the
// depth Jacobian (Jdx, Jdy) and the weights; everything zero when the pair is
// not valid (inverse depth <= 0, or depth in camera j <= z_min).
// ---------------------------------------------------------------------------
template <typename R>
struct PixEdgeT {
  R Jx[6], Jy[6], Jdx, Jdy, rx, ry, wx, wy;
  bool valid;
};
typedef PixEdgeT<double> PixEdge;

template <typename R>
__device__ __forceinline__ R recip(R v);
template <>
__device__ __forceinline__ double recip<double>(double v) { return 1.0 / v; }
template <>
__device__ __forceinline__ float recip<float>(float v) { return __builtin_amdgcn_rcpf(v); }   // 1 ulp

// R = double: the FP64 path; R = float: the mixed-precision path (the
// relative transform is rounded to float once per edge, everything per pixel
// is float).  tgx, tgy, wgx, wgy: the pair's target and weights, loaded by the
// caller (so that loads can be issued ahead of the arithmetic).
template <typename R>
__device__ __forceinline__ void pix_edge_v(const WinDev& W, const OptsDev& o, const double* Rtd, R qx, R qy, R d,
                                           bool inpx, float tgx, float tgy, float wgx, float wgy, bool want_res,
                                           PixEdgeT<R>& q) {
  R Rt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) Rt[c] = (R)Rtd[c];
  const R fx = (R)W.fx, fy = (R)W.fy, cx = (R)W.cx, cy = (R)W.cy;
  const R Px = Rt[0] * qx + Rt[1] * qy + Rt[2] + Rt[9] * d;
  const R Py = Rt[3] * qx + Rt[4] * qy + Rt[5] + Rt[10] * d;
  const R Pz = Rt[6] * qx + Rt[7] * qy + Rt[8] + Rt[11] * d;
  q.valid = inpx && d > (R)0 && Pz > (R)o.z_min * d;
  q.wx = q.valid ? (R)wgx : (R)0;
  q.wy = q.valid ? (R)wgy : (R)0;
  q.rx = (R)0;
  q.ry = (R)0;
  if (q.valid) {
    const R iz = recip<R>(Pz);
    const R xp = Px * iz, yp = Py * iz, dz = d * iz;
    if (want_res) {
      q.rx = (R)tgx - (fx * xp + cx);
      q.ry = (R)tgy - (fy * yp + cy);
    }
    q.Jx[0] = fx * xp * yp;  q.Jx[1] = -fx * ((R)1 + xp * xp); q.Jx[2] = fx * yp;
    q.Jx[3] = -fx * dz;      q.Jx[4] = (R)0;                   q.Jx[5] = fx * xp * dz;
    q.Jy[0] = fy * ((R)1 + yp * yp); q.Jy[1] = -fy * xp * yp;  q.Jy[2] = -fy * xp;
    q.Jy[3] = (R)0;          q.Jy[4] = -fy * dz;               q.Jy[5] = fy * yp * dz;
    q.Jdx = -fx * iz * (Rt[9] - xp * Rt[11]);
    q.Jdy = -fy * iz * (Rt[10] - yp * Rt[11]);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) { q.Jx[c] = (R)0; q.Jy[c] = (R)0; }
    q.Jdx = (R)0;
    q.Jdy = (R)0;
  }
}

template <typename R>
__device__ __forceinline__ void pix_edge(const WinDev& W, const OptsDev& o, const double* Rtd, R qx, R qy, R d,
                                         bool inpx, const float* __restrict__ target,
                                         const float* __restrict__ weight, size_t toff, bool want_res,
                                         PixEdgeT<R>& q) {
  const float tx = (want_res && target) ? target[toff] : 0.0f;
  const float ty = (want_res && target) ? target[toff + W.HW] : 0.0f;
  pix_edge_v<R>(W, o, Rtd, qx, qy, d, inpx, tx, ty, weight[toff], weight[toff + W.HW], want_res, q);
}

// ---------------------------------------------------------------------------
// inertial factors (Eq. 3): residual, 15x30 Jacobian (NULL J: residual only).
// i is the index of the earlier keyframe in the window's arrays.
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
// vision-assembly launch): H = J^T Lambda J, g = -J^T Lambda r, r^T Lambda r.
// LDS: J (450), T (450), Lambda (225), r (15).  f is the global factor index.
__device__ void imu_factor_block(int f, const WinDev& W, const double* __restrict__ Lam, double* __restrict__ Hf,
                                 double* __restrict__ gf, double* __restrict__ icost, double* sm) {
  double* J = sm;
  double* T = J + 450;
  double* Lm = T + 450;
  double* r = Lm + 225;
  const int l = threadIdx.x;
  const int lf = f - W.f_base;
  for (int e = l; e < 450; e += (int)blockDim.x) J[e] = 0.0;
  for (int e = l; e < 225; e += (int)blockDim.x) Lm[e] = Lam[(size_t)f * 225 + e];
  __syncthreads();
  if (l == 0) imu_residual_jacobian(W.pose, W.vel, W.bias, W.imu + lf, W.g, lf, r, J);
  __syncthreads();
  for (int e = l; e < 450; e += (int)blockDim.x) {
    const int a = e / 15, b = e % 15;
    double v = 0.0;
    for (int m = 0; m < 15; ++m) v += J[m * 30 + a] * Lm[m * 15 + b];
    T[a * 15 + b] = v;
  }
  __syncthreads();
  for (int e = l; e < 900; e += (int)blockDim.x) {
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
// Fused vision assembly and Schur Gram.  One 512-thread workgroup per (source
// keyframe, pixel range), walked in chunks of 64 pixels; lane = pixel, wave w
// takes the source's edges w, w + 8, w + 16.  Per (pixel, edge): residual and
// Jacobians in local edge coordinates; per pixel: C and w_d; per edge: the
// local 6x6 Hessian and gradient, summed in each lane's registers over the
// chunks of a block and reduced over the wave once per block (two 16-value
// reduce16 passes).  Of the 21 upper Hessian entries 20 can be non-zero: the
// x row of the local Jacobian has no y-translation term and the y row no
// x-translation term, and the formulas below skip those products.  The 6
// local E-entries of every (pixel, edge) go to a column-major LDS tile
// [6k | w_d | 0][64 px] (two buffers: chunk i + 1 is written while slower
// waves still read chunk i), on which the eight waves then run the Gram
//   Q' = sum_p [L_p; w_d,p][L_p; w_d,p]^T / C_p
// over lower-triangular 16x16 tiles on MFMA 16x16x4 (FP64, or FP32 in mixed
// mode).  The pixels of a chunk are dealt to the MFMA's K index so that the
// 16 operands a lane supplies for one tile are 16 consecutive pixels of one
// tile column, read with 128-bit LDS loads.  MFMA operand layout: lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; it receives D[l/16 + 4 r][l%16]
// (FP64) or D[4 (l/16) + r][l%16] (FP32) in element r.  FP32 sums (mixed
// mode) run over blocks of 8 chunks (512 pixels) and are Kahan-added across
// blocks; FP64 sums run over the whole range.  The E-block never leaves the
// chip.  The column sums C and w_d of a chunk are formed by the last wave
// (which has the fewest edges and Gram tiles).  Inertial factors ride along
// as extra workgroups (the first imu_rows rows of the grid, so that their
// serial rotation algebra starts first and overlaps the vision workgroups).
// ---------------------------------------------------------------------------
constexpr int kVisThreads = 512;
constexpr int kVisWaves = kVisThreads / 64;
constexpr int kVisSumWave = kVisWaves - 1;     // forms C and w_d of each chunk
constexpr int kVisBlockChunks = 8;             // chunks per FP32 block sum

// E-tile column stride in elements: 64 pixel rows plus padding, so that the
// 128-bit reads of the 16 columns one instruction touches hit distinct banks
template <typename R>
constexpr int vis_ldc() { return sizeof(R) == 4 ? 68 : 66; }

// Gram tiles (lower triangle of T x T) and edge slots per wave for a source
// with k outgoing edges
__host__ __device__ constexpr int vis_tiles_T(int k) { return (6 * k + 16) / 16; }

__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

// 16 consecutive LDS values (16-byte aligned) into registers
__device__ __forceinline__ void lds_load16(const float* p, float (&v)[16]) {
  const float4_t* q = (const float4_t*)p;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4_t x = q[i];
    v[4 * i] = x[0]; v[4 * i + 1] = x[1]; v[4 * i + 2] = x[2]; v[4 * i + 3] = x[3];
  }
}
__device__ __forceinline__ void lds_load16(const double* p, double (&v)[16]) {
  const double2_t* q = (const double2_t*)p;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double2_t x = q[i];
    v[2 * i] = x[0]; v[2 * i + 1] = x[1];
  }
}

// an empty asm that takes the 16 values as in-out operands: every load and
// product that forms them is issued before it, and nothing that uses them
// moves above it (one LDS wait per Gram tile instead of one per 4 MFMAs)
__device__ __forceinline__ void pin16(float (&v)[16]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
               "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15]));
}
__device__ __forceinline__ void pin8(double (&v)[8]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]));
}

// per-lane sums of one edge over the chunks of a block: local Hessian (upper
// triangle, row-major, 21 entries; entry (3, 4) stays zero) and gradient (6)
template <typename R>
struct EdgeAcc {
  R h[21], g[6];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 21; ++i) h[i] = (R)0;
#pragma unroll
    for (int i = 0; i < 6; ++i) g[i] = (R)0;
  }
};

// One (pixel, edge) pair: projection P = R_ji q + t_ji d, validity, residual
// r = target - (f P_xy / P_z + c), the local Jacobian rows J_x = f_x u_x,
// J_y = f_y u_y with
//   u_x = (x y, -(1 + x^2), y, -d', 0, x d'),  u_y = (1 + y^2, -x y, -x, 0, -d', y d')
// (x = P_x / P_z, y = P_y / P_z, d' = d / P_z: a perturbation phi, rho of the
// relative transform in camera j moves P by phi x P + d rho), and the depth
// Jacobian J_d = f (-(t_x - x t_z) / P_z, -(t_y - y t_z) / P_z).  Adds the
// pair's terms to the lane's Hessian / gradient sums, C, w_d and the cost,
// and writes its 6 E-entries (J_loc^T W J_d) to column base e of the tile.
// An invalid pair contributes zero everywhere (branch-free: its weights and
// residual are replaced by zero, its depth by a harmless 1).
template <typename R, int LDC>
__device__ __forceinline__ void vis_pair(const R* rt, R fx, R fy, R cx, R cy, R zmin, R qx, R qy, R d, bool inpx,
                                         float tgx, float tgy, float wgx, float wgy, EdgeAcc<R>& A, R* e, R& Cp,
                                         R& Wp, R& cst, R& nv) {
  const R Px = rt[0] * qx + rt[1] * qy + rt[2] + rt[9] * d;
  const R Py = rt[3] * qx + rt[4] * qy + rt[5] + rt[10] * d;
  const R Pz = rt[6] * qx + rt[7] * qy + rt[8] + rt[11] * d;
  const bool valid = inpx && d > (R)0 && Pz > zmin * d;
  const R iz = recip<R>(valid ? Pz : (R)1);
  const R xp = Px * iz, yp = Py * iz, dz = d * iz;
  const R wx = valid ? (R)wgx : (R)0, wy = valid ? (R)wgy : (R)0;
  const R rx = valid ? (R)tgx - (fx * xp + cx) : (R)0;
  const R ry = valid ? (R)tgy - (fy * yp + cy) : (R)0;
  const R xy = xp * yp;
  const R ux[6] = {xy, -((R)1 + xp * xp), yp, -dz, (R)0, xp * dz};
  const R uy[6] = {(R)1 + yp * yp, -xy, -xp, (R)0, -dz, yp * dz};
  const R jdx = -iz * (rt[9] - xp * rt[11]);
  const R jdy = -iz * (rt[10] - yp * rt[11]);
  const R wxf = wx * fx, wyf = wy * fy;
  const R hx = wxf * fx, hy = wyf * fy;       // w f^2
  const R ax = hx * jdx, ay = hy * jdy;       // w f J_d (per unit u)
  const R bx = wxf * rx, by = wyf * ry;       // w f r
  Cp += ax * jdx + ay * jdy;
  Wp -= bx * jdx + by * jdy;
  cst += wx * rx * rx + wy * ry * ry;
  nv += valid ? (R)1 : (R)0;
  // E-entries J_loc^T W J_d
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    R v;
    if (c == 3) v = ax * ux[3];
    else if (c == 4) v = ay * uy[4];
    else v = ax * ux[c] + ay * uy[c];
    e[c * LDC] = v;
  }
  // Hessian and gradient sums (the zero entries of u_x, u_y skipped)
  R px[6], py[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    px[a] = hx * ux[a];
    py[a] = hy * uy[a];
  }
  int m = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
#pragma unroll
    for (int b = a; b < 6; ++b) {
      if (a != 4 && b != 4) A.h[m] += px[a] * ux[b];
      if (a != 3 && b != 3) A.h[m] += py[a] * uy[b];
      ++m;
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    if (a != 4) A.g[a] -= bx * ux[a];
    if (a != 3) A.g[a] -= by * uy[a];
  }
}

// SLOTS: edge slots per wave (k <= 8 SLOTS); TS: Gram tiles per wave (T (T + 1) / 2 <= 8 TS).
template <typename R, int SLOTS, int TS>
__global__ void __launch_bounds__(kVisThreads) k_vis_gram(OptsDev o, DevPlan D, int imu_rows, int F, int nkr_max,
                                                          int ncost, int range, const double* __restrict__ Lam,
                                                          double* __restrict__ Rw, double* __restrict__ rel,
                                                          double* __restrict__ Cd, double* __restrict__ wd,
                                                          double* __restrict__ hpart, double* __restrict__ gpart,
                                                          double* __restrict__ vcost, double* __restrict__ Hf,
                                                          double* __restrict__ gf, double* __restrict__ icost,
                                                          DevStatus* __restrict__ st) {
  constexpr bool kF64 = sizeof(R) == 8;
  constexpr int LDC = vis_ldc<R>();
  extern __shared__ double sm[];
  __shared__ double red[2][kVisWaves];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: per-wave choices stay scalar
  if ((int)blockIdx.y < imu_rows) {
    const int f = (int)blockIdx.y * (int)gridDim.x + (int)blockIdx.x;
    if (f < F && o.use_imu && !(st && st[D.win_of_f[f]].conv)) {   // frozen windows keep their blocks
      const WinDev W = D.win[D.win_of_f[f]];
      imu_factor_block(f, W, Lam, Hf, gf, icost, sm);
    }
    return;
  }
  const int src = blockIdx.y - imu_rows, kr = blockIdx.x;
  if (st && st[D.win_of_kf[src]].conv) return;      // frozen by the tolerance stop: its state is unchanged
  const WinDev W = D.win[D.win_of_kf[src]];
  const int HW = W.HW;
  const int p_beg = kr * range;
  if (p_beg >= HW) return;
  const int p_end = min(HW, p_beg + range);
  const int ls = src - W.kf_base;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int ncol = 6 * k;
  const int T = vis_tiles_T(k);
  const int ntiles = T * (T + 1) / 2;
  const int tsz = 16 * T * LDC;                   // one E-tile buffer
  R* rel_s = (R*)sm;                              // [kMaxOutDegree][12]
  R* Et = rel_s + kMaxOutDegree * 12;             // [2][16 T][LDC]
  R* part = Et + 2 * tsz;                         // [2][kVisWaves][64]  C and w_d partials
  R* invcd = part + 2 * kVisWaves * 64;           // [2][64]
  if (tid < k) {
    const int e = D.src_edges[e0 + tid];
    double r12[12];
    edge_rel(W, ls, D.jj[e] - W.kf_base, r12);
#pragma unroll
    for (int q = 0; q < 12; ++q) rel_s[tid * 12 + q] = (R)r12[q];
    if (kr == 0)
      for (int q = 0; q < 12; ++q) rel[(size_t)e * 12 + q] = r12[q];
  }
  if (kr == 0 && tid == 0) {
    // camera rotation R_c of the keyframe (R_c / s with keyframe scales:
    // R^T / s maps world offsets into the scaled camera frame)
    double Rm[9], pc[3];
    cam_pose(W, ls, Rm, pc);
    const double is = W.scale ? 1.0 / W.scale[ls] : 1.0;
    for (int q = 0; q < 9; ++q) Rw[(size_t)src * 9 + q] = is * Rm[q];
  }
  if (k == 0) {
    // a keyframe without outgoing edges has no residuals (its C, w_d, Gram and
    // blocks are never read): only the non-finite inverse-depth check and an
    // empty cost slot.  k is uniform over the workgroup.
    bool bad = false;
    for (int p = p_beg + tid; p < p_end; p += kVisThreads) bad = bad || !isfinite(dep_load(W, (size_t)ls * HW + p));
    if (st && bad) set_status(st + D.win_of_kf[src], VI_ENONFINITE, -1);
    if (tid == 0) {
      const size_t b = ((size_t)src * ncost + kr) * 2;
      vcost[b] = 0.0;
      vcost[b + 1] = 0.0;
    }
    return;
  }
  for (int i = tid; i < 2 * tsz; i += kVisThreads) Et[i] = (R)0;
  __syncthreads();

  const size_t dsrc = (size_t)ls * HW;            // this keyframe's inverse depths start here
  double* Cds = Cd + W.pix_base + (size_t)ls * HW;
  double* wds = wd + W.pix_base + (size_t)ls * HW;
  const R fx = (R)W.fx, fy = (R)W.fy, cx = (R)W.cx, cy = (R)W.cy, zmin = (R)o.z_min;
  const R ifx = (R)(1.0 / W.fx), ify = (R)(1.0 / W.fy);
  EdgeAcc<R> acc[SLOTS];
  BlockSum<R> hs_a[SLOTS], hs_b[SLOTS];
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) acc[u].zero();
  double4_t gacc[TS];                                   // FP64 Gram
  float4_t gblk[TS], gs[TS], gc[TS];                    // FP32 Gram: block sum, Kahan sum and compensation
#pragma unroll
  for (int u = 0; u < TS; ++u) {
    gacc[u] = double4_t{0.0, 0.0, 0.0, 0.0};
    gblk[u] = gs[u] = gc[u] = float4_t{0.f, 0.f, 0.f, 0.f};
  }
  double cost = 0.0, nval = 0.0;
  // targets, weights and inverse depth of the next chunk are loaded one chunk
  // ahead, so that their latency overlaps the Gram of the current chunk
  size_t eoff[SLOTS];
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int s = wave + kVisWaves * u;
    eoff[u] = s < k ? (size_t)(D.src_edges[e0 + s] - W.e_base) * 2 * HW : 0;
  }
  float ntx[SLOTS], nty[SLOTS], nwx[SLOTS], nwy[SLOTS];
  double nd;
  auto prefetch = [&](int c) {
    const int pp = (c + lane < p_end) ? c + lane : p_beg;
    nd = dep_load(W, dsrc + pp);
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      if (wave + kVisWaves * u < k) {
        const size_t t = eoff[u] + pp;
        ntx[u] = W.target[t];
        nty[u] = W.target[t + HW];
        nwx[u] = W.weight[t];
        nwy[u] = W.weight[t + HW];
      }
    }
  };
  // FP32 with at most two edges per wave: the relative transforms of this
  // wave's edges stay in registers for the whole range (else read from LDS)
  constexpr bool kRegRel = !kF64 && SLOTS <= 2;
  R rtv[kRegRel ? SLOTS : 1][12];
  if constexpr (kRegRel) {
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int sl = min(wave + kVisWaves * u, k - 1);
#pragma unroll
      for (int q = 0; q < 12; ++q) rtv[u][q] = rel_s[sl * 12 + q];
    }
  }
  // Gram tiles of this wave (uniform; FP32: found once for the range)
  int tI[TS], tJ[TS];
#pragma unroll
  for (int u = 0; u < TS; ++u) {
    tI[u] = tJ[u] = 0;
    if (!kF64 && wave + kVisWaves * u < ntiles) tile_ij(wave + kVisWaves * u, tI[u], tJ[u]);
  }
  // this lane's pixel (column x, row y) in the current chunk
  int xq = (p_beg + lane) % W.W, yq = (p_beg + lane) / W.W;
  const int g4 = lane >> 4, m16 = lane & 15;
  prefetch(p_beg);
  int nblk = 0;
  for (int c0 = p_beg, it = 0; c0 < p_end; c0 += 64, ++it) {
    const int buf = it & 1;
    R* E = Et + buf * tsz;
    const int p = c0 + lane;
    const bool inpx = p < p_end;
    const R qx = ((R)xq - cx) * ifx;
    const R qy = ((R)yq - cy) * ify;
    xq += 64;
    while (xq >= W.W) { xq -= W.W; ++yq; }
    const R d = (R)nd;
    float ctx_[SLOTS], cty[SLOTS], cwx[SLOTS], cwy[SLOTS];
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) { ctx_[u] = ntx[u]; cty[u] = nty[u]; cwx[u] = nwx[u]; cwy[u] = nwy[u]; }
    if (c0 + 64 < p_end) prefetch(c0 + 64);
    R Cp = (R)0, Wp = (R)0, cst = (R)0, nv = (R)0;
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int s = wave + kVisWaves * u;
      if (s < k) {
        if constexpr (kRegRel)
          vis_pair<R, LDC>(rtv[u], fx, fy, cx, cy, zmin, qx, qy, d, inpx, ctx_[u], cty[u], cwx[u], cwy[u],
                           acc[u], E + 6 * s * LDC + lane, Cp, Wp, cst, nv);
        else
          vis_pair<R, LDC>(rel_s + s * 12, fx, fy, cx, cy, zmin, qx, qy, d, inpx, ctx_[u], cty[u], cwx[u], cwy[u],
                           acc[u], E + 6 * s * LDC + lane, Cp, Wp, cst, nv);
      }
    }
    cost += (double)cst;
    nval += (double)nv;
    part[wave * 64 + lane] = Cp;
    part[kVisWaves * 64 + wave * 64 + lane] = Wp;
    const bool last = c0 + 64 >= p_end;
    const bool flush = last || (!kF64 && ++nblk == kVisBlockChunks);
    if (flush) {
      // per-edge block sums: reduce over the wave, add into the running sums
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        if (wave + kVisWaves * u < k) {
          R v[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) v[i] = acc[u].h[i];
          hs_a[u].add(reduce16(v, lane));
#pragma unroll
          for (int i = 0; i < 5; ++i) v[i] = acc[u].h[16 + i];
#pragma unroll
          for (int i = 0; i < 6; ++i) v[5 + i] = acc[u].g[i];
#pragma unroll
          for (int i = 11; i < 16; ++i) v[i] = (R)0;
          hs_b[u].add(reduce16(v, lane));
          acc[u].zero();
        }
      }
    }
    __syncthreads();
    if (wave == kVisSumWave) {
      // a non-finite inverse depth fails the window (the state is left as it is)
      if (st && inpx && !isfinite(d)) set_status(st + D.win_of_kf[src], VI_ENONFINITE, -1);
      double C = o.eta, Wv = 0.0;
#pragma unroll
      for (int q = 0; q < kVisWaves; ++q) {
        C += (double)part[q * 64 + lane];
        Wv += (double)part[kVisWaves * 64 + q * 64 + lane];
      }
      if (inpx) {
        Cds[p] = C;
        wds[p] = Wv;
      }
      invcd[buf * 64 + lane] = (inpx && C > 0.0) ? recip<R>((R)C) : (R)0;
      E[ncol * LDC + lane] = inpx ? (R)Wv : (R)0;
    }
    __syncthreads();
    // Gram of this chunk: lane (g4, m16) supplies pixels 16 g4 .. 16 g4 + 15
    {
      R inv[16];
      lds_load16(invcd + buf * 64 + 16 * g4, inv);
#pragma unroll
      for (int u = 0; u < TS; ++u) {
        const int t = wave + kVisWaves * u;
        if (t < ntiles) {
          // all 32 operands of the tile loaded first, B scaled by 1/C into its
          // own registers, then 16 back-to-back MFMAs
          int I = tI[u], J = tJ[u];
          if constexpr (kF64) tile_ij(t, I, J);
          if constexpr (kF64) {
            // in quarters of 4 k-steps: each quarter's 8 operands loaded and
            // scaled, then its 4 MFMAs (one LDS wait per quarter, bounded registers)
            const double* pa = E + (16 * I + m16) * LDC + 16 * g4;
            const double* pb = E + (16 * J + m16) * LDC + 16 * g4;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
              double q8[8];
              const double2_t* xa = (const double2_t*)(pa + 4 * qq);
              const double2_t* xb = (const double2_t*)(pb + 4 * qq);
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const double2_t va = xa[h], vb = xb[h];
                q8[2 * h] = va[0]; q8[2 * h + 1] = va[1];
                q8[4 + 2 * h] = vb[0] * inv[4 * qq + 2 * h]; q8[4 + 2 * h + 1] = vb[1] * inv[4 * qq + 2 * h + 1];
              }
              pin8(q8);
#pragma unroll
              for (int kk = 0; kk < 4; ++kk)
                gacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(q8[kk], q8[4 + kk], gacc[u], 0, 0, 0);
              __builtin_amdgcn_sched_barrier(0);
            }
          } else {
            R a[16], b[16];
            lds_load16(E + (16 * I + m16) * LDC + 16 * g4, a);
            lds_load16(E + (16 * J + m16) * LDC + 16 * g4, b);
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) b[kk] *= inv[kk];
            pin16(a);
            pin16(b);
#pragma unroll
            for (int kk = 0; kk < 16; ++kk)
              gblk[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[kk], gblk[u], 0, 0, 0);
          }
        }
      }
      if constexpr (!kF64) {
        if (flush) {
#pragma unroll
          for (int u = 0; u < TS; ++u) {
            const float4_t y = gblk[u] - gc[u];
            const float4_t tt = gs[u] + y;
            gc[u] = (tt - gs[u]) - y;
            gs[u] = tt;
            gblk[u] = float4_t{0.f, 0.f, 0.f, 0.f};
          }
        }
      }
    }
    if (flush) nblk = 0;
  }
  double* out = gpart + D.gram_off[src] + (size_t)kr * ntiles * 256;
#pragma unroll
  for (int u = 0; u < TS; ++u) {
    const int t = wave + kVisWaves * u;
    if (t < ntiles) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = lane & 15;
        if constexpr (kF64) {
          const int m = (lane >> 4) + 4 * r;
          out[(size_t)t * 256 + m * 16 + n] = gacc[u][r];
        } else {
          const int m = 4 * (lane >> 4) + r;
          out[(size_t)t * 256 + m * 16 + n] = (double)gs[u][r] - (double)gc[u][r];
        }
      }
    }
  }
  // per-edge partials: lane l holds element l >> 2 of each 16-value half
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int s = wave + kVisWaves * u;
    if (s < k && (lane & 3) == 0) {
      double* hp = hpart + ((size_t)(e0 + s) * nkr_max + kr) * 32;
      const int el = lane >> 2;
      hp[el] = hs_a[u].value();
      if (el < 11) hp[16 + el] = hs_b[u].value();
    }
  }
  cost = wave_sum(cost);
  nval = wave_sum(nval);
  if (lane == 0) { red[0][wave] = cost; red[1][wave] = nval; }
  __syncthreads();
  if (tid == 0) {
    double c = 0.0, nv = 0.0;
#pragma unroll
    for (int q = 0; q < kVisWaves; ++q) { c += red[0][q]; nv += red[1][q]; }
    const size_t b = ((size_t)src * ncost + kr) * 2;
    vcost[b] = c;
    vcost[b + 1] = nv;
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
// of every pixel range are summed straight into LDS first.  Extra workgroups
// (one per window) reduce the cost partials into the window's cost trace.
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

// With the camera-IMU extrinsic the unknowns are body increments; the camera
// moves by K (dtheta, dp) with K = [[R_bc^T, 0], [-R_b [t_bc]x, I]] and
// R_b = R_c R_bc^T, so the local maps become M K.  Rc: the camera rotation.
// W is the window in device memory (indexed reads, no private copies).
__device__ __forceinline__ double skew_at(const double* t, int q, int c) {
  // [t]x = [[0, -t2, t1], [t2, 0, -t0], [-t1, t0, 0]]
  if (q == c) return 0.0;
  const double v = t[3 - q - c];
  return ((q + 1) % 3 == c) ? -v : v;
}

__device__ __forceinline__ double K_at(const WinDev& W, const double* Rc, int m, int c) {
  if (m < 3) return c < 3 ? W.Rbc[c * 3 + m] : 0.0;
  if (c >= 3) return (m == c) ? 1.0 : 0.0;
  // -(R_b [t]x)[m-3][c], R_b[p][q] = sum_u Rc[p][u] Rbc[q][u]
  double v = 0.0;
  for (int q = 0; q < 3; ++q) {
    double rb = 0.0;
    for (int u = 0; u < 3; ++u) rb += Rc[(m - 3) * 3 + u] * W.Rbc[q * 3 + u];
    v += rb * skew_at(W.tbc, q, c);
  }
  return -v;
}

__device__ __forceinline__ double Mi_body(const WinDev& W, const double* Rt, const double* Rj, const double* Rci,
                                          int r, int c) {
  if (c >= 3) return Mi_at(Rt, Rj, r, c);
  double v = 0.0;
  for (int m = 0; m < 6; ++m) v += Mi_at(Rt, Rj, r, m) * K_at(W, Rci, m, c);
  return v;
}

// M_j K_j = [[-R_bc^T, 0], [R_bc^T [t_bc]x, -R_j^T]] (R_j: the camera rotation)
__device__ __forceinline__ double Mj_body(const WinDev& W, const double* Rj, int r, int c) {
  if (r < 3) return c < 3 ? -W.Rbc[c * 3 + r] : 0.0;
  if (c >= 3) return -Rj[(c - 3) * 3 + (r - 3)];
  double v = 0.0;
  for (int q = 0; q < 3; ++q) v += W.Rbc[q * 3 + (r - 3)] * skew_at(W.tbc, q, c);
  return v;
}

// cost trace of window w: sum of its vision partials (ranges of range_px pixels
// per source keyframe) and of its inertial factor costs.  Any power-of-two
// block size; s0 holds 2 * blockDim.x doubles.
__device__ void cost_reduce_block(const WinDev& W, int w, int ncost, int range_px, const double* __restrict__ vcost,
                                  const double* __restrict__ icost, int use_imu, double* __restrict__ trace,
                                  int slot, double* s0) {
  const int nt = blockDim.x;
  double* s1 = s0 + nt;
  const int t = threadIdx.x;
  const int nk = (W.HW + range_px - 1) / range_px;
  double c = 0.0, n = 0.0;
  for (int i = t; i < W.N * nk; i += nt) {
    const size_t b = ((size_t)(W.kf_base + i / nk) * ncost + i % nk) * 2;
    c += vcost[b];
    n += vcost[b + 1];
  }
  if (use_imu)
    for (int i = t; i < W.F; i += nt) c += icost[W.f_base + i];
  s0[t] = c;
  s1[t] = n;
  __syncthreads();
  for (int q = nt / 2; q > 0; q >>= 1) {
    if (t < q) { s0[t] += s0[t + q]; s1[t] += s1[t + q]; }
    __syncthreads();
  }
  if (t == 0) {
    trace[(size_t)w * kTraceLen + 2 * slot] = s0[0];
    trace[(size_t)w * kTraceLen + 2 * slot + 1] = s1[0];
  }
}

// Sums of n partials for NS streams at once, s-th stream p[s][0], p[s][stride[s]],
// ..., each in order of its index: U partials of every stream are loaded per
// round (clamped in range and masked), so that NS x U loads are in flight
// before the first one returns.
template <int U, int NS>
__device__ __forceinline__ void sum_partials(const double* const (&p)[NS], const size_t (&stride)[NS], int n,
                                             double (&out)[NS]) {
#pragma unroll
  for (int q = 0; q < NS; ++q) out[q] = 0.0;
  for (int r0 = 0; r0 < n; r0 += U) {
    double v[NS][U];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) v[q][u] = p[q][(size_t)min(r0 + u, n - 1) * stride[q]];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) out[q] += (r0 + u < n) ? v[q][u] : 0.0;
  }
}

constexpr int kLocalThreads = 1024;

__global__ void __launch_bounds__(kLocalThreads) k_local(int N, int nkr_max, int ncost, int range, DevPlan D,
                                                         const double* __restrict__ Rw, const double* __restrict__ rel,
                                                         const double* __restrict__ hpart,
                                                         const double* __restrict__ gpart, double* __restrict__ Z,
                                                         double* __restrict__ ZB, double* __restrict__ ZV,
                                                         const double* __restrict__ vcost,
                                                         const double* __restrict__ icost, int use_imu,
                                                         double* __restrict__ trace, int slot, double tol,
                                                         DevStatus* __restrict__ st) {
  extern __shared__ double sm[];
  if ((int)blockIdx.x >= N) {
    const int w = blockIdx.x - N;
    cost_reduce_block(D.win[w], w, ncost, range, vcost, icost, use_imu, trace, slot, sm);
    // tolerance stop: F at this linearisation point against the previous one
    // (written by this same thread); once the relative decrease is at most tol
    // the window takes no further step
    if (threadIdx.x == 0 && st && tol > 0.0 && slot > 0) {
      const double prev = trace[(size_t)w * kTraceLen + 2 * (slot - 1)];
      const double cur = trace[(size_t)w * kTraceLen + 2 * slot];
      if (!(prev - cur > tol * prev)) st[w].conv = 1;
    }
    return;
  }
  const int src = blockIdx.x;
  const WinDev& Wsrc = D.win[D.win_of_kf[src]];
  const int nkr = Wsrc.nkr;
  const bool ext = Wsrc.ext != 0;     // camera-IMU extrinsic: general M_j (else its block structure is used)
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int tid = threadIdx.x;
  constexpr int NT = kLocalThreads;
  const int K1 = k + 1;
  double* Zs = Z + D.z_off[src];
  double* ZBs = ZB + D.zb_off[src];
  double* ZVs = ZV + D.zb_off[src];
  if (k == 0) {
    for (int i = tid; i < 36; i += NT) Zs[i] = 0.0;
    for (int i = tid; i < 6; i += NT) { ZBs[i] = 0.0; ZVs[i] = 0.0; }
    return;
  }
  const int ncol = 6 * k, nq = ncol + 1;
  const int T = (ncol + 16) / 16;
  const int ntiles = T * (T + 1) / 2;
  double* Qs = sm;                  // [nq][nq] symmetric
  double* Mi = Qs + nq * nq;        // [k][36]  M_i of edge s (with the extrinsic: M_i K_i)
  double* Rj = Mi + 36 * k;         // [k][9]   R_j of edge s (M_j = -blockdiag(I, R_j^T))
  double* Mj = Rj + 9 * k;          // [k][36]  M_j K_j (with the extrinsic only)
  double* Hs = Mj + 36 * k;         // [k][36]  full symmetric
  double* gs = Hs + 36 * k;         // [k][6]   g - y
  double* Wt = gs + 6 * k;          // [k][36]
  // Gram partials -> Q.  The lower tiles hold the data; the lower triangle is
  // mirrored into both halves (inside a diagonal tile the MFMA result is not
  // exactly symmetric, so only its a >= b entries are used: one writer per slot).
  const double* gp = gpart + D.gram_off[src];
  const size_t gstride = (size_t)ntiles * 256;
  const int nent = ntiles * 256;
  // Every thread first forms all the sums it owns in a pass (four Gram
  // entries; in the first pass also one edge-Hessian entry and one gradient
  // entry), so that the partial loads of all of them are in flight together,
  // and then writes them to LDS.  One pass covers up to 12 edges.
  const bool own_h = tid < k * 36, own_g = tid < k * 6;
  for (int base = 0; base < nent; base += 4 * NT) {
    const bool first = base == 0;
    // streams: four Gram entries, one edge-Hessian entry, one gradient entry
    // (the last two only in the first pass; else they repeat the first stream)
    const double* ps[6];
    size_t strd[6];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      ps[h] = gp + min(base + tid + h * NT, nent - 1);
      strd[h] = gstride;
    }
    ps[4] = ps[5] = ps[0];
    strd[4] = strd[5] = gstride;
    if (first && own_h) {
      const int rc = tid % 36, r = rc / 6, c = rc % 6;
      const int a = min(r, c), b = max(r, c);
      const int qq = a * 6 - a * (a - 1) / 2 + (b - a);
      ps[4] = hpart + (size_t)(e0 + tid / 36) * nkr_max * 32 + qq;
      strd[4] = 32;
    }
    if (first && own_g) {
      ps[5] = hpart + (size_t)(e0 + tid / 6) * nkr_max * 32 + 21 + tid % 6;
      strd[5] = 32;
    }
    double sums[6];
    sum_partials<4, 6>(ps, strd, nkr, sums);
    double vq[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) vq[h] = sums[h];
    const double vh = sums[4], vg = sums[5];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int i = base + tid + h * NT;
      if (i >= nent) continue;
      const int t = i >> 8, e = i & 255;
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      const int J = t - I * (I + 1) / 2;
      const int a = 16 * I + (e >> 4), b = 16 * J + (e & 15);
      if (a < nq && b < nq && a >= b) {
        Qs[a * nq + b] = vq[h];
        Qs[b * nq + a] = vq[h];
      }
    }
    if (first && own_h) {
      const int hs_s = tid / 36, rc = tid % 36;
      const int e = D.src_edges[e0 + hs_s];
      const double* Rt = rel + (size_t)e * 12;
      const double* Rjs = Rw + (size_t)D.jj[e] * 9;
      if (!ext) Mi[tid] = Mi_at(Rt, Rjs, rc / 6, rc % 6);
      if (rc < 9) Rj[hs_s * 9 + rc] = Rjs[rc];
      Hs[tid] = vh;
    }
    if (first && own_g) gs[tid] = vg;
  }
  if (ext) {
    // the maps of body increments, M_i K_i and M_j K_j (a pass of its own,
    // after the partial sums' registers are free)
    for (int i = tid; i < 36 * k; i += NT) {
      const int s2 = i / 36, rc = i % 36;
      const int e = D.src_edges[e0 + s2];
      const double* Rjs = Rw + (size_t)D.jj[e] * 9;
      Mi[i] = Mi_body(Wsrc, rel + (size_t)e * 12, Rjs, Rw + (size_t)src * 9, rc / 6, rc % 6);
      Mj[i] = Mj_body(Wsrc, Rjs, rc / 6, rc % 6);
    }
  }
  __syncthreads();
  for (int i = tid; i < k * 6; i += NT) gs[i] -= Qs[ncol * nq + i];
  // W_t = sum_s M_i,s^T X_st,  X_st = delta_st H_s - Q_st
  for (int i = tid; i < k * 36; i += NT) {
    const int t = i / 36, a = (i % 36) / 6, b = i % 6;
    double v = 0.0;
    for (int s2 = 0; s2 < k; ++s2) {
      const double* Ms = Mi + s2 * 36;
      const double* Qr = Qs + (6 * s2) * nq + 6 * t + b;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        double x = -Qr[m * nq];
        if (s2 == t) x += Hs[s2 * 36 + m * 6 + b];
        v += Ms[m * 6 + a] * x;
      }
    }
    Wt[i] = v;
  }
  // Z_s+1,t+1 = M_j,s^T X_st M_j,t; without the extrinsic M_j = -P with
  // P = blockdiag(I, R_j^T): [[X11, X12 R_t^T], [R_s X21, R_s X22 R_t^T]]
  // Four waves per quadrant of the 6x6 blocks (a < 3 or not, b < 3 or not), so
  // that the lanes of a wave take the same branch below: in each quadrant 28
  // groups of 9 lanes (one lane per entry of the 3x3 quadrant) walk the block
  // pairs st = s k + t, 28 apart (no integer division in the walk)
  static_assert(NT == 1024, "four waves per quadrant");
  const int quad = tid >> 8, lt = tid & 255, grp = lt / 9, ab = lt % 9;
  const int a = ab / 3 + 3 * (quad >> 1), b = ab % 3 + 3 * (quad & 1);
  int s2 = grp / k, t = grp % k;
  for (int st = grp; grp < 28 && st < k * k; st += 28) {
    const double* Qb = Qs + (6 * s2) * nq + 6 * t;
    const bool diag = s2 == t;
    const double* Hb = Hs + s2 * 36;
    auto X = [&](int m, int n) { return (diag ? Hb[m * 6 + n] : 0.0) - Qb[m * nq + n]; };
    double v = 0.0;
    if (ext) {
      // general M_j (its upper-right 3x3 block is zero: zero entries skipped)
      const double* Ms = Mj + s2 * 36;
      const double* Mt = Mj + t * 36;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const double ma = Ms[m * 6 + a];
        if (ma == 0.0) continue;
        double u = 0.0;
#pragma unroll
        for (int n = 0; n < 6; ++n) {
          const double mb = Mt[n * 6 + b];
          if (mb != 0.0) u += X(m, n) * mb;
        }
        v += ma * u;
      }
    } else {
      const double* Rs = Rj + s2 * 9;
      const double* Rt = Rj + t * 9;
      if (a < 3 && b < 3) {
        v = X(a, b);
      } else if (a < 3) {
#pragma unroll
        for (int n = 0; n < 3; ++n) v += X(a, 3 + n) * Rt[(b - 3) * 3 + n];
      } else if (b < 3) {
#pragma unroll
        for (int m = 0; m < 3; ++m) v += Rs[(a - 3) * 3 + m] * X(3 + m, b);
      } else {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          double u = 0.0;
#pragma unroll
          for (int n = 0; n < 3; ++n) u += X(3 + m, 3 + n) * Rt[(b - 3) * 3 + n];
          v += Rs[(a - 3) * 3 + m] * u;
        }
      }
    }
    Zs[(size_t)((s2 + 1) * K1 + t + 1) * 36 + a * 6 + b] = v;
    t += 28;
    while (t >= k) {
      t -= k;
      ++s2;
    }
  }
  __syncthreads();
  // Z_0,t+1 = W_t M_j,t (= -W_t P_t without the extrinsic) and its transpose;
  // Z_00 = sum_t W_t M_i,t
  for (int i = tid; i < k * 36; i += NT) {
    const int t = i / 36, a = (i % 36) / 6, b = i % 6;
    const double* Wb = Wt + t * 36 + a * 6;
    double v = 0.0;
    if (ext) {
      const double* Mt = Mj + t * 36;
#pragma unroll
      for (int n = 0; n < 6; ++n) v += Wb[n] * Mt[n * 6 + b];
    } else if (b < 3) {
      v = -Wb[b];
    } else {
      const double* Rt = Rj + t * 9;
      v = -(Wb[3] * Rt[(b - 3) * 3 + 0] + Wb[4] * Rt[(b - 3) * 3 + 1] + Wb[5] * Rt[(b - 3) * 3 + 2]);
    }
    Zs[(size_t)(0 * K1 + t + 1) * 36 + a * 6 + b] = v;
    Zs[(size_t)((t + 1) * K1 + 0) * 36 + b * 6 + a] = v;
  }
  // per-edge terms of Z_00 = sum_t W_t M_i,t and of the first block row of
  // the diagonal / right-hand side (sum_s M_i,s^T H_s M_i,s, M_i,s^T (g - y)),
  // into the Gram's LDS area (no longer needed), then summed over the edges
  // in order
  double* scr = Qs;
  for (int i = tid; i < k * 36; i += NT) {
    const int t = i / 36, a = (i % 36) / 6, b = i % 6;
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) v += Wt[t * 36 + a * 6 + m] * Mi[t * 36 + m * 6 + b];
    scr[i] = v;
  }
  for (int i = tid; i < k * 6; i += NT) {
    const int s2 = i / 6, a = i % 6;
    const double* M = Mi + s2 * 36;
    double zb = 0.0, zv = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double hm = 0.0;
#pragma unroll
      for (int nn = 0; nn < 6; ++nn) hm += Hs[s2 * 36 + m * 6 + nn] * M[nn * 6 + a];
      zb += M[m * 6 + a] * hm;
      zv += M[m * 6 + a] * gs[s2 * 6 + m];
    }
    scr[k * 36 + 2 * i] = zb;
    scr[k * 36 + 2 * i + 1] = zv;
  }
  __syncthreads();
  for (int i = tid; i < 36; i += NT) {
    double v = 0.0;
    for (int t = 0; t < k; ++t) v += scr[t * 36 + i];
    Zs[i] = v;
  }
  for (int i = tid; i < 6 * K1; i += NT) {
    const int ra = i / 6, a = i % 6;
    double zb = 0.0, zv = 0.0;
    if (ra == 0) {
      for (int s2 = 0; s2 < k; ++s2) {
        zb += scr[k * 36 + 2 * (s2 * 6 + a)];
        zv += scr[k * 36 + 2 * (s2 * 6 + a) + 1];
      }
    } else if (ext) {
      // diag(M_j^T H M_j) and M_j^T (g - y)
      const int s2 = ra - 1;
      const double* H = Hs + s2 * 36;
      const double* g = gs + s2 * 6;
      const double* M = Mj + s2 * 36;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        double hm = 0.0;
#pragma unroll
        for (int nn = 0; nn < 6; ++nn) hm += H[m * 6 + nn] * M[nn * 6 + a];
        zb += M[m * 6 + a] * hm;
        zv += M[m * 6 + a] * g[m];
      }
    } else {
      // M_j = -P: diag(P^T H P) and -P^T (g - y)
      const int s2 = ra - 1;
      const double* H = Hs + s2 * 36;
      const double* g = gs + s2 * 6;
      if (a < 3) {
        zb = H[a * 6 + a];
        zv = -g[a];
      } else {
        const double* R = Rj + s2 * 9 + (a - 3) * 3;   // row a-3 of R_j: P[3+m][a] = R_j[a-3][m]
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          double hm = 0.0;
#pragma unroll
          for (int nn = 0; nn < 3; ++nn) hm += H[(3 + m) * 6 + 3 + nn] * R[nn];
          zb += R[m] * hm;
          zv -= R[m] * g[3 + m];
        }
      }
    }
    ZBs[i] = zb;
    ZVs[i] = zv;
  }
}

// ---------------------------------------------------------------------------
// reduced system of each window (blockIdx.y): one lane per entry of the
// (npad + NB) x npad matrix whose leading n x n block is S (damped, gauge and
// inactive rows replaced by identity), whose row npad is the right-hand side s
// (so the Cholesky forward pass produces L^-1 s in that row), and whose
// padding is the identity.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool coord_active(const OptsDev& o, int a, int ra, int N) {
  if (ra < 6) return a >= o.n_fixed;
  if (!o.use_imu) return false;
  if (ra >= 9 && o.bias_fixed) return false;
  if (ra >= 9 && o.bias_global) return a == N - 1;   // the shared bias sits in the last keyframe's slot
  return true;
}

// inertial part of the entry ((a, ra), (b, cb)) of B: the blocks of the
// factors (a - 1, a) and (a, a + 1) of the window (Hw: [F][30][30])
__device__ __forceinline__ double imu_hess(const double* Hw, int N, int a, int ra, int b, int cb) {
  double v = 0.0;
  if (a == b) {
    if (a > 0) v += Hw[(size_t)(a - 1) * 900 + (15 + ra) * 30 + 15 + cb];
    if (a < N - 1) v += Hw[(size_t)a * 900 + ra * 30 + cb];
  } else if (b == a + 1) {
    v += Hw[(size_t)a * 900 + ra * 30 + 15 + cb];
  } else if (a == b + 1) {
    v += Hw[(size_t)b * 900 + (15 + ra) * 30 + cb];
  }
  return v;
}

// inertial part of w_xi at (b, cb) (gw: [F][30])
__device__ __forceinline__ double imu_grad(const double* gw, int N, int b, int cb) {
  double v = 0.0;
  if (b > 0) v += gw[(size_t)(b - 1) * 30 + 15 + cb];
  if (b < N - 1) v += gw[(size_t)b * 30 + cb];
  return v;
}

// The same entries with one bias for the window (Table 6 (f)): the bias
// coordinates of every keyframe are the one unknown in the last keyframe's
// slot, so the folded system G^T B G sums an entry over the keyframes whose
// bias it touches (those of the inertial factors next to the other index)
__device__ double imu_hess_folded(const double* Hw, int N, int a, int ra, int b, int cb, bool global) {
  const bool ga = global && ra >= 9, gb = global && cb >= 9;
  if (!ga && !gb) return imu_hess(Hw, N, a, ra, b, cb);
  double v = 0.0;
  if (ga && gb) {
    for (int f = 0; f < N - 1; ++f) {
      const double* H = Hw + (size_t)f * 900;
      v += H[ra * 30 + cb] + H[ra * 30 + 15 + cb] + H[(15 + ra) * 30 + cb] + H[(15 + ra) * 30 + 15 + cb];
    }
  } else if (gb) {
    for (int b2 = max(a - 1, 0); b2 <= min(a + 1, N - 1); ++b2) v += imu_hess(Hw, N, a, ra, b2, cb);
  } else {
    for (int a2 = max(b - 1, 0); a2 <= min(b + 1, N - 1); ++a2) v += imu_hess(Hw, N, a2, ra, b, cb);
  }
  return v;
}

__device__ double imu_grad_folded(const double* gw, int N, int b, int cb, bool global) {
  if (!(global && cb >= 9)) return imu_grad(gw, N, b, cb);
  double v = 0.0;
  for (int b2 = 0; b2 < N; ++b2) v += imu_grad(gw, N, b2, cb);
  return v;
}

__global__ void k_assemble(OptsDev o, DevPlan D, const double* __restrict__ Z, const double* __restrict__ ZB,
                           const double* __restrict__ ZV, const double* __restrict__ Hf,
                           const double* __restrict__ gf, double* __restrict__ A, int* __restrict__ flags,
                           int* __restrict__ sync, DevStatus* st) {
  const int w = blockIdx.y;
  const WinDev& W = D.win[w];
  const int N = W.N, n = W.n, npad = W.npad;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)(npad + kCholNB) * npad;
  // the Cholesky tile flags and ticket counter start from zero
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
  const double* Hw = Hf + (size_t)W.f_base * 900;
  const double* gw = gf + (size_t)W.f_base * 30;
  const int* poff = D.pair_off + W.pair_base;
  double val = 0.0;
  if (r < n && c < n) {
    // block positions -> keyframes (the window's order of the reduced system)
    const int a = D.kf_at[W.kf_base + r / 15], ra = r % 15, b = D.kf_at[W.kf_base + c / 15], cb = c % 15;
    if (coord_active(o, a, ra, N) && coord_active(o, b, cb, N)) {
      double bd = 0.0;
      if (ra < 6 && cb < 6) {
        // the pair blocks of (a, b) in list order, eight gathers in flight
        const int p0 = poff[a * N + b], p1 = poff[a * N + b + 1];
        for (int it0 = p0; it0 < p1; it0 += 8) {
          int iz[8], ib[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int it = min(it0 + u, p1 - 1);
            iz[u] = D.pair_z[it];
            ib[u] = D.pair_zb[it];
          }
          double vz[8], vb[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            vz[u] = Z[iz[u] + ra * 6 + cb];
            vb[u] = (r == c) ? ZB[ib[u] + ra] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (it0 + u < p1) {
              val += vz[u];
              bd += vb[u];
            }
        }
      }
      if (o.use_imu) {
        const double vi = imu_hess_folded(Hw, N, a, ra, b, cb, o.bias_global != 0);
        val += vi;
        if (r == c) bd += vi;
      }
      if (r == c) val += o.lambda * bd;
    } else {
      val = (r == c) ? 1.0 : 0.0;
    }
    if (!isfinite(val)) set_status(st + w, VI_ENONFINITE, 15 * a + ra);
  } else if (r < npad) {
    val = (r == c) ? 1.0 : 0.0;
  } else if (r == npad && c < n) {
    const int b = D.kf_at[W.kf_base + c / 15], cb = c % 15;
    if (coord_active(o, b, cb, N)) {
      if (cb < 6) {
        const int p0 = poff[b * N + b], p1 = poff[b * N + b + 1];
        for (int it0 = p0; it0 < p1; it0 += 8) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = ZV[D.pair_zb[min(it0 + u, p1 - 1)] + cb];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (it0 + u < p1) val += v[u];
        }
      }
      if (o.use_imu) val += imu_grad_folded(gw, N, b, cb, o.bias_global != 0);
    }
    if (!isfinite(val)) set_status(st + w, VI_ENONFINITE, n + 15 * b + cb);
  }
  A[W.A_off + idx] = val;
}

// ---------------------------------------------------------------------------
// back-substitution (Eq. 4: dd = C^-1 (w_d - E^T dxi)) and retraction.  The
// E^T dxi term is L_p . u with u_e = M_i,e dxi_i + M_j,e dxi_j (pose parts),
// the local increment of each edge; L_p is recomputed from the weights and the
// Jacobians (cheaper than storing it).  Workgroups with blockIdx.y >= N retract
// the keyframe states of window blockIdx.y - N.  A window whose status holds
// an error is left untouched.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_backsub_retract(OptsDev o, int N, DevPlan D, const double* __restrict__ Rw,
                                                         const double* __restrict__ rel,
                                                         const double* __restrict__ Cd,
                                                         const double* __restrict__ wd,
                                                         const double* __restrict__ x, int ppt, DevStatus* st) {
  __shared__ double u[kMaxOutDegree * 6];
  __shared__ double rel_s[kMaxOutDegree * 12];
  __shared__ double xcam[(kMaxOutDegree + 1) * 6];
  const int tid = threadIdx.x;
  if ((int)blockIdx.y >= N) {
    const int w = blockIdx.y - N;
    if (blockIdx.x != 0 || st[w].code != 0 || st[w].conv != 0) return;
    const WinDev& W = D.win[w];
    const double* xw = x + W.x_off;
    // one bias for the window: its increment (the last keyframe's slot) moves every keyframe's
    const double* dxb = o.bias_global ? xw + (size_t)D.kf_pos[W.kf_base + W.N - 1] * 15 : nullptr;
    for (int t = tid; t < W.N; t += 256) {
      const double* dx = xw + (size_t)D.kf_pos[W.kf_base + t] * 15;
      const double* db = dxb ? dxb + 9 : dx + 9;
      double* q = W.pose + (size_t)t * 7;
      quat_retract(q + 3, dx);
      for (int k = 0; k < 3; ++k) {
        q[k] += dx[3 + k];
        W.vel[(size_t)t * 3 + k] += dx[6 + k];
      }
      for (int k = 0; k < 6; ++k) W.bias[(size_t)t * 6 + k] += db[k];
      if (W.rep_dxi) {
        for (int k = 0; k < 9; ++k) W.rep_dxi[(size_t)t * 15 + k] = dx[k];
        for (int k = 0; k < 6; ++k) W.rep_dxi[(size_t)t * 15 + 9 + k] = db[k];
      }
    }
    if (tid == 0) st[w].iters += 1;
    return;
  }
  const int src = blockIdx.y;
  const int w = D.win_of_kf[src];
  const WinDev W = D.win[w];
  const int HW = W.HW;
  if (st[w].code != 0 || st[w].conv != 0 || (int)blockIdx.x * 256 * ppt >= HW) return;
  const int ls = src - W.kf_base;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const double* xw = x + W.x_off;
  for (int i = tid; i < 12 * k; i += 256) rel_s[i] = rel[(size_t)D.src_edges[e0 + i / 12] * 12 + i % 12];
  if (W.ext) {
    // the body increments of the source (slot 0) and of the targets as
    // camera increments, K x (W.ext is uniform over the workgroup)
    const WinDev& Wg = D.win[w];
    for (int i = tid; i < 6 * (k + 1); i += 256) {
      const int s = i / 6, c = i % 6;
      const int kf = s == 0 ? src : D.jj[D.src_edges[e0 + s - 1]];
      const double* Rc = Rw + (size_t)kf * 9;
      const double* xb = xw + (size_t)D.kf_pos[kf] * 15;
      double v = 0.0;
      for (int m = 0; m < 6; ++m) v += K_at(Wg, Rc, c, m) * xb[m];
      xcam[i] = v;
    }
    __syncthreads();
  }
  for (int i = tid; i < 6 * k; i += 256) {
    const int s = i / 6, c = i % 6;
    const int e = D.src_edges[e0 + s];
    const double* Rt = rel + (size_t)e * 12;
    const double* Rj = Rw + (size_t)D.jj[e] * 9;
    const double* xi = W.ext ? xcam : xw + (size_t)D.kf_pos[src] * 15;
    const double* xj = W.ext ? xcam + 6 * (s + 1) : xw + (size_t)D.kf_pos[D.jj[e]] * 15;
    double v = 0.0;
    for (int m = 0; m < 6; ++m) v += Mi_at(Rt, Rj, c, m) * xi[m] + Mj_at(Rj, c, m) * xj[m];
    u[i] = v;
  }
  __syncthreads();
  // ppt pixels per thread, 256 apart (the setup above is shared by all of them)
  for (int j = 0; j < ppt; ++j) {
    const int p = (blockIdx.x * ppt + j) * 256 + tid;
    if (p >= HW) break;
    const size_t pl = (size_t)ls * HW + p;
    const size_t pi = W.pix_base + pl;
    const double cd = Cd[pi];
    const double d = dep_load(W, pl);
    double ddv = 0.0;
    if (cd > 0.0 && k > 0) {
      // E^T dxi at this pixel: sum over edges of L_e,p . u_e, with L = J_loc^T W J_d
      const R qx = (R)(((double)(p % W.W) - W.cx) / W.fx);
      const R qy = (R)(((double)(p / W.W) - W.cy) / W.fy);
      R et = (R)0;
      // edges in groups of 4 with all their weight loads issued first
      for (int s0 = 0; s0 < k; s0 += 4) {
        float wgx[4], wgy[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int s = min(s0 + g, k - 1);
          const size_t t = (size_t)(D.src_edges[e0 + s] - W.e_base) * 2 * HW + p;
          wgx[g] = W.weight[t];
          wgy[g] = W.weight[t + HW];
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int s = s0 + g;
          if (s < k) {
            PixEdgeT<R> q;
            pix_edge_v<R>(W, o, rel_s + s * 12, qx, qy, (R)d, true, 0.0f, 0.0f, wgx[g], wgy[g], false, q);
            const R ax = q.wx * q.Jdx, ay = q.wy * q.Jdy;
#pragma unroll
            for (int c = 0; c < 6; ++c) et += (ax * q.Jx[c] + ay * q.Jy[c]) * (R)u[s * 6 + c];
          }
        }
      }
      ddv = (double)(((R)wd[pi] - et) / (R)cd);
    }
    dep_store(W, pl, fmax(d + ddv, o.d_min));
    if (W.rep_dd) W.rep_dd[pl] = ddv;
  }
}

__global__ void k_reset_status(DevStatus* st, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { st[i].code = 0; st[i].detail = 0; st[i].iters = 0; st[i].conv = 0; }
}

// ---------------------------------------------------------------------------
// cost at the current state (residuals only)
// ---------------------------------------------------------------------------
// corrected inverse depth of pixel p of keyframe src (up4 of its cell grid)
__device__ __forceinline__ double warm_corrected_depth(const WinDev& W, int src, int p, int HQ, int WQ,
                                                       const float* __restrict__ dd, double d, double d_min) {
  const int hq0 = (W.H + 3) / 4, wq0 = (W.W + 3) / 4;
  const float* g = dd + (size_t)src * HQ * WQ;
  const int y = p / W.W, x = p % W.W;
  const double fy = fmin(fmax((y - 1.5) / 4.0, 0.0), hq0 - 1.0);
  const double fx = fmin(fmax((x - 1.5) / 4.0, 0.0), wq0 - 1.0);
  const int y0 = (int)floor(fy), x0 = (int)floor(fx);
  const int y1 = min(y0 + 1, hq0 - 1), x1 = min(x0 + 1, wq0 - 1);
  const double ay = fy - y0, ax = fx - x0;
  const double v = (1 - ay) * ((1 - ax) * g[y0 * WQ + x0] + ax * g[y0 * WQ + x1]) +
                   ay * ((1 - ax) * g[y1 * WQ + x0] + ax * g[y1 * WQ + x1]);
  return fmax(d + v, d_min);
}

template <typename R>
// With dd set, the warm-start corrections are applied first (each workgroup to
// its own pixels, workgroup 0 of a keyframe to its bias) and the cost is that
// of the corrected state.
__global__ void __launch_bounds__(256) k_vis_cost(OptsDev o, DevPlan D, int ncost, double* __restrict__ vcost,
                                                  const float* __restrict__ dd, const float* __restrict__ db, int HQ,
                                                  int WQ, double d_min) {
  __shared__ double red[2][4];
  __shared__ double rel[kMaxOutDegree * 12];
  const int src = blockIdx.y, kr = blockIdx.x;
  const WinDev W = D.win[D.win_of_kf[src]];
  const int HW = W.HW;
  if (kr * kVisBlock >= HW) return;
  const int ls = src - W.kf_base;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < k) edge_rel(W, ls, D.jj[D.src_edges[e0 + tid]] - W.kf_base, rel + tid * 12);
  __syncthreads();
  const int p = kr * kVisBlock + tid;
  const bool inpx = p < HW;
  const int pc = inpx ? p : 0;
  const R qx = (R)(((double)(pc % W.W) - W.cx) / W.fx);
  const R qy = (R)(((double)(pc / W.W) - W.cy) / W.fy);
  double dsrc = dep_load(W, (size_t)ls * HW + pc);
  if (dd) {
    if (inpx) {
      dsrc = warm_corrected_depth(W, src, pc, HQ, WQ, dd, dsrc, d_min);
      dep_store(W, (size_t)ls * HW + pc, dsrc);
      dsrc = dep_load(W, (size_t)ls * HW + pc);   // the stored value (rounded when FP32)
    }
    // biases that the step does not solve (no inertial terms, or held fixed) keep their value
    if (kr == 0 && tid < 6 && o.use_imu && !o.bias_fixed) W.bias[(size_t)ls * 6 + tid] += (double)db[(size_t)src * 6 + tid];
  }
  const R d = (R)dsrc;
  const R fx = (R)W.fx, fy = (R)W.fy, cx = (R)W.cx, cy = (R)W.cy;
  double cost = 0.0, nval = 0.0;
  // edges in groups of 4 with all their target and weight loads issued first
  // (the sums still run over the edges in order)
  for (int s0 = 0; s0 < k; s0 += 4) {
    float tgx[4], tgy[4], wgx[4], wgy[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int e = D.src_edges[e0 + min(s0 + g, k - 1)];
      const size_t toff = (size_t)(e - W.e_base) * 2 * HW + pc;
      tgx[g] = W.target[toff];
      tgy[g] = W.target[toff + HW];
      wgx[g] = W.weight[toff];
      wgy[g] = W.weight[toff + HW];
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int s = s0 + g;
      if (s >= k) break;
      R Rt[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) Rt[c] = (R)rel[s * 12 + c];
      const R Px = Rt[0] * qx + Rt[1] * qy + Rt[2] + Rt[9] * d;
      const R Py = Rt[3] * qx + Rt[4] * qy + Rt[5] + Rt[10] * d;
      const R Pz = Rt[6] * qx + Rt[7] * qy + Rt[8] + Rt[11] * d;
      const bool valid = inpx && d > (R)0 && Pz > (R)o.z_min * d;
      if (valid) {
        const R iz = recip<R>(Pz);
        const R rx = (R)tgx[g] - (fx * Px * iz + cx);
        const R ry = (R)tgy[g] - (fy * Py * iz + cy);
        cost += (double)((R)wgx[g] * rx * rx + (R)wgy[g] * ry * ry);
        nval += 1.0;
      }
    }
  }
  cost = wave_sum(cost);
  nval = wave_sum(nval);
  if (lane == 0) { red[0][wave] = cost; red[1][wave] = nval; }
  __syncthreads();
  if (tid == 0) {
    const size_t b = ((size_t)src * ncost + kr) * 2;
    vcost[b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    vcost[b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// r^T Lambda r per inertial factor, one wave per factor: every lane forms the
// residual (the same values), lane a < 15 takes row a of the quadratic form
// (its 15 loads in flight together), the wave sums the rows.
__global__ void __launch_bounds__(256) k_imu_cost(int F, DevPlan D, const double* __restrict__ Lam,
                                                  double* __restrict__ icost) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= F) return;
  const int lane = threadIdx.x & 63;
  const WinDev& W = D.win[D.win_of_f[f]];
  const int lf = f - W.f_base;
  double r[15];
  imu_residual_jacobian(W.pose, W.vel, W.bias, W.imu + lf, W.g, lf, r, nullptr);
  const int a = lane < 15 ? lane : 0;
  const double* La = Lam + (size_t)f * 225 + a * 15;
  double u = 0.0, ra = 0.0;
#pragma unroll
  for (int b = 0; b < 15; ++b) {
    u += La[b] * r[b];
    if (b == a) ra = r[b];
  }
  const double c = wave_sum(lane < 15 ? ra * u : 0.0);
  if (lane == 0) icost[f] = c;
}

__global__ void __launch_bounds__(256) k_cost_reduce(int ncost, int range_px, DevPlan D,
                                                     const double* __restrict__ vcost,
                                                     const double* __restrict__ icost, int use_imu,
                                                     double* __restrict__ trace, int slot) {
  __shared__ double s0[512];
  const int w = blockIdx.x;
  cost_reduce_block(D.win[w], w, ncost, range_px, vcost, icost, use_imu, trace, slot, s0);
}

// ---------------------------------------------------------------------------
// warm-start inputs: per keyframe (as the source of its outgoing edges) and
// 4 x 4-pixel cell of the canvas, at the current state:
//   0: sum w_x r_x / (sum w_x + 1e-6)   1: sum w_y r_y / (sum w_y + 1e-6)
//   2: sum (w_x + w_y) / (2 k n_cell)   3: mean inverse depth of the cell
//   4-12: inertial residual of the factor (i, i+1) (rotation x 100,
//         position x 10, velocity x 10), constant over the cells; zero for
//         the last keyframe or without inertial factors
//   13: -sum(w J_d r) / (h + 1e-6) / 0.2, the depth-only Gauss-Newton step
//       of the cell (J_d = dr/dd of Eq. 1, h = sum w J_d^2), in units of 0.2
//   14: log(1 + h / n_cell)
// and dims[img] = the keyframe's own cell grid.  Zero outside it.
// ---------------------------------------------------------------------------
// saved_d / saved_b (optional): a copy of every inverse depth and bias of the
// state the planes are formed at (as k_warm_state keeps it), made on the way
__global__ void __launch_bounds__(256) k_warm_features(OptsDev o, DevPlan D, int HQ, int WQ, float* __restrict__ feat,
                                                       int* __restrict__ dims, double* __restrict__ saved_d,
                                                       double* __restrict__ saved_b) {
  // 16 canvas cells per workgroup, one thread per pixel of a cell (lane
  // 16 c + j: cell c, pixel (j / 4, j % 4) of it); the cell sums are reduced
  // over the 16 lanes of the cell in a fixed order
  __shared__ double rel_s[kMaxOutDegree * 12];
  __shared__ double rimu[15];
  const int src = blockIdx.y;
  const WinDev W = D.win[D.win_of_kf[src]];
  const int ls = src - W.kf_base;
  const int e0 = D.src_off[src];
  const int k = D.src_off[src + 1] - e0;
  const int tid = threadIdx.x;
  const int hq0 = (W.H + 3) / 4, wq0 = (W.W + 3) / 4;
  const int npix = HQ * WQ;
  if (tid < k) edge_rel(W, ls, D.jj[D.src_edges[e0 + tid]] - W.kf_base, rel_s + tid * 12);
  if (blockIdx.x == 0 && tid == 0) {
    for (int q = 0; q < 15; ++q) rimu[q] = 0.0;
    if (o.use_imu && ls + 1 < W.N) imu_residual_jacobian(W.pose, W.vel, W.bias, W.imu + ls, W.g, ls, rimu, nullptr);
    dims[2 * src] = hq0;
    dims[2 * src + 1] = wq0;
  }
  if (saved_b && blockIdx.x == 0 && tid < 6) saved_b[(size_t)src * 6 + tid] = W.bias[(size_t)ls * 6 + tid];
  __syncthreads();
  float* f = feat + (size_t)src * kWCin * npix;
  const int p = blockIdx.x * 16 + (tid >> 4), j = tid & 15;
  const int cy = p / WQ, cx = p % WQ;
  const bool cell_in = p < npix && cy < hq0 && cx < wq0;
  const int y = 4 * cy + (j >> 2), x = 4 * cx + (j & 3);
  // per pixel: sum_e w r (x, y), sum_e w (x, y), sum_e w J_d r, sum_e w J_d^2, d, pixel count
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (cell_in && y < W.H && x < W.W) {
    const int pix = y * W.W + x;
    const double d = dep_load(W, (size_t)ls * W.HW + pix);
    if (saved_d) saved_d[W.pix_base + (size_t)ls * W.HW + pix] = d;
    v[6] = d;
    v[7] = 1.0;
    const double qx = ((double)x - W.cx) / W.fx, qy = ((double)y - W.cy) / W.fy;
    for (int s2 = 0; s2 < k; ++s2) {
      const int e = D.src_edges[e0 + s2];
      PixEdge q;
      pix_edge<double>(W, o, rel_s + s2 * 12, qx, qy, d, true, W.target, W.weight,
                       (size_t)(e - W.e_base) * 2 * W.HW + pix, true, q);
      v[0] += q.wx * q.rx;
      v[1] += q.wy * q.ry;
      v[2] += q.wx;
      v[3] += q.wy;
      v[4] += q.wx * q.Jdx * q.rx + q.wy * q.Jdy * q.ry;
      v[5] += q.wx * q.Jdx * q.Jdx + q.wy * q.Jdy * q.Jdy;
    }
  }
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1)
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] += __shfl_xor(v[c], m);
  if (j == 0 && p < npix) {
    double out[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (cell_in) {
      const double nc = v[7];
      out[0] = v[0] / (v[2] + 1e-6);
      out[1] = v[1] / (v[3] + 1e-6);
      out[2] = (v[2] + v[3]) / (2.0 * max(k, 1) * nc);
      out[3] = v[6] / nc;
      out[4] = -v[4] / (v[5] + 1e-6) / 0.2;
      out[5] = log1p(v[5] / nc);
    }
    const int ch[6] = {0, 1, 2, 3, 13, 14};
#pragma unroll
    for (int c = 0; c < 6; ++c) f[(size_t)ch[c] * npix + p] = (float)out[c];
  }
  if (blockIdx.x == 0) {
    for (int e = tid; e < 9 * npix; e += 256) {
      const int c = e / npix, pp = e % npix;
      const int yy = pp / WQ, xx = pp % WQ;
      const double scale = c < 3 ? 100.0 : 10.0;
      f[(size_t)(4 + c) * npix + pp] = (yy < hq0 && xx < wq0) ? (float)(rimu[c] * scale) : 0.0f;
    }
  }
}

// Apply the proposed corrections: d <- max(d + up4(dd), d_min) per pixel, where
// up4 reads the keyframe's cell grid bilinearly at ((y - 1.5) / 4, (x - 1.5) / 4)
// clamped to the grid, and b <- b + db per keyframe when the biases are
// solved (apply_bias; otherwise they keep their value).
__global__ void __launch_bounds__(256) k_warm_apply(DevPlan D, int HQ, int WQ, const float* __restrict__ dd,
                                                    const float* __restrict__ db, double d_min, int apply_bias) {
  const int src = blockIdx.y;
  const WinDev W = D.win[D.win_of_kf[src]];
  const int ls = src - W.kf_base;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (apply_bias && blockIdx.x == 0 && threadIdx.x < 6) W.bias[(size_t)ls * 6 + threadIdx.x] += (double)db[(size_t)src * 6 + threadIdx.x];
  if (p >= W.HW) return;
  const size_t pd = (size_t)ls * W.HW + p;
  dep_store(W, pd, warm_corrected_depth(W, src, p, HQ, WQ, dd, dep_load(W, pd), d_min));
}

// Keep (restore = 0) or put back (restore = 1) a keyframe's inverse depths and
// bias: saved_d is indexed like the per-pixel workspace arrays (pix_base),
// saved_b by global keyframe.  When restoring, a window is put back only if
// its cost at the corrected state (trace slot 1) is not below the cost at
// the initial state (slot 0); a non-finite corrected cost counts as not below.
__global__ void __launch_bounds__(256) k_warm_state(DevPlan D, double* __restrict__ saved_d,
                                                    double* __restrict__ saved_b, const double* __restrict__ trace,
                                                    int restore) {
  const int src = blockIdx.y;
  const int w = D.win_of_kf[src];
  const WinDev W = D.win[w];
  const int ls = src - W.kf_base;
  if (restore) {
    const double f0 = trace[(size_t)w * kTraceLen], f1 = trace[(size_t)w * kTraceLen + 2];
    if (f1 < f0) return;
  }
  const int p = blockIdx.x * 256 + threadIdx.x;
  const size_t pd = (size_t)ls * W.HW + p;
  double* sd = saved_d + W.pix_base + (size_t)ls * W.HW;
  if (p < W.HW) {
    if (restore) dep_store(W, pd, sd[p]);
    else sd[p] = dep_load(W, pd);
  }
  if (blockIdx.x == 0 && threadIdx.x < 6) {
    double* b = W.bias + (size_t)ls * 6 + threadIdx.x;
    double* sb = saved_b + (size_t)src * 6 + threadIdx.x;
    if (restore) *b = *sb;
    else *sb = *b;
  }
}

}  // namespace

// dynamic LDS of the fused assembly: relative transforms, two E-tile
// buffers, the C / w_d partials and 1/C of two chunks; the inertial
// workgroups need 1140 doubles
static size_t vis_lds(int kmax, bool f64) {
  const size_t T = vis_tiles_T(kmax);
  const size_t esz = f64 ? sizeof(double) : sizeof(float);
  const size_t ldc = f64 ? vis_ldc<double>() : vis_ldc<float>();
  const size_t vis = esz * ((size_t)kMaxOutDegree * 12 + 2 * 16 * T * ldc + 2 * kVisWaves * 64 + 2 * 64);
  const size_t imu = sizeof(double) * (450 + 450 + 225 + 15);
  return std::max(vis, imu);
}

typedef void (*VisKernel)(OptsDev, DevPlan, int, int, int, int, int, const double*, double*, double*, double*,
                          double*, double*, double*, double*, double*, double*, double*, DevStatus*);

// the instantiation of the fused assembly for the largest out-degree of a batch:
// edge slots per wave ceil(kmax / 8), Gram tiles per wave ceil(T (T + 1) / 16)
template <typename R>
static VisKernel vis_kernel(int kmax) {
  const int T = vis_tiles_T(kmax);
  const int ts = (T * (T + 1) / 2 + kVisWaves - 1) / kVisWaves;
  const int slots = (kmax + kVisWaves - 1) / kVisWaves;
  if (slots <= 1) return ts <= 1 ? k_vis_gram<R, 1, 1> : k_vis_gram<R, 1, 2>;
  if (slots == 2) return ts <= 2 ? k_vis_gram<R, 2, 2> : (ts == 3 ? k_vis_gram<R, 2, 3> : k_vis_gram<R, 2, 4>);
  return k_vis_gram<R, 3, 4>;
}
static size_t local_lds(int kmax) {
  const size_t k = kmax, nq = 6 * k + 1;
  return sizeof(double) * std::max<size_t>(nq * nq + 4 * 36 * k + 9 * k + 6 * k, 2 * kLocalThreads);
}

void launch_reset_status(hipStream_t s, DevStatus* st, int n) {
  hipLaunchKernelGGL(k_reset_status, dim3((n + 63) / 64), dim3(64), 0, s, st, n);
}

void chol_set_attributes();

void step_set_attributes(int kmax) {
  chol_set_attributes();
  // every instantiation of the fused assembly may run for some batch: each
  // gets the LDS cap of the largest out-degree it serves
  for (int km = 1; km <= kMaxOutDegree; ++km) {
    (void)hipFuncSetAttribute((const void*)vis_kernel<double>(km), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)vis_lds(kMaxOutDegree, true));
    (void)hipFuncSetAttribute((const void*)vis_kernel<float>(km), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)vis_lds(kMaxOutDegree, false));
  }
  (void)hipFuncSetAttribute((const void*)k_local, hipFuncAttributeMaxDynamicSharedMemorySize, (int)local_lds(kmax));
}

// the fused assembly (with the inertial factors) and the local blocks
static void launch_front(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o, int iter,
                         StageMark mark, void* mark_user, DevStatus* st) {
  const int N = P.N;
  auto done = [&](int stage) { if (mark) mark(mark_user, stage); };
  const int F = (o.use_imu && P.F > 0) ? P.F : 0;
  const int nkr_run = (P.hw_max + P.range - 1) / P.range;          // workgroups per source in x
  const int imu_rows = (F + nkr_run - 1) / nkr_run;
  const int ncost = cost_slots(P);
  const bool f64 = o.precision != VI_PREC_MIXED;
  VisKernel kern = f64 ? vis_kernel<double>(P.kmax) : vis_kernel<float>(P.kmax);
  hipLaunchKernelGGL(kern, dim3(nkr_run, N + imu_rows), dim3(kVisThreads), vis_lds(P.kmax, f64), s, o, D, imu_rows, F,
                     P.nkr_max, ncost, P.range, w.Lam, w.Rw, w.rel, w.Cd, w.wd, w.hpart, w.gpart, w.vcost, w.Hf,
                     w.gf, w.icost, st);
  done(kStVis);
  hipLaunchKernelGGL(k_local, dim3(N + P.n_win), dim3(kLocalThreads), local_lds(P.kmax), s, N, P.nkr_max, ncost,
                     P.range, D, w.Rw, w.rel, w.hpart, w.gpart, w.Z, w.ZB, w.ZV, w.vcost, w.icost, o.use_imu, w.trace,
                     iter, o.tol, st);
  done(kStLocal);
}

void launch_vis_assembly(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                         DevStatus* st) {
  const int nkr_run = (P.hw_max + P.range - 1) / P.range;
  const bool f64 = o.precision != VI_PREC_MIXED;
  VisKernel kern = f64 ? vis_kernel<double>(P.kmax) : vis_kernel<float>(P.kmax);
  hipLaunchKernelGGL(kern, dim3(nkr_run, P.N), dim3(kVisThreads), vis_lds(P.kmax, f64), s, o, D, 0, 0, P.nkr_max,
                     cost_slots(P), P.range, w.Lam, w.Rw, w.rel, w.Cd, w.wd, w.hpart, w.gpart, w.vcost, w.Hf, w.gf,
                     w.icost, st);
}

void launch_vis_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o) {
  auto kvc = (o.precision == VI_PREC_MIXED) ? k_vis_cost<float> : k_vis_cost<double>;
  hipLaunchKernelGGL(kvc, dim3((P.hw_max + kVisBlock - 1) / kVisBlock, P.N), dim3(256), 0, s, o, D, cost_slots(P),
                     w.vcost, nullptr, nullptr, 0, 0, 0.0);
}

void launch_tune_stages(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o,
                        StageMark mark, void* mark_user) {
  launch_front(s, P, D, w, o, 0, mark, mark_user, nullptr);
}

void launch_step(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o, int iter,
                 DevStatus* st, StageMark mark, void* mark_user) {
  const int N = P.N;
  auto done = [&](int stage) { if (mark) mark(mark_user, stage); };
  launch_front(s, P, D, w, o, iter, mark, mark_user, st);
  size_t total_max = 0;
  for (const WinDev& W : P.win) total_max = std::max(total_max, (size_t)(W.npad + kCholNB) * W.npad);
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((total_max + 255) / 256), P.n_win), dim3(256), 0, s, o, D, w.Z,
                     w.ZB, w.ZV, w.Hf, w.gf, w.A, w.flags, w.sync, st);
  done(kStAssemble);
  launch_chol(s, P, D, w, st);
  done(kStChol);
  auto kbs = (o.precision == VI_PREC_MIXED) ? k_backsub_retract<float> : k_backsub_retract<double>;
  // pixels per thread: 1 for small batches, up to 4 once the batch holds more
  // than about 2048 workgroups' worth (the per-workgroup setup, a few
  // dependent loads, is then shared by more pixels)
  const int ppt = (int)std::min<long long>(4, std::max<long long>(1, P.pix_total / (256LL * 2048)));
  const int pxb = 256 * ppt;
  hipLaunchKernelGGL(kbs, dim3((P.hw_max + pxb - 1) / pxb, N + P.n_win), dim3(256), 0, s, o, N, D, w.Rw,
                     w.rel, w.Cd, w.wd, w.x, ppt, st);
  done(kStBacksub);
}

void launch_final_cost(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& o, int slot,
                       double* trace, const float* dd, const float* db, int HQ, int WQ, double d_min) {
  const int N = P.N;
  const int ncost = cost_slots(P);
  auto kvc = (o.precision == VI_PREC_MIXED) ? k_vis_cost<float> : k_vis_cost<double>;
  hipLaunchKernelGGL(kvc, dim3((P.hw_max + kVisBlock - 1) / kVisBlock, N), dim3(256), 0, s, o, D, ncost,
                     w.vcost, dd, db, HQ, WQ, d_min);
  if (o.use_imu && P.F > 0)
    hipLaunchKernelGGL(k_imu_cost, dim3((P.F + 3) / 4), dim3(256), 0, s, P.F, D, w.Lam, w.icost);
  hipLaunchKernelGGL(k_cost_reduce, dim3(P.n_win), dim3(256), 0, s, ncost, kVisBlock, D, w.vcost, w.icost,
                     o.use_imu, trace ? trace : w.trace, slot);
}

void launch_warm_features(hipStream_t s, const Plan& P, const DevPlan& D, const OptsDev& o, int HQ, int WQ,
                          float* feat, int* dims, double* saved_d, double* saved_b) {
  hipLaunchKernelGGL(k_warm_features, dim3((HQ * WQ + 15) / 16, P.N), dim3(256), 0, s, o, D, HQ, WQ, feat, dims,
                     saved_d, saved_b);
}

void launch_warm_apply(hipStream_t s, const Plan& P, const DevPlan& D, int HQ, int WQ, const float* dd,
                       const float* db, double d_min, int apply_bias) {
  hipLaunchKernelGGL(k_warm_apply, dim3((P.hw_max + 255) / 256, P.N), dim3(256), 0, s, D, HQ, WQ, dd, db, d_min,
                     apply_bias);
}

void launch_warm_state(hipStream_t s, const Plan& P, const DevPlan& D, double* saved_d, double* saved_b,
                       const double* trace, int restore) {
  hipLaunchKernelGGL(k_warm_state, dim3((P.hw_max + 255) / 256, P.N), dim3(256), 0, s, D, saved_d, saved_b, trace,
                     restore);
}

}  // namespace vi
