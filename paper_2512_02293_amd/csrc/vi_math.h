// Device-side FP64 helpers for the visual-inertial step: 3x3 algebra, the
// rotation exponential/logarithm and right Jacobians, and quaternions.
// Matrices are row-major double[9].  All functions are written for single
// lanes; no cross-lane communication happens here.
#pragma once
#include <hip/hip_runtime.h>

namespace vi {

__device__ __forceinline__ void m3_mul(const double* A, const double* B, double* C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[r * 3 + c] = A[r * 3 + 0] * B[0 * 3 + c] + A[r * 3 + 1] * B[1 * 3 + c] + A[r * 3 + 2] * B[2 * 3 + c];
}

// C = A^T B
__device__ __forceinline__ void m3_tmul(const double* A, const double* B, double* C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[r * 3 + c] = A[0 * 3 + r] * B[0 * 3 + c] + A[1 * 3 + r] * B[1 * 3 + c] + A[2 * 3 + r] * B[2 * 3 + c];
}

// y = A x
__device__ __forceinline__ void m3_vec(const double* A, const double* x, double* y) {
#pragma unroll
  for (int r = 0; r < 3; ++r) y[r] = A[r * 3 + 0] * x[0] + A[r * 3 + 1] * x[1] + A[r * 3 + 2] * x[2];
}

// y = A^T x
__device__ __forceinline__ void m3_tvec(const double* A, const double* x, double* y) {
#pragma unroll
  for (int r = 0; r < 3; ++r) y[r] = A[0 * 3 + r] * x[0] + A[1 * 3 + r] * x[1] + A[2 * 3 + r] * x[2];
}

__device__ __forceinline__ void skew(const double* w, double* S) {
  S[0] = 0.0;   S[1] = -w[2]; S[2] = w[1];
  S[3] = w[2];  S[4] = 0.0;   S[5] = -w[0];
  S[6] = -w[1]; S[7] = w[0];  S[8] = 0.0;
}

// Exp(w) by Rodrigues: I + a K + b K^2 with K = [w]x, a = sin t / t, b = (1 - cos t) / t^2.
__device__ inline void so3_exp(const double* w, double* R) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double a, b;
  if (t2 < 1e-16) {
    a = 1.0 - t2 / 6.0;
    b = 0.5 - t2 / 24.0;
  } else {
    const double t = sqrt(t2);
    a = sin(t) / t;
    b = (1.0 - cos(t)) / t2;
  }
  // K^2 = w w^T - t2 I
  const double x = w[0], y = w[1], z = w[2];
  R[0] = 1.0 + b * (x * x - t2); R[1] = -a * z + b * x * y;     R[2] = a * y + b * x * z;
  R[3] = a * z + b * x * y;      R[4] = 1.0 + b * (y * y - t2); R[5] = -a * x + b * y * z;
  R[6] = -a * y + b * x * z;     R[7] = a * x + b * y * z;      R[8] = 1.0 + b * (z * z - t2);
}

// Log(R): angle from atan2(|vee(R - R^T)|/2, (tr R - 1)/2); near pi the axis
// comes from the symmetric part.
__device__ inline void so3_log(const double* R, double* w) {
  const double vx = R[7] - R[5], vy = R[2] - R[6], vz = R[3] - R[1];
  const double s = 0.5 * sqrt(vx * vx + vy * vy + vz * vz);
  const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  const double t = atan2(s, c);
  if (t < 1e-6) {
    const double f = 0.5 * (1.0 + t * t / 6.0);
    w[0] = f * vx; w[1] = f * vy; w[2] = f * vz;
    return;
  }
  if (M_PI - t > 1e-6) {
    const double f = 0.5 * t / sin(t);
    w[0] = f * vx; w[1] = f * vy; w[2] = f * vz;
    return;
  }
  // u u^T = (R + R^T - 2 c I) / (2 (1 - c))
  const double den = 2.0 * (1.0 - c);
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) M[r * 3 + q] = (R[r * 3 + q] + R[q * 3 + r] - (r == q ? 2.0 * c : 0.0)) / den;
  // column k of the largest diagonal entry, chosen by selects (an index into
  // M would put M in scratch memory)
  int k = 0;
  double mk = M[0];
  if (M[4] > mk) { k = 1; mk = M[4]; }
  if (M[8] > mk) { k = 2; mk = M[8]; }
  const double nk = sqrt(fmax(mk, 1e-300));
  double u[3] = {(k == 0 ? M[0] : k == 1 ? M[1] : M[2]) / nk, (k == 0 ? M[3] : k == 1 ? M[4] : M[5]) / nk,
                 (k == 0 ? M[6] : k == 1 ? M[7] : M[8]) / nk};
  if (u[0] * vx + u[1] * vy + u[2] * vz < 0.0) { u[0] = -u[0]; u[1] = -u[1]; u[2] = -u[2]; }
  w[0] = t * u[0]; w[1] = t * u[1]; w[2] = t * u[2];
}

// Right Jacobian: I - a K + b K^2, a = (1 - cos t)/t^2, b = (t - sin t)/t^3.
__device__ inline void so3_jr(const double* w, double* J) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double a, b;
  if (t2 < 1e-12) {
    a = 0.5 - t2 / 24.0;
    b = 1.0 / 6.0 - t2 / 120.0;
  } else {
    const double t = sqrt(t2);
    a = (1.0 - cos(t)) / t2;
    b = (t - sin(t)) / (t2 * t);
  }
  const double x = w[0], y = w[1], z = w[2];
  J[0] = 1.0 + b * (x * x - t2); J[1] = a * z + b * x * y;       J[2] = -a * y + b * x * z;
  J[3] = -a * z + b * x * y;     J[4] = 1.0 + b * (y * y - t2); J[5] = a * x + b * y * z;
  J[6] = a * y + b * x * z;      J[7] = -a * x + b * y * z;     J[8] = 1.0 + b * (z * z - t2);
}

// Inverse right Jacobian: I + K/2 + c K^2, c = 1/t^2 - (1 + cos t) / (2 t sin t).
__device__ inline void so3_jr_inv(const double* w, double* J) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double c;
  if (t2 < 1e-12) {
    c = 1.0 / 12.0 + t2 / 720.0;
  } else {
    const double t = sqrt(t2);
    c = 1.0 / t2 - (1.0 + cos(t)) / (2.0 * t * sin(t));
  }
  const double x = w[0], y = w[1], z = w[2];
  J[0] = 1.0 + c * (x * x - t2); J[1] = -0.5 * z + c * x * y;    J[2] = 0.5 * y + c * x * z;
  J[3] = 0.5 * z + c * x * y;    J[4] = 1.0 + c * (y * y - t2); J[5] = -0.5 * x + c * y * z;
  J[6] = -0.5 * y + c * x * z;   J[7] = 0.5 * x + c * y * z;    J[8] = 1.0 + c * (z * z - t2);
}

// Rotation matrix of the quaternion (x, y, z, w), normalised on the fly.
__device__ inline void quat_to_rot(const double* q, double* R) {
  const double n = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const double s = 2.0 / n;
  const double x = q[0], y = q[1], z = q[2], w = q[3];
  R[0] = 1.0 - s * (y * y + z * z); R[1] = s * (x * y - z * w);       R[2] = s * (x * z + y * w);
  R[3] = s * (x * y + z * w);       R[4] = 1.0 - s * (x * x + z * z); R[5] = s * (y * z - x * w);
  R[6] = s * (x * z - y * w);       R[7] = s * (y * z + x * w);       R[8] = 1.0 - s * (x * x + y * y);
}

// Unit quaternion (x, y, z, w) of a rotation matrix, from the largest of
// 1 + tr R, 1 + 2 R_00 - tr R, 1 + 2 R_11 - tr R, 1 + 2 R_22 - tr R (the
// numerically safe pivot), normalised at the end.
__device__ inline void rot_to_quat(const double* R, double* q) {
  const double tr = R[0] + R[4] + R[8];
  const double c[4] = {1.0 + tr, 1.0 + 2.0 * R[0] - tr, 1.0 + 2.0 * R[4] - tr, 1.0 + 2.0 * R[8] - tr};
  int k = 0;
  double ck = c[0];                     // c[k], kept by value (an index into c would put c in scratch memory)
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (c[i] > ck) { k = i; ck = c[i]; }
  const double s = 0.5 / sqrt(ck);     // 4 * (the pivot component) = 2 sqrt(c[k])
  double x, y, z, w;
  if (k == 0) {
    w = 0.5 * sqrt(c[0]); x = (R[7] - R[5]) * s; y = (R[2] - R[6]) * s; z = (R[3] - R[1]) * s;
  } else if (k == 1) {
    x = 0.5 * sqrt(c[1]); w = (R[7] - R[5]) * s; y = (R[1] + R[3]) * s; z = (R[2] + R[6]) * s;
  } else if (k == 2) {
    y = 0.5 * sqrt(c[2]); w = (R[2] - R[6]) * s; x = (R[1] + R[3]) * s; z = (R[5] + R[7]) * s;
  } else {
    z = 0.5 * sqrt(c[3]); w = (R[3] - R[1]) * s; x = (R[2] + R[6]) * s; y = (R[5] + R[7]) * s;
  }
  const double n = 1.0 / sqrt(x * x + y * y + z * z + w * w);
  q[0] = x * n; q[1] = y * n; q[2] = z * n; q[3] = w * n;
}

// q <- normalise(q (x) exp_q(w)): the quaternion form of R <- R Exp(w).
__device__ inline void quat_retract(double* q, const double* w) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double sh, ch;
  if (t2 < 1e-16) {
    sh = 0.5 - t2 / 48.0;      // sin(t/2)/t
    ch = 1.0 - t2 / 8.0;       // cos(t/2)
  } else {
    const double t = sqrt(t2);
    sh = sin(0.5 * t) / t;
    ch = cos(0.5 * t);
  }
  const double bx = w[0] * sh, by = w[1] * sh, bz = w[2] * sh, bw = ch;
  const double ax = q[0], ay = q[1], az = q[2], aw = q[3];
  double nx = aw * bx + ax * bw + ay * bz - az * by;
  double ny = aw * by - ax * bz + ay * bw + az * bx;
  double nz = aw * bz + ax * by - ay * bx + az * bw;
  double nw = aw * bw - ax * bx - ay * by - az * bz;
  const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz + nw * nw);
  q[0] = nx * inv; q[1] = ny * inv; q[2] = nz * inv; q[3] = nw * inv;
}

}  // namespace vi
