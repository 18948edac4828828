// FP64 Cholesky solve of the reduced pose/velocity/bias system of Eq. 4.
//
// The matrix buffer of a window holds S (npad x npad, row-major, lower
// triangle used) followed by a 32-row right-hand-side block whose first row is
// s, so the factorisation carries the forward substitution along: at the end
// that row holds y = L^-1 s.
//
// Factorisation: a tile-level dataflow over 32 x 32 tiles (i, j), j <= i,
// i = nblk being the right-hand-side block, of every window of the batch in
// one launch.  Each tile is one wave:
//   X = S_ij - sum_{k < j} L_ik L_jk^T        (FP64 MFMA 16x16x4, operands
//                                              straight from global memory)
//   i == j : factor X = L_jj L_jj^T in registers (lane = row) and invert it;
//   i != j : L_ij = X L_jj^-T                 (FP64 MFMA)
// and publishes the result with a release flag.  Tiles are handed out by an
// atomic ticket counter in column-major order (column j, then window, then
// row i), and a tile only ever waits for tiles of smaller tickets, which were
// taken by running workgroups: every wait ends without any assumption on
// how many workgroups are resident.  Every wait is also bounded: past the
// limit the batch is aborted (VI_EDEVICE) and every workgroup exits.
//
// Back-substitution x = L^-T y runs per window in one 1024-thread workgroup,
// block column by block column: x_b = L_bb^-T t_b, then t_c -= L_bc^T x_b
// for every c < b in parallel over the waves.
//
// Windows with npad <= kSmallMaxNpad (sliding windows) are factored and
// solved entirely inside one 512-thread workgroup instead (no inter-
// workgroup traffic; the critical path is the chain of diagonal-tile
// factorisations).  That path skips the tiles outside the window's band: a
// banded matrix (every nonzero within w of the diagonal) has a banded Cholesky
// factor, so tiles with 32 (i - j) - 31 > w stay zero.  The diagonal tile is
// factored recursively (two 16 x 16 leaves, the coupling block by MFMA), which
// halves the serial broadcast chain of a flat 32-pivot factorisation.
#include <algorithm>

#include "vi_internal.h"

namespace vi {

namespace {

constexpr int NB = kCholNB;          // 32
constexpr int LD = NB + 1;
constexpr int kSpinLimit = 1 << 22;  // polls (each with a short sleep) before the batch is aborted
constexpr int kMaxDataflowWG = 4096;
constexpr int kSmallMaxNpad = kCholSmallMaxNpad;

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void set_status(DevStatus* st, int code, int detail) {
  if (atomicCAS(&st->code, 0, code) == 0) st->detail = detail;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_readlane(lo, l);
  hi = __builtin_amdgcn_readlane(hi, l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int load_flag(const int* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (whole wave) until *f is set.  false: the batch was aborted.
__device__ __forceinline__ bool wait_flag(const int* f, int* sync) {
  int spins = 0;
  while (__builtin_amdgcn_readfirstlane(load_flag(f)) == 0) {
    if (__builtin_amdgcn_readfirstlane(load_flag(sync + 1)) != 0) return false;
    if (++spins > kSpinLimit) {
      if (threadIdx.x == 0) __hip_atomic_store(sync + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__device__ __forceinline__ void publish(int* f) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// acc (2x2 blocks of 16x16 in MFMA output layout: lane l, element r holds row
// (l >> 4) + 4 r, column l & 15 of its block) <-> a row-major 32x32 array
__device__ __forceinline__ void acc_to_lds(const double4_t (&acc)[2][2], double* T) {
  const int l = threadIdx.x;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) T[(16 * bm + (l >> 4) + 4 * r) * LD + 16 * bn + (l & 15)] = acc[bm][bn][r];
}

__device__ __forceinline__ double rsqrt_refined(double v) {
  // hardware reciprocal square root, then two Newton steps to full precision
  double y = __builtin_amdgcn_rsq(v);
  const double h = 0.5 * v;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}

__global__ void __launch_bounds__(64) k_chol_df(DevPlan D, int ntickets, double* __restrict__ Aall,
                                                double* __restrict__ Linvall, int* __restrict__ flagsall,
                                                int* __restrict__ sync, DevStatus* __restrict__ stall) {
  __shared__ double T[NB * LD];
  __shared__ double rinv[NB];
  const int lane = threadIdx.x;
  const int mrow = lane & 15, kq = lane >> 4;
  while (true) {
    int t = 0;
    if (lane == 0) t = atomicAdd(sync, 1);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= ntickets) return;
    const int w = D.chol_tiles[2 * t];
    const int ij = D.chol_tiles[2 * t + 1];
    const int i = ij >> 16, j = ij & 0xffff;
    const WinDev& W = D.win[w];
    const int npad = W.npad, nblk = W.nblk;
    double* A = Aall + W.A_off;
    double* Lv = Linvall + W.Linv_off;
    int* fl = flagsall + W.flag_off;
    // X = S_ij in MFMA layout
    double4_t acc[2][2];
    const double* Sij = A + (size_t)(NB * i) * npad + NB * j;
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[bm][bn][r] = Sij[(size_t)(16 * bm + kq + 4 * r) * npad + 16 * bn + mrow];
    // X -= L_ik L_jk^T: lane supplies A[m][q] = L_ik[m][q], B[q][n] = L_jk[n][q]
    for (int k = 0; k < j; ++k) {
      if (!wait_flag(fl + i * nblk + k, sync)) return;
      if (i != j && !wait_flag(fl + j * nblk + k, sync)) return;
      const double* Li = A + (size_t)(NB * i) * npad + NB * k;
      const double* Lj = A + (size_t)(NB * j) * npad + NB * k;
      double a[2][8], b[2][8];
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          a[h][s] = -Li[(size_t)(16 * h + mrow) * npad + 4 * s + kq];
          b[h][s] = Lj[(size_t)(16 * h + mrow) * npad + 4 * s + kq];
        }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
          for (int bn = 0; bn < 2; ++bn)
            acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm][s], b[bn][s], acc[bm][bn], 0, 0, 0);
    }
    acc_to_lds(acc, T);
    __syncthreads();
    if (i == j) {
      // factor: lane i (< 32) holds row i; lanes >= 32 mirror rows 0..31 and are ignored
      const int row = lane & 31;
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = T[row * LD + c];
      int bad = -1;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double piv = readlane_d(x[c], c);
        if (!(piv > 0.0)) {
          if (bad < 0) bad = c;
          piv = 1.0;
        }
        const double r = rsqrt_refined(piv);
        if (lane == c) rinv[c] = r;
        x[c] = (row == c) ? piv * r : (row > c ? x[c] * r : x[c]);
#pragma unroll
        for (int m = 1; m < NB; ++m) {
          if (m > c) {
            const double lm = readlane_d(x[c], m);
            if (row >= m) x[m] -= x[c] * lm;
          }
        }
      }
      if (bad >= 0 && lane == 0 && NB * j + bad < W.n) set_status(stall + w, VI_ENOTPD, NB * j + bad);
#pragma unroll
      for (int c = 0; c < NB; ++c) T[row * LD + c] = (c <= row) ? x[c] : 0.0;
      __syncthreads();
      // inverse: lane c (< 32) computes column c of L^-1
      double y[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        double v = (r == row) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < NB - 1; ++q)
          if (q < r) v -= T[r * LD + q] * y[q];
        y[r] = v * rinv[r];
      }
      if (lane < NB) {
        double* Lo = Lv + (size_t)j * NB * NB;
#pragma unroll
        for (int r = 0; r < NB; ++r) Lo[r * NB + lane] = y[r];
      }
      publish(fl + j * nblk + j);
    } else {
      if (!wait_flag(fl + j * nblk + j, sync)) return;
      // L_ij = X L_jj^-T: A[m][q] = X[m][q], B[q][n] = Linv[n][q]
      const double* Li = Lv + (size_t)j * NB * NB;
      double4_t out[2][2];
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) out[bm][bn] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        double a[2], b[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          a[h] = T[(16 * h + mrow) * LD + 4 * s + kq];
          b[h] = Li[(16 * h + mrow) * NB + 4 * s + kq];
        }
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
          for (int bn = 0; bn < 2; ++bn)
            out[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm], b[bn], out[bm][bn], 0, 0, 0);
      }
      double* Oij = A + (size_t)(NB * i) * npad + NB * j;
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
          for (int r = 0; r < 4; ++r) Oij[(size_t)(16 * bm + kq + 4 * r) * npad + 16 * bn + mrow] = out[bm][bn][r];
      publish(fl + i * nblk + j);
    }
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// one-wave helpers on 16 x 16 blocks in LDS (row-major with stride ld)
// ---------------------------------------------------------------------------
// In-place Cholesky of the SPD block M (lower triangle of the result is L,
// upper set to zero); rinv[c] = 1 / L[c][c].  Returns the first bad pivot
// index or -1.  Lane r (< 16) holds row r; other lanes mirror it.
__device__ __forceinline__ int leaf16_factor(double* M, int ld, double* rinv) {
  const int lane = threadIdx.x & 63, row = lane & 15;
  double x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = M[row * ld + c];
  int bad = -1;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double piv = readlane_d(x[c], c);
    if (!(piv > 0.0)) {
      if (bad < 0) bad = c;
      piv = 1.0;
    }
    const double r = rsqrt_refined(piv);
    if (lane == c) rinv[c] = r;
    x[c] = (row == c) ? piv * r : (row > c ? x[c] * r : x[c]);
#pragma unroll
    for (int m = 1; m < 16; ++m) {
      if (m > c) {   // constant trip count: fully unrolled, x stays in registers
        const double lm = readlane_d(x[c], m);
        if (row >= m) x[m] -= x[c] * lm;
      }
    }
  }
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) M[row * ld + c] = (c <= row) ? x[c] : 0.0;
  }
  return bad;
}

// Minv = L^-1 for the lower-triangular 16 x 16 L in M (rinv = 1 / diag);
// lane c (< 16) computes column c.
__device__ __forceinline__ void leaf16_inverse(const double* M, int ld, const double* rinv, double* Minv, int ldi) {
  const int lane = threadIdx.x & 63, col = lane & 15;
  double y[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double v = (r == col) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < 15; ++q)
      if (q < r) v -= M[r * ld + q] * y[q];
    y[r] = v * rinv[r];
  }
  if (lane < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Minv[r * ldi + col] = y[r];
  }
}

// acc += sA * (A B) for 16 x 16 blocks: A(m, q) = Aop[m * lda + q] (or its
// transpose when ta), B(q, n) = Bop[q * ldb + n] (or Bop[n * ldb + q] when tb).
__device__ __forceinline__ double4_t mm16(double4_t acc, const double* Aop, int lda, bool ta, const double* Bop,
                                          int ldb, bool tb, double sA) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int q = 4 * s + kq;
    const double a = ta ? Aop[q * lda + mrow] : Aop[mrow * lda + q];
    const double b = tb ? Bop[mrow * ldb + q] : Bop[q * ldb + mrow];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA * a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ double4_t load16(const double* M, int ld) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
  double4_t v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = M[(kq + 4 * r) * ld + mrow];
  return v;
}

__device__ __forceinline__ void store16(double* M, int ld, double4_t v) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) M[(kq + 4 * r) * ld + mrow] = v[r];
}

// Cholesky factor L and inverse X = L^-1 of an 8x8 SPD block, computed by
// every lane redundantly in registers (no cross-lane traffic at all); packed
// lower-triangular storage, entry (i, j) at i (i + 1) / 2 + j.  Returns the
// first bad pivot or -1.
__device__ __forceinline__ constexpr int tri8(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ __forceinline__ int leaf8(const double* M, int ld, double (&L)[36], double (&X)[36]) {
  double a[36];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j <= i) a[tri8(i, j)] = M[i * ld + j];
  int bad = -1;
  double rv[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double piv = a[tri8(j, j)];
    if (!(piv > 0.0)) {
      if (bad < 0) bad = j;
      piv = 1.0;
    }
    const double r = rsqrt_refined(piv);
    rv[j] = r;
    L[tri8(j, j)] = piv * r;
#pragma unroll
    for (int i = 1; i < 8; ++i)
      if (i > j) L[tri8(i, j)] = a[tri8(i, j)] * r;
#pragma unroll
    for (int i = 1; i < 8; ++i)
#pragma unroll
      for (int m = 1; m < 8; ++m)
        if (i > j && m > j && m <= i) a[tri8(i, m)] -= L[tri8(i, j)] * L[tri8(m, j)];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    X[tri8(c, c)] = rv[c];
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      if (r > c) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q)
          if (q >= c && q < r) v += L[tri8(r, q)] * X[tri8(q, c)];
        X[tri8(r, c)] = -v * rv[r];
      }
    }
  }
  return bad;
}

// packed lower 8x8 (all lanes hold it) -> rows/columns of a padded LDS block,
// zeros above the diagonal; written by lane 0
__device__ __forceinline__ void put8(const double (&P)[36], double* D, int ld) {
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) D[i * ld + j] = (j <= i) ? P[tri8(i, j)] : 0.0;
  }
}

// One wave: inverse Cholesky factor of the 16x16 SPD block M (stride ld) into
// Mi (stride ldi), by two register-resident 8x8 leaves:
//   X11 = chol(A11)^-1, L21 = A21 X11^T, X22 = chol(A22 - L21 L21^T)^-1,
//   X21 = -X22 L21 X11.
// M's lower blocks are overwritten (L21, the updated A22).  S: 8 x 9 scratch.
// Returns the first bad pivot (0..15) or -1.
__device__ __forceinline__ int leaf16_factor_inverse(double* M, int ld, double* Mi, int ldi, double* S) {
  const int lane = threadIdx.x & 63, i = lane >> 3, j = lane & 7;
  double L[36], X[36];
  int bad = leaf8(M, ld, L, X);
  put8(X, Mi, ldi);                                           // X11
  // L21 = A21 X11^T (one entry per lane)
  {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) v += M[(8 + i) * ld + q] * Mi[j * ldi + q];
    M[(8 + i) * ld + j] = v;
  }
  // A22 -= L21 L21^T
  {
    double v = M[(8 + i) * ld + 8 + j];
#pragma unroll
    for (int q = 0; q < 8; ++q) v -= M[(8 + i) * ld + q] * M[(8 + j) * ld + q];
    M[(8 + i) * ld + 8 + j] = v;
  }
  const int bad2 = leaf8(M + 8 * ld + 8, ld, L, X);
  if (bad < 0 && bad2 >= 0) bad = 8 + bad2;
  put8(X, Mi + 8 * ldi + 8, ldi);                             // X22
  // P = L21 X11 -> S, X21 = -X22 P, X12 = 0
  {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) v += M[(8 + i) * ld + q] * Mi[q * ldi + j];
    S[i * 9 + j] = v;
  }
  {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) v += Mi[(8 + i) * ldi + 8 + q] * S[q * 9 + j];
    Mi[(8 + i) * ldi + j] = -v;
    Mi[i * ldi + 8 + j] = 0.0;
  }
  return bad;
}

// One wave: the 32 x 32 SPD tile T (LDS, stride LD) -> Li = L^-1 (LDS, stride
// LD), via X11 = chol(A11)^-1, L21 = A21 X11^T, X22 = chol(A22 - L21 L21^T)^-1,
// L^-1 = [[X11, 0], [-X22 L21 X11, X22]].  T is overwritten.
// Returns the first bad pivot (0..31) or -1.  U: 16 x 17 LDS scratch.
__device__ __forceinline__ int factor_invert32(double* T, double* Li, double* U, double* rinv) {
  (void)rinv;
  int bad = leaf16_factor_inverse(T, LD, Li, LD, U);                    // I11
  double4_t z = double4_t{0.0, 0.0, 0.0, 0.0};
  // L21 = A21 I11^T
  double4_t l21 = mm16(z, T + 16 * LD, LD, false, Li, LD, true, 1.0);
  store16(T + 16 * LD, LD, l21);
  // A22 -= L21 L21^T
  double4_t a22 = load16(T + 16 * LD + 16, LD);
  a22 = mm16(a22, T + 16 * LD, LD, false, T + 16 * LD, LD, true, -1.0);
  store16(T + 16 * LD + 16, LD, a22);
  const int bad2 = leaf16_factor_inverse(T + 16 * LD + 16, LD, Li + 16 * LD + 16, LD, U);   // I22
  if (bad < 0 && bad2 >= 0) bad = 16 + bad2;
  // P = L21 I11 (into U), X = -I22 P
  double4_t p = mm16(z, T + 16 * LD, LD, false, Li, LD, false, 1.0);
  store16(U, 17, p);
  double4_t xx = mm16(z, Li + 16 * LD + 16, LD, false, U, 17, false, -1.0);
  store16(Li + 16 * LD, LD, xx);
  const int lane = threadIdx.x & 63;
  // upper-right block of L^-1 is zero
  for (int e = lane; e < 256; e += 64) Li[(e >> 4) * LD + 16 + (e & 15)] = 0.0;
  return bad;
}

// acc(2x2 blocks of 16x16) += sA * X Y^T over K = 32, X, Y 32 x 32 row-major
// with strides ldx, ldy (global or LDS)
__device__ __forceinline__ void mm32_abt(double4_t (&acc)[2][2], const double* X, size_t ldx, const double* Y,
                                         size_t ldy, double sA) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
  double a[2][8], b[2][8];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a[h][s] = sA * X[(16 * h + mrow) * ldx + 4 * s + kq];
      b[h][s] = Y[(16 * h + mrow) * ldy + 4 * s + kq];
    }
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm][s], b[bn][s], acc[bm][bn], 0, 0, 0);
}

__device__ __forceinline__ void load_tile32(double4_t (&acc)[2][2], const double* M, size_t ld) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bm][bn][r] = M[(16 * bm + kq + 4 * r) * ld + 16 * bn + mrow];
}

__device__ __forceinline__ void store_tile32(const double4_t (&acc)[2][2], double* M, size_t ld) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) M[(16 * bm + kq + 4 * r) * ld + 16 * bn + mrow] = acc[bm][bn][r];
}

// 32 x 32 tile in LDS without padding, column index XOR-swizzled by row so
// that the MFMA operand reads (16 rows x 4 columns per instruction) and the
// row-wise reads of the back-substitution hit distinct banks.
__device__ __forceinline__ int swz(int r, int c) { return r * NB + (c ^ ((r * 4) & 31)); }

// acc(2x2 blocks of 16x16) += sA * X Y^T over K = 32, X and Y swizzled LDS tiles
__device__ __forceinline__ void mm32_abt_lds(double4_t (&acc)[2][2], const double* X, const double* Y, double sA) {
  const int lane = threadIdx.x & 63, mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    double a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a[h] = sA * X[swz(16 * h + mrow, 4 * s + kq)];
      b[h] = Y[swz(16 * h + mrow, 4 * s + kq)];
    }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm], b[bn], acc[bm][bn], 0, 0, 0);
  }
}

// global 32 x 32 tile -> padded LDS tile, all loads in flight at once (one wave)
__device__ __forceinline__ void tile_to_lds(double* T, const double* M, size_t ld) {
  const int lane = threadIdx.x & 63;
  double v[16];
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int e = lane + 64 * it;
    v[it] = M[(size_t)(e >> 5) * ld + (e & 31)];
  }
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int e = lane + 64 * it;
    T[(e >> 5) * LD + (e & 31)] = v[it];
  }
}

// y_b <- L_bb^-1 y_b in place (32 entries of yv; Li padded, lower triangular); one wave
__device__ __forceinline__ void fwd_block(const double* Li, double* yb) {
  const int lane = threadIdx.x & 63, c = lane & 31;
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) v += Li[c * LD + q] * yb[q];
  if (lane < NB) yb[c] = v;
}

// Whole factorisation and solve of one small window per 512-thread workgroup.
// Right-looking over 32-wide block columns inside the band, with the forward
// substitution interleaved (y_b = L_bb^-1 s_b, then s_i -= L_ib y_b) and one
// step of look-ahead: while waves 1.. apply the trailing update of column b,
// wave 0 updates and factors the next diagonal tile.  The current panel
// L_ib (b < i <= b + band) is kept in LDS for the trailing update.
constexpr int kSmallThreads = 512;
constexpr int kPanelSlots = kSmallMaxNpad / NB;     // 16: panel tiles, then the diagonal inverses
__global__ void __launch_bounds__(kSmallThreads) k_chol_small(DevPlan D, double* __restrict__ Aall,
                                                              double* __restrict__ Linvall, double* __restrict__ xall,
                                                              DevStatus* __restrict__ stall) {
  extern __shared__ double P[];                 // [kPanelSlots][NB * NB], swizzled
  __shared__ double T[NB * LD];                 // diagonal tile being factored; the solution in the back-solve
  __shared__ double Li[2][NB * LD];             // L_bb^-1 of the current and the next column
  __shared__ double U[16 * 17];
  __shared__ double rinv[NB];
  __shared__ double yv[kSmallMaxNpad];          // right-hand side -> y = L^-1 s -> running rhs of L^T x = y
  const int w = blockIdx.x;
  const WinDev& W = D.win[w];
  const int npad = W.npad, nblk = W.nblk, n = W.n;
  if (npad > kSmallMaxNpad) return;
  const int bw = W.band;
  double* A = Aall + W.A_off;
  double* Lv = Linvall + W.Linv_off;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int NW = kSmallThreads / 64;
  for (int r = tid; r < npad; r += kSmallThreads) yv[r] = A[(size_t)npad * npad + r];
  if (wave == 0) {
    tile_to_lds(T, A, npad);
    const int bad = factor_invert32(T, Li[0], U, rinv);
    if (bad >= 0 && lane == 0 && bad < n) set_status(stall + w, VI_ENOTPD, bad);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = lane + 64 * it;
      Lv[e] = Li[0][(e >> 5) * LD + (e & 31)];
    }
  }
  __syncthreads();
  if (wave == 0) fwd_block(Li[0], yv);
  __syncthreads();
  for (int b = 0; b < nblk; ++b) {
    const int hi = min(b + bw, nblk - 1);       // last block row of column b inside the band
    const int m = hi - b;                       // panel tiles below the diagonal
    const double* Lc = Li[b & 1];
    // panel: L_ib = A_ib L_bb^-T, b < i <= hi -> global (for the back-solve) and LDS
    for (int u = wave; u < m; u += NW) {
      const int i = b + 1 + u;
      double4_t acc[2][2];
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) acc[bm][bn] = double4_t{0.0, 0.0, 0.0, 0.0};
      double* Aib = A + (size_t)(NB * i) * npad + NB * b;
      mm32_abt(acc, Aib, npad, Lc, LD, 1.0);
      store_tile32(acc, Aib, npad);
      double* Pu = P + u * NB * NB;
      const int mrow = lane & 15, kq = lane >> 4;
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
          for (int r = 0; r < 4; ++r) Pu[swz(16 * bm + kq + 4 * r, 16 * bn + mrow)] = acc[bm][bn][r];
    }
    __syncthreads();
    // forward substitution: s_i -= L_ib y_b (one thread per row of the panel)
    {
      const int u = tid >> 5, r = tid & 31;
      if (u < m) {
        const double* Pu = P + u * NB * NB;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) v += Pu[swz(r, q)] * yv[NB * b + q];
        yv[NB * (b + 1 + u) + r] -= v;
      }
    }
    if (m > 0) {
      if (wave == 0) {
        // look-ahead: the next diagonal tile (its rhs rows were updated by this
        // wave just above), its factor, inverse and forward block
        const int nb1 = b + 1;
        double4_t acc[2][2];
        load_tile32(acc, A + (size_t)(NB * nb1) * npad + NB * nb1, npad);
        mm32_abt_lds(acc, P, P, -1.0);
        acc_to_lds(acc, T);
        double* Ln = Li[nb1 & 1];
        const int bad = factor_invert32(T, Ln, U, rinv);
        if (bad >= 0 && lane == 0 && NB * nb1 + bad < n) set_status(stall + w, VI_ENOTPD, NB * nb1 + bad);
#pragma unroll
        for (int it = 0; it < 16; ++it) {
          const int e = lane + 64 * it;
          Lv[(size_t)nb1 * NB * NB + e] = Ln[(e >> 5) * LD + (e & 31)];
        }
        fwd_block(Ln, yv + NB * nb1);
      } else {
        // trailing update (i, j), b < j <= i <= hi, except (b+1, b+1)
        const int ntri = m * (m + 1) / 2;
        for (int u = wave; u < ntri; u += NW - 1) {
          int jj = 0, rem = u;
          while (rem >= m - jj) { rem -= m - jj; ++jj; }
          const int j = b + 1 + jj, i = j + rem;
          double4_t acc[2][2];
          double* Aij = A + (size_t)(NB * i) * npad + NB * j;
          load_tile32(acc, Aij, npad);
          mm32_abt_lds(acc, P + (i - b - 1) * NB * NB, P + (j - b - 1) * NB * NB, -1.0);
          store_tile32(acc, Aij, npad);
        }
      }
    }
    __syncthreads();
  }
  // back-substitution x = L^-T y inside the band; the diagonal inverses go to LDS
  double* xs = T;
  for (int e = tid; e < nblk * NB * NB; e += kSmallThreads) {
    const int bb = e >> 10, rc = e & 1023;
    P[bb * NB * NB + swz(rc >> 5, rc & 31)] = Lv[e];
  }
  __syncthreads();
  const int q = lane & 31, half = lane >> 5;
  for (int b = nblk - 1; b >= 0; --b) {
    const int c0 = max(0, b - bw);
    // prefetch this wave's first block L_bc while x_b is formed
    const int cw = c0 + wave;
    double pre[16];
    if (cw < b) {
#pragma unroll
      for (int uu = 0; uu < 16; ++uu) pre[uu] = A[(size_t)(NB * b + 16 * half + uu) * npad + NB * cw + q];
    }
    if (tid < NB) {
      const double* Lb = P + b * NB * NB;
      double v = 0.0;
#pragma unroll
      for (int r = 0; r < NB; ++r) v += Lb[swz(r, tid)] * yv[NB * b + r];
      xs[NB * b + tid] = v;
    }
    __syncthreads();
    for (int c = cw; c < b; c += NW) {
      double v = 0.0;
      if (c == cw) {
#pragma unroll
        for (int uu = 0; uu < 16; ++uu) v += pre[uu] * xs[NB * b + 16 * half + uu];
      } else {
#pragma unroll
        for (int uu = 0; uu < 16; ++uu)
          v += A[(size_t)(NB * b + 16 * half + uu) * npad + NB * c + q] * xs[NB * b + 16 * half + uu];
      }
      v += __shfl_xor(v, 32);
      if (half == 0) yv[NB * c + q] -= v;
    }
    __syncthreads();
  }
  double* x = xall + W.x_off;
  for (int i = tid; i < npad; i += kSmallThreads) x[i] = (i < n) ? xs[i] : 0.0;
}

// x = L^-T y per window (blockIdx.x); 1024 threads.  After an aborted
// factorisation every window is marked failed (its state is then left alone).
__global__ void __launch_bounds__(1024) k_chol_backsolve(DevPlan D, const double* __restrict__ Aall,
                                                         const double* __restrict__ Linvall, double* __restrict__ xall,
                                                         const int* __restrict__ sync, DevStatus* __restrict__ stall) {
  extern __shared__ double sh[];
  const WinDev& W = D.win[blockIdx.x];
  const int n = W.n, npad = W.npad, nblk = W.nblk;
  if (npad <= kSmallMaxNpad) return;
  if (load_flag(sync + 1) != 0) {
    if (threadIdx.x == 0) set_status(stall + blockIdx.x, VI_EDEVICE, -1);
    return;
  }
  const double* A = Aall + W.A_off;
  const double* Lv = Linvall + W.Linv_off;
  double* tv = sh;            // running right-hand side [npad]
  double* xs = sh + npad;     // solution [npad]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane & 31, half = lane >> 5;
  for (int r = tid; r < npad; r += 1024) tv[r] = A[(size_t)npad * npad + r];
  __syncthreads();
  for (int b = nblk - 1; b >= 0; --b) {
    // prefetch this wave's first block L_bc (c = wave) while x_b is formed
    double pre[16];
    const bool has = wave < b;
    if (has) {
#pragma unroll
      for (int u = 0; u < 16; ++u) pre[u] = A[(size_t)(NB * b + 16 * half + u) * npad + NB * wave + q];
    }
    if (tid < NB) {
      const double* Lb = Lv + (size_t)b * NB * NB;
      double v = 0.0;
      for (int r = tid; r < NB; ++r) v += Lb[r * NB + tid] * tv[NB * b + r];
      xs[NB * b + tid] = v;
    }
    __syncthreads();
    for (int c = wave; c < b; c += 16) {
      double v = 0.0;
      if (c == wave) {
#pragma unroll
        for (int u = 0; u < 16; ++u) v += pre[u] * xs[NB * b + 16 * half + u];
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u)
          v += A[(size_t)(NB * b + 16 * half + u) * npad + NB * c + q] * xs[NB * b + 16 * half + u];
      }
      v += __shfl_xor(v, 32);
      if (half == 0) tv[NB * c + q] -= v;
    }
    __syncthreads();
  }
  double* x = xall + W.x_off;
  for (int i = tid; i < npad; i += 1024) x[i] = (i < n) ? xs[i] : 0.0;
}

}  // namespace

void chol_set_attributes() {
  const int lds = (int)(sizeof(double) * 2 * ((15 * kMaxKeyframes + NB - 1) / NB * NB));
  (void)hipFuncSetAttribute((const void*)k_chol_backsolve, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_chol_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * kPanelSlots * NB * NB));
}

void launch_chol(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st) {
  int npad_max = 0;
  bool small = false;
  for (const WinDev& W : P.win) {
    npad_max = std::max(npad_max, W.npad);
    small = small || W.npad <= kSmallMaxNpad;
  }
  if (small)
    hipLaunchKernelGGL(k_chol_small, dim3(P.n_win), dim3(kSmallThreads), sizeof(double) * kPanelSlots * NB * NB, s, D,
                       w.A, w.Linv, w.x, st);
  if (P.n_tickets > 0) {
    const int grid = std::min(P.n_tickets, kMaxDataflowWG);
    hipLaunchKernelGGL(k_chol_df, dim3(grid), dim3(64), 0, s, D, P.n_tickets, w.A, w.Linv, w.flags, w.sync, st);
    hipLaunchKernelGGL(k_chol_backsolve, dim3(P.n_win), dim3(1024), sizeof(double) * 2 * npad_max, s, D, w.A,
                       w.Linv, w.x, w.sync, st);
  }
}

}  // namespace vi
