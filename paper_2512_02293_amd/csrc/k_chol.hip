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
//                                              straight from global memory,
//                                              those of k + 1 in flight
//                                              during the MFMAs of k; one
//                                              acquire per run of published k)
//   i == j : factor and invert X (register-resident 8 x 8 leaves joined by MFMA);
//   i != j : L_ij = X L_jj^-T                 (FP64 MFMA)
// and publishes the result with a release flag.  Tiles are handed out by an
// atomic ticket counter in column-major order (column j, then window, then
// row i), and a tile only ever waits for tiles of smaller tickets, which were
// taken by running workgroups: every wait ends without any assumption on
// how many workgroups are resident.  Every wait is also bounded: past the
// limit the batch is aborted (VI_EDEVICE) and every workgroup exits.
//
// Back-substitution x = L^-T y is a second dataflow, over block columns:
// column c subtracts L_bc^T x_b from y_c as the x_b (b > c) are published,
// then publishes x_c = L_cc^-T t_c.
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

// The lane index behind an opaque move: address arithmetic derived from it
// is recomputed where it is used instead of being hoisted out of the step
// loops and held (spilled) across them.
__device__ __forceinline__ int lane_id() {
  int l;
  asm volatile("v_and_b32 %0, 63, %1" : "=v"(l) : "v"((int)threadIdx.x));
  return l;
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
  // hardware reciprocal square root (relative error about 2^-23), then one
  // third-order step: with e = 1 - v y^2, v^-1/2 = y (1 - e)^-1/2 =
  // y (1 + e/2 + 3 e^2/8 + 5 e^3/16 + ...); the dropped terms are below 2^-64
  // relative.  Four dependent operations after the estimate, where two
  // Newton steps take six (the pivot chain of the leaf factor runs through it).
  const double y = __builtin_amdgcn_rsq(v);
  const double e = __builtin_fma(-v, y * y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(0.375, e, 0.5), y);
}

// ---------------------------------------------------------------------------
// one-wave helpers on 16 x 16 blocks in LDS (row-major with stride ld)
// ---------------------------------------------------------------------------
// acc += sA * (A B) for 16 x 16 blocks: A(m, q) = Aop[m * lda + q] (or its
// transpose when ta), B(q, n) = Bop[q * ldb + n] (or Bop[n * ldb + q] when tb).
__device__ __forceinline__ double4_t mm16(double4_t acc, const double* Aop, int lda, bool ta, const double* Bop,
                                          int ldb, bool tb, double sA) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
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
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
  double4_t v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = M[(kq + 4 * r) * ld + mrow];
  return v;
}

__device__ __forceinline__ void store16(double* M, int ld, double4_t v) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) M[(kq + 4 * r) * ld + mrow] = v[r];
}

// Cholesky factor L and inverse X = L^-1 of an 8x8 SPD block M (stride ld),
// computed by every lane redundantly in registers (no cross-lane traffic;
// packed lower-triangular storage, entry (i, j) at i (i + 1) / 2 + j); X is
// written to D (stride ldd, zeros above the diagonal) by lane 0.  Returns the
// first bad pivot or -1.
__device__ __forceinline__ constexpr int tri8(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ __forceinline__ int leaf8_inv(const double* M, int ld, double* D, int ldd) {
  // right-looking, in place: L holds the partly reduced block until column j is final
  double L[36];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j <= i) L[tri8(i, j)] = M[i * ld + j];
  int bad = -1;
  double rv[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    // a pivot that is not positive is taken as 1 (so that the block stays
    // finite) and reported; the estimate starts from |pivot| so that this
    // choice stays off the dependent chain from one pivot to the next
    const double piv = L[tri8(j, j)];
    const bool ok = piv > 0.0;
    if (!ok && bad < 0) bad = j;
    const double r = ok ? rsqrt_refined(__builtin_fabs(piv)) : 1.0;
    rv[j] = r;
    L[tri8(j, j)] = ok ? piv * r : 1.0;
#pragma unroll
    for (int i = 1; i < 8; ++i)
      if (i > j) L[tri8(i, j)] *= r;
#pragma unroll
    for (int i = 1; i < 8; ++i)
#pragma unroll
      for (int m = 1; m < 8; ++m)
        if (i > j && m > j && m <= i) L[tri8(i, m)] -= L[tri8(i, j)] * L[tri8(m, j)];
  }
  // X = L^-1: lane c (mod 8) forms column c by forward substitution against
  // e_c (x_r = 0 above the diagonal, x_c = 1 / L_cc), so that the eight
  // columns are computed side by side and stored with one write per row
  const int c = threadIdx.x & 7;
  double x[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q)
      if (q < r) v += L[tri8(r, q)] * x[q];
    x[r] = (r == c) ? rv[r] : ((r < c) ? 0.0 : -v * rv[r]);
  }
  if ((threadIdx.x & 63) < 8) {
#pragma unroll
    for (int r = 0; r < 8; ++r) D[r * ldd + c] = x[r];
  }
  return bad;
}

// One wave: inverse Cholesky factor of the 16x16 SPD block M (stride ld) into
// Mi (stride ldi), by two register-resident 8x8 leaves:
//   X11 = chol(A11)^-1, L21 = A21 X11^T, X22 = chol(A22 - L21 L21^T)^-1,
//   X21 = -X22 L21 X11.
// M's lower blocks are overwritten (L21, the updated A22).  S: 8 x 9 scratch.
// Returns the first bad pivot (0..15) or -1.
__device__ __forceinline__ int leaf16_factor_inverse(double* M, int ld, double* Mi, int ldi, double* S) {
  const int lane = threadIdx.x & 63, i = lane >> 3, j = lane & 7;
  int bad = leaf8_inv(M, ld, Mi, ldi);                        // X11
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
  const int bad2 = leaf8_inv(M + 8 * ld + 8, ld, Mi + 8 * ldi + 8, ldi);   // X22
  if (bad < 0 && bad2 >= 0) bad = 8 + bad2;
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
__device__ __forceinline__ int factor_invert32(double* T, double* Li, double* U) {
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
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
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

// acc += sA X X^T into a diagonal tile: the upper-right 16x16 quarter, which
// the tile's factor never reads, is not formed
__device__ __forceinline__ void mm32_aat_diag(double4_t (&acc)[2][2], const double* X, size_t ldx, double sA) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
  double a[2][8], b[2][8];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      b[h][s] = X[(16 * h + mrow) * ldx + 4 * s + kq];
      a[h][s] = sA * b[h][s];
    }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][s], b[0][s], acc[0][0], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][s], b[0][s], acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][s], b[1][s], acc[1][1], 0, 0, 0);
  }
}

__device__ __forceinline__ void load_tile32(double4_t (&acc)[2][2], const double* M, size_t ld) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bm][bn][r] = M[(16 * bm + kq + 4 * r) * ld + 16 * bn + mrow];
}

__device__ __forceinline__ void store_tile32(const double4_t (&acc)[2][2], double* M, size_t ld) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
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
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
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

// The same for a diagonal tile, acc += sA X X^T: the upper-right 16x16
// quarter, which no later step reads (the factor of a diagonal tile uses its
// lower blocks only), is not formed
__device__ __forceinline__ void mm32_abt_lds_diag(double4_t (&acc)[2][2], const double* X, double sA) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    double a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      b[h] = X[swz(16 * h + mrow, 4 * s + kq)];
      a[h] = sA * b[h];
    }
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc[0][0], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[0], acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], acc[1][1], 0, 0, 0);
  }
}

// acc(2x2 blocks of 16x16) += X Y^T over K = 32, X a swizzled LDS tile, Y a
// padded (stride LD) LDS tile
__device__ __forceinline__ void mm32_abt_swz_pad(double4_t (&acc)[2][2], const double* X, const double* Y) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    double a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a[h] = X[swz(16 * h + mrow, 4 * s + kq)];
      b[h] = Y[(16 * h + mrow) * LD + 4 * s + kq];
    }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm], b[bn], acc[bm][bn], 0, 0, 0);
  }
}

__device__ __forceinline__ void acc_to_swz(const double4_t (&acc)[2][2], double* S) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) S[swz(16 * bm + kq + 4 * r, 16 * bn + mrow)] = acc[bm][bn][r];
}

__device__ __forceinline__ void swz_to_acc(double4_t (&acc)[2][2], const double* S) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bm][bn][r] = S[swz(16 * bm + kq + 4 * r, 16 * bn + mrow)];
}

// LDS flags between the waves of one workgroup.  LDS operations of a wave
// complete in order, so a flag written after the wave's data writes have
// completed is seen only after them, and reads issued after the flag was seen
// return the new data.
__device__ __forceinline__ void lds_publish(int* f, int v) {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // this wave's LDS writes are done
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  asm volatile("" ::: "memory");
}

// Wait until *f == v in every active lane (f may differ between lanes); the
// publishing waves never wait on the waiting one, so the wait ends; it is
// bounded all the same.  Returns false when the bound was reached (the
// caller then fails the window: the data it waited for is not there).
__device__ __forceinline__ bool lds_wait(const int* f, int v) {
  bool ok = false;
  for (int spin = 0; spin < kSpinLimit; ++spin) {
    const bool pending = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != v;
    if (__ballot(pending) == 0) { ok = true; break; }
    __builtin_amdgcn_s_sleep(1);
  }
  asm volatile("" ::: "memory");
  return ok;
}

// Wait until *f >= v (a counter that only grows); bounded like lds_wait.
__device__ __forceinline__ bool lds_wait_ge(const int* f, int v) {
  bool ok = false;
  for (int spin = 0; spin < kSpinLimit; ++spin) {
    const bool pending = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < v;
    if (__ballot(pending) == 0) { ok = true; break; }
    __builtin_amdgcn_s_sleep(1);
  }
  asm volatile("" ::: "memory");
  return ok;
}

// global 32 x 32 tile -> swizzled LDS tile, all loads in flight at once (one wave)
__device__ __forceinline__ void tile_to_swz(double* S, const double* M, size_t ld) {
  double4_t acc[2][2];
  load_tile32(acc, M, ld);
  acc_to_swz(acc, S);
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

// A run of published tiles of a tile's k-loop: the number of consecutive
// k' = k, k + 1, ... (at most 32, below kend) whose flags (i, k') and (j, k')
// are both set, from one vector load of 64 flags (relaxed; the caller issues
// the acquire fence once for the whole run).
__device__ __forceinline__ int ready_run(const int* fi, const int* fj, int k, int kend) {
  const int lane = threadIdx.x & 63, off = lane & 31;
  const int* f = lane < 32 ? fi : fj;
  const int v = (k + off < kend) ? load_flag(f + k + off) : 0;
  const unsigned long long miss = __ballot(v == 0);
  const unsigned comb = (unsigned)miss | (unsigned)(miss >> 32);
  return comb ? __builtin_ctz(comb) : 32;
}

// Wait (whole wave) until *f is set, without a fence.  false: the batch was aborted.
__device__ __forceinline__ bool spin_flag(const int* f, int* sync) {
  int spins = 0;
  while (__builtin_amdgcn_readfirstlane(load_flag(f)) == 0) {
    if (__builtin_amdgcn_readfirstlane(load_flag(sync + 1)) != 0) return false;
    if (++spins > kSpinLimit) {
      if (threadIdx.x == 0) __hip_atomic_store(sync + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// MFMA operands of one update X -= L_ik L_jk^T: lane supplies A[m][q] = L_ik[m][q]
// (negated) and B[q][n] = L_jk[n][q] for its 16 rows and 4-column slices
__device__ __forceinline__ void load_update(double (&a)[2][8], double (&b)[2][8], const double* Li, const double* Lj,
                                            size_t ld) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a[h][s2] = -Li[(size_t)(16 * h + mrow) * ld + 4 * s2 + kq];
      b[h][s2] = Lj[(size_t)(16 * h + mrow) * ld + 4 * s2 + kq];
    }
}

__device__ __forceinline__ void mfma_update(double4_t (&acc)[2][2], const double (&a)[2][8], const double (&b)[2][8]) {
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm][s2], b[bn][s2], acc[bm][bn], 0, 0, 0);
}

// the same into a diagonal tile, acc += a a^T: its upper-right 16x16 quarter,
// which the tile's factor never reads, is not formed
__device__ __forceinline__ void mfma_update_diag(double4_t (&acc)[2][2], const double (&a)[2][8]) {
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) {
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][s2], a[0][s2], acc[0][0], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][s2], a[0][s2], acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][s2], a[1][s2], acc[1][1], 0, 0, 0);
  }
}

// k-loop of a dataflow ticket over [k, kend): X -= L_ik L_jk^T, and with PAIR
// also Y += L_ik L_ik^T (ONLY2: Y alone; the operand a = -L_ik serves as both
// MFMA inputs, so Y holds the negated diagonal update), over runs of
// published k with one acquire per run and the operands of k + 1 loaded while
// the MFMAs of k run.  false: the batch was aborted.
template <bool PAIR, bool ONLY2>
__device__ __forceinline__ bool df_kloop(double4_t (&acc)[2][2], double4_t (&acc2)[2][2], const double* Ri,
                                         const double* Rj, size_t npad, const int* fi, const int* fj, int k, int kend,
                                         int* sync) {
  auto step = [&](const double (&a)[2][8], const double (&b)[2][8]) {
    if (!ONLY2) mfma_update(acc, a, b);
    if (PAIR || ONLY2) mfma_update_diag(acc2, a);
  };
  while (k < kend) {
    const int run = ready_run(fi, fj, k, kend);
    if (run == 0) {
      if (!spin_flag(fi + k, sync)) return false;
      if (fj != fi && !spin_flag(fj + k, sync)) return false;
      continue;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int ke = k + run;
    double a0[2][8], b0[2][8], a1[2][8], b1[2][8];
    load_update(a0, b0, Ri + NB * k, Rj + NB * k, npad);
    for (; k < ke; k += 2) {
      const bool has1 = k + 1 < ke;
      if (has1) load_update(a1, b1, Ri + NB * (k + 1), Rj + NB * (k + 1), npad);
      step(a0, b0);
      if (!has1) { ++k; break; }
      if (k + 2 < ke) load_update(a0, b0, Ri + NB * (k + 2), Rj + NB * (k + 2), npad);
      step(a1, b1);
    }
    k = ke;
  }
  return true;
}

// L_ij = X L_jj^-T for the tile X in T (LDS, padded), L_jj^-1 row-major at Li
__device__ __forceinline__ void solve_panel(double4_t (&out)[2][2], const double* T, const double* Li) {
  const int lane = lane_id(), mrow = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) out[bm][bn] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) {
    double a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a[h] = T[(16 * h + mrow) * LD + 4 * s2 + kq];
      b[h] = Li[(16 * h + mrow) * NB + 4 * s2 + kq];
    }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
        out[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm], b[bn], out[bm][bn], 0, 0, 0);
  }
}

// Tickets: (window, (i << 16) | j), with kPairTicket set on the ticket of
// tile (j + 1, j) when it also carries the diagonal tile (j + 1, j + 1): that
// wave accumulates X_ij and X_ii together (the operands L_ik are shared),
// publishes L_ij as soon as L_jj^-1 is in, then subtracts L_ij L_ij^T, factors
// the diagonal tile and publishes L_ii^-1 itself, so that the chain from one
// diagonal factor to the next holds one hand-off instead of two.
constexpr int kPairTicket = kPairTicketFlag;

__global__ void __launch_bounds__(64) k_chol_df(DevPlan D, int ntickets, double* __restrict__ Aall,
                                                double* __restrict__ Linvall, int* __restrict__ flagsall,
                                                int* __restrict__ sync, DevStatus* __restrict__ stall) {
  __shared__ double T[NB * LD];
  __shared__ double Lt[NB * LD];
  __shared__ double U[16 * 17];
  const int lane = threadIdx.x;
  while (true) {
    int t = 0;
    if (lane == 0) t = atomicAdd(sync, 1);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= ntickets) return;
    const int w = D.chol_tiles[2 * t];
    const int ij = D.chol_tiles[2 * t + 1];
    const bool pair = (ij & kPairTicket) != 0;
    const int i = (ij >> 16) & 0x3fff, j = ij & 0xffff;
    const WinDev& W = D.win[w];
    const int npad = W.npad, nblk = W.nblk;
    double* A = Aall + W.A_off;
    double* Lv = Linvall + W.Linv_off;
    int* fl = flagsall + W.flag_off;
    const int* fc = D.chol_fc + W.fc_off;
    const double* Ri = A + (size_t)(NB * i) * npad;
    const double* Rj = A + (size_t)(NB * j) * npad;
    // X = S_ij - sum_k L_ik L_jk^T; L_ik and L_jk are zero left of the
    // envelope (k < fc[i] or k < fc[j])
    double4_t acc[2][2], acc2[2][2];
    load_tile32(acc, Ri + NB * j, npad);
    const int k1 = max(fc[i], fc[j]);
    if (!pair) {
      if (!df_kloop<false, false>(acc, acc2, Ri, Rj, npad, fl + i * nblk, fl + j * nblk, k1, j, sync)) return;
    } else {
      // and X2 = S_ii - sum_{k < j} L_ik L_ik^T alongside (k >= fc[i]), as
      // its negative -S_ii + sum L_ik L_ik^T
      load_tile32(acc2, Ri + NB * i, npad);
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) acc2[bm][bn] = -acc2[bm][bn];
      if (!df_kloop<true, true>(acc, acc2, Ri, Ri, npad, fl + i * nblk, fl + i * nblk, fc[i], k1, sync)) return;
      if (!df_kloop<true, false>(acc, acc2, Ri, Rj, npad, fl + i * nblk, fl + j * nblk, k1, j, sync)) return;
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) acc2[bm][bn] = -acc2[bm][bn];
    }
    acc_to_lds(acc, T);
    __syncthreads();
    if (i == j) {
      // factor and invert (register leaves joined by MFMA), publish L_jj^-1
      const int bad = factor_invert32(T, Lt, U);
      if (bad >= 0 && lane == 0 && NB * j + bad < W.n) set_status(stall + w, VI_ENOTPD, NB * j + bad);
      double* Lo = Lv + (size_t)j * NB * NB;
#pragma unroll
      for (int it = 0; it < 16; ++it) {
        const int e = lane + 64 * it;
        Lo[e] = Lt[(e >> 5) * LD + (e & 31)];
      }
      publish(fl + j * nblk + j);
    } else {
      if (!wait_flag(fl + j * nblk + j, sync)) return;
      // L_ij = X L_jj^-T: A[m][q] = X[m][q], B[q][n] = Linv[n][q]
      double4_t out[2][2];
      solve_panel(out, T, Lv + (size_t)j * NB * NB);
      store_tile32(out, A + (size_t)(NB * i) * npad + NB * j, npad);
      publish(fl + i * nblk + j);
      if (pair) {
        // X2 -= L_ij L_ij^T (L_ij through LDS into the operand layout), then
        // factor and invert the diagonal tile (i, i) and publish L_ii^-1
        __syncthreads();
        acc_to_lds(out, Lt);
        __syncthreads();
        mm32_aat_diag(acc2, Lt, LD, -1.0);
        acc_to_lds(acc2, T);
        __syncthreads();
        const int bad = factor_invert32(T, Lt, U);
        if (bad >= 0 && lane == 0 && NB * i + bad < W.n) set_status(stall + w, VI_ENOTPD, NB * i + bad);
        double* Lo = Lv + (size_t)i * NB * NB;
#pragma unroll
        for (int it = 0; it < 16; ++it) {
          const int e = lane + 64 * it;
          Lo[e] = Lt[(e >> 5) * LD + (e & 31)];
        }
        publish(fl + i * nblk + i);
      }
    }
    __syncthreads();
  }
}

// Whole factorisation and solve of one small window per 512-thread workgroup.
// Right-looking over 32-wide block columns inside the band, with the forward
// substitution interleaved (y_b = L_bb^-1 s_b, then s_i -= L_ib y_b) and one
// step of look-ahead: while waves 1.. apply the trailing update of column b,
// wave 0 updates and factors the next diagonal tile.  The current panel
// L_ib (b < i <= b + band) is kept in LDS for the trailing update.
// With a band of at most kLdsBand tiles the tiles that the next step starts
// from never leave LDS: the trailing update of column b writes the updated
// tiles of column b + 1 (below the diagonal) into one of two column buffers
// and the updated diagonal tile b + 2 into one of two diagonal buffers, so
// that neither the next panel nor the next look-ahead waits on global
// memory.  Wider bands keep every updated tile in global memory.
constexpr int kSmallThreads = 512;
constexpr int kPanelSlots = kSmallMaxNpad / NB;     // 16: panel tiles, then the diagonal inverses
constexpr int kLdsBand = (kPanelSlots - 2) / 2;     // 7: two column buffers and two diagonal tiles
__global__ void __launch_bounds__(kSmallThreads) k_chol_small(DevPlan D, double* __restrict__ Aall,
                                                              double* __restrict__ Linvall, double* __restrict__ xall,
                                                              DevStatus* __restrict__ stall) {
  extern __shared__ double P[];                 // [kPanelSlots][NB * NB], swizzled
  __shared__ double T[NB * LD];                 // diagonal tile being factored; the solution in the back-solve
  __shared__ double Li[2][NB * LD];             // L_bb^-1 of the current and the next column
  __shared__ double U[16 * 17];
  __shared__ double yv[kSmallMaxNpad];          // right-hand side -> y = L^-1 s -> running rhs of L^T x = y
  __shared__ int ydone;                         // step b once block b of yv holds y_b = L_bb^-1 s_b
  __shared__ int pready[kPanelSlots];           // step b + 1 once panel tile u of column b is in LDS
  __shared__ int xdone;                         // back-substitution: blocks of x published so far
  const int w = blockIdx.x;
  const WinDev& W = D.win[w];
  const int npad = W.npad, nblk = W.nblk, n = W.n;
  if (npad > kSmallMaxNpad || stall[w].conv != 0) return;   // frozen windows take no step
  const int bw = W.band;
  double* A = Aall + W.A_off;
  double* Lv = Linvall + W.Linv_off;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int NW = kSmallThreads / 64;
  for (int r = tid; r < npad; r += kSmallThreads) yv[r] = A[(size_t)npad * npad + r];
  const bool lds = bw <= kLdsBand;
  // LDS mode: column buffer c & 1 holds tiles (i, c), c < i <= c + band, at
  // slot i - c - 1; diagonal buffer c & 1 holds tile (c, c)
  auto colbuf = [&](int c) { return P + (size_t)(c & 1) * kLdsBand * NB * NB; };
  auto diagbuf = [&](int c) { return P + (size_t)(2 * kLdsBand + (c & 1)) * NB * NB; };
  if (wave == 0) {
    tile_to_lds(T, A, npad);
    const int bad = factor_invert32(T, Li[0], U);
    if (bad >= 0 && lane == 0 && bad < n) set_status(stall + w, VI_ENOTPD, bad);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = lane + 64 * it;
      Lv[e] = Li[0][(e >> 5) * LD + (e & 31)];
    }
  } else if (lds) {
    // column 0 below the diagonal and diagonal tile 1, as given
    const int m0 = min(bw, nblk - 1);
    for (int u = wave - 1; u <= m0; u += NW - 1) {
      if (u < m0) tile_to_swz(colbuf(0) + u * NB * NB, A + (size_t)(NB * (1 + u)) * npad, npad);
      else if (nblk > 1) tile_to_swz(diagbuf(1), A + (size_t)NB * npad + NB, npad);
    }
  }
  __syncthreads();
  if (wave == 0) fwd_block(Li[0], yv);
  if (tid == 0) ydone = 0;
  if (tid == 0) xdone = 0;
  if (tid < kPanelSlots) pready[tid] = 0;
  __syncthreads();
  // Wave roles: wave 0 carries the chain of diagonal factorisations; wave 4
  // shares its SIMD and so takes the memory work (copies, the deferred global
  // copy of L_bb^-1, panel tiles beyond the seventh) and then, in steps with
  // at least 14 trailing tiles, every seventh of them; the six other waves
  // take the panel, the forward substitution and the rest of the trailing
  // update.
  // a bounded wait that expired fails the window (VI_EDEVICE): the solution is
  // not used and the window's state is left as it was
  auto wait_eq = [&](const int* f, int v) {
    if (!lds_wait(f, v) && lane == 0) set_status(stall + w, VI_EDEVICE, -2);
  };
  auto wait_ge = [&](const int* f, int v) {
    if (!lds_wait_ge(f, v) && lane == 0) set_status(stall + w, VI_EDEVICE, -2);
  };
  const int pw = wave < 4 ? wave : (wave == 4 ? 7 : wave - 1);   // panel order: 0,1,2,3,5,6,7, then 4
  const int cw = wave < 4 ? wave - 1 : wave - 2;                 // compute worker 0..5 (waves 1-3, 5-7)
  for (int b = 0; b < nblk; ++b) {
    const int hi = min(b + bw, nblk - 1);       // last block row of column b inside the band
    const int m = hi - b;                       // panel tiles below the diagonal
    const double* Lc = Li[b & 1];
    double* Pc = lds ? colbuf(b) : P;           // the panel of column b, swizzled
    // global copy of L_bb^-1 (factored during the previous step) for the back-solve
    if (b > 0 && wave == 4) {
#pragma unroll
      for (int it = 0; it < 16; ++it) {
        const int e = lane + 64 * it;
        Lv[(size_t)b * NB * NB + e] = Lc[(e >> 5) * LD + (e & 31)];
      }
    }
    // y_b = L_bb^-1 s_b (its rows were completed during the previous step) on
    // wave 1, off the look-ahead chain; the forward substitution waits for it
    if (b > 0 && wave == 1) {
      fwd_block(Lc, yv + NB * b);
      lds_publish(&ydone, b);
    }
    // panel: L_ib = A_ib L_bb^-T, b < i <= hi -> global (for the back-solve) and LDS
    for (int u = pw; u < m; u += NW) {
      const int i = b + 1 + u;
      double4_t acc[2][2];
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) acc[bm][bn] = double4_t{0.0, 0.0, 0.0, 0.0};
      double* Aib = A + (size_t)(NB * i) * npad + NB * b;
      double* Pu = Pc + u * NB * NB;
      if (lds)
        mm32_abt_swz_pad(acc, Pu, Lc);
      else
        mm32_abt(acc, Aib, npad, Lc, LD, 1.0);
      store_tile32(acc, Aib, npad);
      acc_to_swz(acc, Pu);                      // same wave, reads of Pu done: in-place is safe
      lds_publish(&pready[u], b + 1);
    }
    // no barrier here: the look-ahead needs only its own panel tile, and the
    // other consumers wait for the flags of the tiles they read (the panel's
    // global copy is read only by the back-solve, after full barriers)
    // forward substitution: s_i -= L_ib y_b, one thread per row of the panel
    // on the six compute waves, once y_b is in
    if (wave != 0 && wave != 4) {
      wait_eq(&ydone, b);
      const int t6 = cw * 64 + lane;
      for (int u = t6 >> 5; u < m; u += 12) {
        const int r = t6 & 31;
        wait_eq(&pready[u], b + 1);
        const double* Pu = Pc + u * NB * NB;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) v += Pu[swz(r, q)] * yv[NB * b + q];
        yv[NB * (b + 1 + u) + r] -= v;
      }
    }
    if (m > 0) {
      if (wave == 0) {
        // look-ahead: the next diagonal tile, its factor and inverse
        const int nb1 = b + 1;
        double4_t acc[2][2];
        if (lds)
          swz_to_acc(acc, diagbuf(nb1));
        else
          load_tile32(acc, A + (size_t)(NB * nb1) * npad + NB * nb1, npad);
        mm32_abt_lds_diag(acc, Pc, -1.0);
        acc_to_lds(acc, T);
        double* Ln = Li[nb1 & 1];
        const int bad = factor_invert32(T, Ln, U);
        if (bad >= 0 && lane == 0 && NB * nb1 + bad < n) set_status(stall + w, VI_ENOTPD, NB * nb1 + bad);
        // its global copy and y_{b+1} are formed during the next step
      } else {
        // trailing update (i, j), b < j <= i <= hi, except (b+1, b+1); in LDS
        // mode also the copies of the next step's inputs that no update
        // touches here (the new band row of column b + 1, diagonal b + 2)
        const int ntri = m * (m + 1) / 2;
        const int hi1 = min(b + 1 + bw, nblk - 1);
        const bool cp_row = lds && hi1 > hi;                    // tile (hi1, b + 1), as given
        const bool cp_diag = lds && b + 2 < nblk && b + 2 > hi;  // tile (b + 2, b + 2), as given
        if (wave == 4) {
          if (cp_row)
            tile_to_swz(colbuf(b + 1) + (hi1 - b - 2) * NB * NB, A + (size_t)(NB * hi1) * npad + NB * (b + 1),
                        npad);
          if (cp_diag) tile_to_swz(diagbuf(b + 2), A + (size_t)(NB * (b + 2)) * npad + NB * (b + 2), npad);
        }
        // workers: the six compute waves and, after its copies, wave 4, whose
        // SIMD also runs the look-ahead chain.  A wave's tiles run one after
        // the other, so the step takes about as long as the largest number of
        // tiles per wave: wave 4 joins only when a seventh worker lowers that
        // number (at least 14 tiles), and otherwise leaves SIMD 0 to the chain
        // (the same tiles per wave, and a faster chain).
        // Each tile's successor is loaded while the tile is updated (one
        // global latency per wave and step instead of one per tile).
        const int tw = (wave == 4) ? NW - 2 : cw;
        const int nt = ntri - 1;
        const int nwk = (nt + 6) / 7 < (nt + 5) / 6 ? NW - 1 : NW - 2;
        auto tile_of = [&](int u, int& i, int& j) {
          int jj = 0, rem = u;
          while (rem >= m - jj) { rem -= m - jj; ++jj; }
          j = b + 1 + jj;
          i = j + rem;
        };
        double4_t nxt[2][2];
        if (tw < nwk && 1 + tw < ntri) {
          int i, j;
          tile_of(1 + tw, i, j);
          load_tile32(nxt, A + (size_t)(NB * i) * npad + NB * j, npad);
        }
        for (int u = tw < nwk ? 1 + tw : ntri; u < ntri; u += nwk) {
          int i, j;
          tile_of(u, i, j);
          double4_t acc[2][2];
#pragma unroll
          for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) acc[bm][bn] = nxt[bm][bn];
          if (u + nwk < ntri) {
            int i2, j2;
            tile_of(u + nwk, i2, j2);
            load_tile32(nxt, A + (size_t)(NB * i2) * npad + NB * j2, npad);
          }
          double* Aij = A + (size_t)(NB * i) * npad + NB * j;
          wait_eq(&pready[i - b - 1], b + 1);
          wait_eq(&pready[j - b - 1], b + 1);
          if (i == j)
            mm32_abt_lds_diag(acc, Pc + (i - b - 1) * NB * NB, -1.0);
          else
            mm32_abt_lds(acc, Pc + (i - b - 1) * NB * NB, Pc + (j - b - 1) * NB * NB, -1.0);
          if (lds && j == b + 1)
            acc_to_swz(acc, colbuf(b + 1) + (i - b - 2) * NB * NB);
          else if (lds && i == b + 2 && j == b + 2)
            acc_to_swz(acc, diagbuf(b + 2));
          else
            store_tile32(acc, Aij, npad);
        }
      }
    }
    __syncthreads();
  }
  // back-substitution x = L^-T y inside the band, as a dataflow between the
  // waves instead of two barriers per block: block c of x, its diagonal
  // inverse and every update of its right-hand side belong to wave c mod NW.
  // For b = nblk-1 .. 0 the owner of block b forms x_b = L_bb^-T y_b (all its
  // updates are in) and publishes it (xdone = nblk - b, in order of b); the
  // owners of the blocks c in [b - band, b) then apply y_c -= L_bc^T x_b with
  // the tile of L_bc loaded before they wait for x_b.
  double* xs = T;
  for (int c = wave; c < nblk; c += NW) {
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = lane + 64 * it;
      P[c * NB * NB + swz(e >> 5, e & 31)] = Lv[(size_t)c * NB * NB + e];
    }
  }
  const int q = lane & 31, half = lane >> 5;
  for (int b = nblk - 1; b >= 0; --b) {
    if (b % NW == wave) {
      wait_ge(&xdone, nblk - 1 - b);        // x_{b+1} is out, so is the last update of y_b
      if (lane < NB) {
        const double* Lb = P + b * NB * NB;
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < NB; ++r) v += Lb[swz(r, lane)] * yv[NB * b + r];
        xs[NB * b + lane] = v;
      }
      lds_publish(&xdone, nblk - b);
    }
    const int c0 = max(0, b - bw);
    for (int c = c0 + ((wave - c0 % NW) + NW) % NW; c < b; c += NW) {
      double pre[16];
#pragma unroll
      for (int uu = 0; uu < 16; ++uu) pre[uu] = A[(size_t)(NB * b + 16 * half + uu) * npad + NB * c + q];
      wait_ge(&xdone, nblk - b);
      double v = 0.0;
#pragma unroll
      for (int uu = 0; uu < 16; ++uu) v += pre[uu] * xs[NB * b + 16 * half + uu];
      v += __shfl_xor(v, 32);
      if (half == 0) yv[NB * c + q] -= v;
    }
  }
  __syncthreads();
  double* x = xall + W.x_off;
  for (int i = tid; i < npad; i += kSmallThreads) x[i] = (i < n) ? xs[i] : 0.0;
}

// x = L^-T y for the windows of the tile dataflow, as a dataflow over block
// columns: one 256-thread workgroup per (window, block column c), handed out
// by a ticket counter in decreasing c, so that a column only waits for
// columns of smaller tickets.  Column c starts from t_c = y_c and, as the
// solutions x_b of the columns b > c are published, subtracts L_bc^T x_b
// (tile (b, c) read before its x_b is waited for); then x_c = L_cc^-T t_c is
// written and published.  After an aborted factorisation (or a wait past its
// bound) the window is marked failed and the waits stop; every wave runs the
// same barriers either way.
__global__ void __launch_bounds__(256) k_chol_bs(DevPlan D, int t0, int nbs, const double* __restrict__ Aall,
                                                 const double* __restrict__ Linvall, double* __restrict__ xall,
                                                 int* __restrict__ flagsall, int* __restrict__ sync,
                                                 DevStatus* __restrict__ stall) {
  __shared__ double part[2][8][NB];
  __shared__ double tv[NB];
  __shared__ double xa[NB];
  __shared__ int tk;
  const int tid = threadIdx.x, q = tid & 31, r8 = tid >> 5, lane = tid & 63;
  while (true) {
    if (tid == 0) tk = atomicAdd(sync + 2, 1);
    __syncthreads();
    const int t = tk;
    __syncthreads();
    if (t >= nbs) return;
    // two block columns per ticket: c and c - 1 (when c > 0), so that the
    // chain of the back-substitution hands over between workgroups at every
    // second block only
    const int w = D.chol_tiles[2 * (t0 + t)];
    const int c = D.chol_tiles[2 * (t0 + t) + 1] & 0xffff;
    const bool two = c > 0;
    const int cb = c - 1;
    const WinDev& W = D.win[w];
    const int npad = W.npad, nblk = W.nblk;
    const double* A = Aall + W.A_off;
    const double* Lcc = Linvall + W.Linv_off + (size_t)c * NB * NB;
    double* x = xall + W.x_off;
    int* xf = flagsall + W.flag_off + (nblk + 1) * nblk;     // x_b published
    const int* fc = D.chol_fc + W.fc_off;
    bool aborted = load_flag(sync + 1) != 0;
    // columns q of L_cc^-1, of L_(c-1)(c-1)^-1 and of L_c,c-1 for the last
    // steps, loaded before any wait
    double lcc[NB], lbb[NB], lcb[NB];
    if (tid < NB) {
#pragma unroll
      for (int r = 0; r < NB; ++r) lcc[r] = Lcc[r * NB + q];
      if (two) {
        const double* Lbb = Linvall + W.Linv_off + (size_t)cb * NB * NB;
#pragma unroll
        for (int r = 0; r < NB; ++r) lbb[r] = Lbb[r * NB + q];
        const bool in_env = fc[c] <= cb;      // L_c,c-1 = 0 outside the envelope
#pragma unroll
        for (int r = 0; r < NB; ++r) lcb[r] = in_env ? A[(size_t)(NB * c + r) * npad + NB * cb + q] : 0.0;
      }
    }
    // t_c = y_c - sum_b L_bc^T x_b over b = nblk-1 .. c+1 (in that order),
    // and the same sum for column c - 1, inside the envelope: the flags of up
    // to 32 blocks are read at once (a block outside the envelope counts as
    // ready) and every ready run is summed with one acquire and its loads in
    // flight.  The tiles of block c + 1, whose x comes last (it waits for the
    // previous ticket), are loaded before any wait: the factor is final.
    double acc = 0.0, accb = 0.0;
    double vl[4], vlb[4];
    if (c + 1 < nblk) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const size_t row = (size_t)(NB * (c + 1) + r8 + 8 * u) * npad;
        vl[u] = fc[c + 1] <= c ? A[row + NB * c + q] : 0.0;
        vlb[u] = (two && fc[c + 1] <= cb) ? A[row + NB * cb + q] : 0.0;
      }
    }
    int b = nblk - 1;
    while (b > c) {
      const int bq = b - (lane & 31);
      const int ready = (bq > c && fc[bq] <= c) ? load_flag(xf + bq) : 1;   // blocks outside the envelope: not needed
      const unsigned long long miss = __ballot(ready == 0);
      const int run = min((int)(miss ? __builtin_ctzll(miss) : 32), b - c);
      if (run == 0) {
        if (!aborted) aborted = !spin_flag(xf + b, sync);
        if (aborted) {
          b = c;                      // the batch was aborted: no more waits
          break;
        }
        continue;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      for (const int bend = b - run; b > bend; --b) {
        if (fc[b] > c) continue;      // L_bc = 0 outside the envelope (and L_b,c-1)
        const bool use_b = two && fc[b] <= cb;
        double v[4], vb[4], xv[4];
        if (b == c + 1) {
#pragma unroll
          for (int u = 0; u < 4; ++u) { v[u] = vl[u]; vb[u] = vlb[u]; }
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const size_t row = (size_t)(NB * b + r8 + 8 * u) * npad;
            v[u] = A[row + NB * c + q];
            vb[u] = use_b ? A[row + NB * cb + q] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = x[NB * b + r8 + 8 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc += v[u] * xv[u];
          accb += vb[u] * xv[u];
        }
      }
    }
    part[0][r8][q] = acc;
    part[1][r8][q] = accb;
    __syncthreads();
    if (tid < NB) {
      double s = A[(size_t)npad * npad + NB * c + q];
#pragma unroll
      for (int k = 0; k < 8; ++k) s -= part[0][k][q];
      tv[q] = s;
    }
    __syncthreads();
    if (tid < NB) {
      // x_c = L_cc^-T t_c: x[q] = sum_r Linv[r][q] t[r]
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < NB; ++r) s += lcc[r] * tv[r];
      s = (NB * c + q < W.n) ? s : 0.0;
      x[NB * c + q] = s;
      xa[q] = s;
    }
    __syncthreads();
    if (two && tid < NB) {
      // t_c-1 = y_c-1 - sum_b L_b,c-1^T x_b - L_c,c-1^T x_c, then x_c-1
      double s = A[(size_t)npad * npad + NB * cb + q];
#pragma unroll
      for (int k = 0; k < 8; ++k) s -= part[1][k][q];
#pragma unroll
      for (int r = 0; r < NB; ++r) s -= lcb[r] * xa[r];
      tv[q] = s;
    }
    __syncthreads();
    if (tid < 64) {
      if (two && tid < NB) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < NB; ++r) s += lbb[r] * tv[r];
        x[NB * cb + q] = (NB * cb + q < W.n) ? s : 0.0;
      }
      if (aborted) {
        if (lane == 0) set_status(stall + w, VI_EDEVICE, -1);
      } else {
        // both blocks published by one release
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
          __hip_atomic_store(xf + c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (two) __hip_atomic_store(xf + cb, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace

void chol_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_chol_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * kPanelSlots * NB * NB));
}

void launch_chol(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st) {
  bool small = false;
  for (const WinDev& W : P.win) small = small || W.npad <= kSmallMaxNpad;
  if (small)
    hipLaunchKernelGGL(k_chol_small, dim3(P.n_win), dim3(kSmallThreads), sizeof(double) * kPanelSlots * NB * NB, s, D,
                       w.A, w.Linv, w.x, st);
  if (P.n_tickets > 0) {
    const int grid = std::min(P.n_tickets, kMaxDataflowWG);
    hipLaunchKernelGGL(k_chol_df, dim3(grid), dim3(64), 0, s, D, P.n_tickets, w.A, w.Linv, w.flags, w.sync, st);
    hipLaunchKernelGGL(k_chol_bs, dim3(std::min(P.n_bs, kMaxDataflowWG)), dim3(256), 0, s, D, P.n_tickets, P.n_bs,
                       w.A, w.Linv, w.x, w.flags, w.sync, st);
  }
}

}  // namespace vi
