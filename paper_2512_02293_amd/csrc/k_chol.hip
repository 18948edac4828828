// FP64 Cholesky solve of the reduced pose/velocity/bias system of Eq. 4.
//
// The matrix buffer holds S (npad x npad, row-major, lower triangle used) with
// the right-hand side stored as row npad, so the blocked factorisation carries
// the forward substitution along: at the end row npad holds y = L^-1 s.
//
// Every window of a batch has its own system (blockIdx.y = window); windows
// with fewer block columns than the step index simply exit.
//
// Right-looking, 64-wide block columns, ONE launch per block column kb:
//   * panel workgroups (block rows r = kb .. nblk, nblk being the right-hand-
//     side block) first apply the pending update of block column kb-1 to the
//     diagonal tile and to their own tile, then factor the 64x64 diagonal tile
//     (one wave, one row per lane, in registers), invert it (one wave, one
//     column per lane), and form L_r,kb = S_r,kb L_kb,kb^-T;
//   * trailing workgroups apply the update of block column kb-1 to every tile
//     (i, j) with j > kb, which later steps consume.
// A single-workgroup pass then back-substitutes x = L^-T y block by block with
// the stored inverses of the diagonal tiles (staged through LDS).
#include <algorithm>

#include "vi_internal.h"

namespace vi {

namespace {

constexpr int NB = kCholNB;       // 64
constexpr int LD = NB + 1;        // padded LDS row

__device__ __forceinline__ void set_status(DevStatus* st, int code, int detail) {
  if (atomicCAS(&st->code, 0, code) == 0) st->detail = detail;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_readlane(lo, l);
  hi = __builtin_amdgcn_readlane(hi, l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void load_tile(double* dst, const double* A, int npad, int r0, int c0) {
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx % NB;
    dst[r * LD + c] = A[(size_t)(r0 + r) * npad + c0 + c];
  }
}

// C[r][c] -= sum_m P[r][m] Q[c][m] for the 64x64 tile C (all in LDS).
__device__ __forceinline__ void tile_sub_abt(double* Cm, const double* P, const double* Q) {
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx % NB;
    double v0 = 0.0, v1 = 0.0;
#pragma unroll 8
    for (int m = 0; m < NB; m += 2) {
      v0 += P[r * LD + m] * Q[c * LD + m];
      v1 += P[r * LD + m + 1] * Q[c * LD + m + 1];
    }
    Cm[r * LD + c] -= v0 + v1;
  }
}

__global__ void __launch_bounds__(256) k_chol_step(DevPlan D, int kb, double* __restrict__ Aall,
                                                   double* __restrict__ Linvall, DevStatus* stall) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const WinDev& W = D.win[blockIdx.y];
  const int n = W.n, npad = W.npad, nblk = W.nblk;
  if (kb >= nblk) return;
  const int n_panel = nblk - kb + 1;
  int n_trail = 0;
  if (kb > 0)
    for (int jb = kb + 1; jb < nblk; ++jb) n_trail += nblk - jb + 1;
  if ((int)blockIdx.x >= n_panel + n_trail) return;
  double* A = Aall + W.A_off;
  double* Linv = Linvall + W.Linv_off;
  DevStatus* st = stall + blockIdx.y;
  const int k0 = kb * NB;
  if ((int)blockIdx.x >= n_panel) {
    // trailing tile (i, j), kb < j <= nblk - 1, j <= i <= nblk: apply block column kb-1
    int t = blockIdx.x - n_panel;
    int jb = kb + 1;
    while (true) {
      const int cnt = nblk - jb + 1;
      if (t < cnt) break;
      t -= cnt;
      ++jb;
    }
    const int ib = jb + t;
    double* Pa = sm;
    double* Pb = sm + NB * LD;
    load_tile(Pa, A, npad, ib * NB, k0 - NB);
    load_tile(Pb, A, npad, jb * NB, k0 - NB);
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 256) {
      const int r = idx / NB, c = idx % NB;
      double v0 = 0.0, v1 = 0.0;
#pragma unroll 8
      for (int m = 0; m < NB; m += 2) {
        v0 += Pa[r * LD + m] * Pb[c * LD + m];
        v1 += Pa[r * LD + m + 1] * Pb[c * LD + m + 1];
      }
      A[(size_t)(ib * NB + r) * npad + jb * NB + c] -= v0 + v1;
    }
    return;
  }
  // panel workgroup for block row r
  const int r0 = (kb + blockIdx.x) * NB;
  double* Dg = sm;                 // diagonal tile -> L_kk
  double* Lk = sm + NB * LD;       // L_kb,kb-1, later L_kk^-1
  double* X = sm + 2 * NB * LD;    // own tile
  double* Lr = sm + 3 * NB * LD;   // L_r,kb-1
  load_tile(Dg, A, npad, k0, k0);
  load_tile(X, A, npad, r0, k0);
  if (kb > 0) {
    load_tile(Lk, A, npad, k0, k0 - NB);
    load_tile(Lr, A, npad, r0, k0 - NB);
  }
  __syncthreads();
  if (kb > 0) {
    tile_sub_abt(Dg, Lk, Lk);
    if (blockIdx.x != 0) tile_sub_abt(X, Lr, Lk);
    __syncthreads();
  }
  // factor the diagonal tile: lane i holds row i
  if (wave == 0) {
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = Dg[lane * LD + c];
    int bad = -1;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double piv = readlane_d(a[j], j);
      if (!(piv > 0.0)) {
        if (bad < 0) bad = j;
        piv = 1.0;
      }
      const double dj = sqrt(piv);
      const double inv = 1.0 / dj;
      a[j] = (lane == j) ? dj : a[j] * inv;
#pragma unroll
      for (int m = j + 1; m < NB; ++m) a[m] -= a[j] * readlane_d(a[j], m);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) Dg[lane * LD + c] = (c <= lane) ? a[c] : 0.0;
    if (bad >= 0 && lane == 0 && blockIdx.x == 0 && k0 + bad < n) set_status(st, VI_ENOTPD, k0 + bad);
  }
  __syncthreads();
  // inverse of the diagonal factor: lane c of wave 0 owns column c
  if (wave == 0) {
    double x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) x[r] = (r == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      x[m] = x[m] / Dg[m * LD + m];
#pragma unroll
      for (int r = m + 1; r < NB; ++r) x[r] -= Dg[r * LD + m] * x[m];
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) Lk[r * LD + lane] = x[r];
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int idx = tid; idx < NB * NB; idx += 256) {
      const int r = idx / NB, c = idx % NB;
      A[(size_t)(k0 + r) * npad + k0 + c] = Dg[r * LD + c];
      Linv[(size_t)kb * NB * NB + idx] = Lk[r * LD + c];
    }
    return;
  }
  // L_r,kb = X L^-T: out[r][c] = sum_{m <= c} X[r][m] Linv[c][m]
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx / NB, c = idx % NB;
    double v0 = 0.0, v1 = 0.0;
    int m = 0;
    for (; m + 1 <= c; m += 2) {
      v0 += X[r * LD + m] * Lk[c * LD + m];
      v1 += X[r * LD + m + 1] * Lk[c * LD + m + 1];
    }
    if (m <= c) v0 += X[r * LD + m] * Lk[c * LD + m];
    A[(size_t)(r0 + r) * npad + k0 + c] = v0 + v1;
  }
}

// x = L^-T y, block by block from the last; 1024 threads.
__global__ void __launch_bounds__(1024) k_chol_solve(DevPlan D, const double* __restrict__ Aall,
                                                     const double* __restrict__ Linvall, double* __restrict__ xall) {
  extern __shared__ double xs[];        // [npad]
  __shared__ double part[16][NB];
  __shared__ double tv[NB];
  __shared__ double Li[NB][LD];
  const int tid = threadIdx.x;
  const WinDev& W = D.win[blockIdx.x];
  const int n = W.n, npad = W.npad, nblk = W.nblk;
  const double* A = Aall + W.A_off;
  const double* Linv = Linvall + W.Linv_off;
  double* x = xall + W.x_off;
  const double* y = A + (size_t)npad * npad;
  const int j = tid & (NB - 1), sl = tid >> 6;   // 64 columns x 16 row slices
  for (int b = nblk - 1; b >= 0; --b) {
    for (int idx = tid; idx < NB * NB; idx += 1024) Li[idx / NB][idx % NB] = Linv[(size_t)b * NB * NB + idx];
    double a0 = 0.0, a1 = 0.0;
    int r = (b + 1) * NB + sl;
    for (; r + 16 < npad; r += 32) {
      a0 += A[(size_t)r * npad + b * NB + j] * xs[r];
      a1 += A[(size_t)(r + 16) * npad + b * NB + j] * xs[r + 16];
    }
    if (r < npad) a0 += A[(size_t)r * npad + b * NB + j] * xs[r];
    part[sl][j] = a0 + a1;
    __syncthreads();
    if (tid < NB) {
      double v = y[b * NB + tid];
#pragma unroll
      for (int s = 0; s < 16; ++s) v -= part[s][tid];
      tv[tid] = v;
    }
    __syncthreads();
    if (tid < NB) {
      double v = 0.0;
      for (int m = tid; m < NB; ++m) v += Li[m][tid] * tv[m];
      xs[b * NB + tid] = v;
    }
    __syncthreads();
  }
  for (int i = tid; i < npad; i += 1024) x[i] = (i < n) ? xs[i] : 0.0;
}

size_t step_lds() { return sizeof(double) * 4 * NB * LD; }

}  // namespace

void chol_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_chol_step, hipFuncAttributeMaxDynamicSharedMemorySize, (int)step_lds());
}

void launch_chol(hipStream_t s, const Plan& P, const DevPlan& D, const Work& w, DevStatus* st) {
  int npad_max = 0;
  for (const WinDev& W : P.win) npad_max = std::max(npad_max, W.npad);
  for (int kb = 0; kb < P.nblk_max; ++kb) {
    int wgs = 0;
    for (const WinDev& W : P.win) {
      if (kb >= W.nblk) continue;
      int cnt = W.nblk - kb + 1;
      if (kb > 0)
        for (int jb = kb + 1; jb < W.nblk; ++jb) cnt += W.nblk - jb + 1;
      wgs = std::max(wgs, cnt);
    }
    hipLaunchKernelGGL(k_chol_step, dim3(wgs, P.n_win), dim3(256), step_lds(), s, D, kb, w.A, w.Linv, st);
  }
  hipLaunchKernelGGL(k_chol_solve, dim3(P.n_win), dim3(1024), sizeof(double) * npad_max, s, D, w.A, w.Linv, w.x);
}

}  // namespace vi
