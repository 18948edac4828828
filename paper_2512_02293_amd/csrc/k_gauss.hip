// Loop-closure update of a Gaussian map (Sec. 3.3, "Loop Closure Gaussian
// Update", Eq. 7-8).
//
// Every Gaussian anchored to keyframe k is taken into k's old camera frame,
// scaled by ds_k and mapped out of k's new camera frame; its covariance is
// rotated alike and scaled by ds_k^2.  Both steps compose, per keyframe, into
// one similarity x -> A x + b with A = ds R+ (R-)^T and b = t+ - A t-, so that
// Sigma -> A Sigma A^T.  A small FP64 kernel folds the two poses and the scale
// of every keyframe into (A, b) once (rounded to FP32 at the end); the map
// kernel then streams the FP32 means and covariances from HBM once, applying
// the affine map of each Gaussian's keyframe.
//
// The map kernel is HBM-bound (about 108 flops per 76 bytes of algorithmic
// traffic: anchor 4, mean 12 + 12, covariance 24 + 24).  Each thread owns four
// consecutive Gaussians, so that its anchor, means and covariances are whole
// 16-byte vectors (1, 3 and 6 of them), and when the four share a keyframe (the
// usual case: Gaussians are created keyframe by keyframe) its 48-byte table row
// is read once.  Means and covariances pass through LDS so that global memory
// sees only contiguous wave-wide float4 spans, with non-temporal loads and
// stores (the map is streamed once per call).
#include <mutex>

#include "vi_internal.h"
#include "vi_math.h"

namespace vi {

// Keyframe table of the allocation-free entry point: a file-scope device
// array (one copy per GPU, kept until the process ends).  In host code its
// name is only a stand-in: kernels get the device address obtained per device
// by reanchor_scratch_init.  Every call on a GPU shares that GPU's copy, so
// calls that overlap on one GPU race.
constexpr int kReanchorNoAllocMaxKeyframes = 16384;          // 16384 x 48 B = 768 KiB
static __device__ __align__(256) float4 scratch[3 * kReanchorNoAllocMaxKeyframes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

constexpr int kGaussThreads = 256;
constexpr int kGaussPerBlock = 4 * kGaussThreads;

// table row of keyframe k: float4 tab[3k + r] = (A[r][0], A[r][1], A[r][2], b[r]);
// a keyframe whose update is not valid gets NaN rows
__global__ void k_reanchor_prep(int n_kf, const double* __restrict__ pre, const double* __restrict__ post,
                                const double* __restrict__ ds, float4* __restrict__ tab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_kf) return;
  double a[7], b[7];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    a[i] = pre[7 * k + i];
    b[i] = post[7 * k + i];
    ok = ok && isfinite(a[i]) && isfinite(b[i]);
  }
  const double s = ds[k];
  ok = ok && isfinite(s) && s > 0.0;
  ok = ok && (a[3] * a[3] + a[4] * a[4] + a[5] * a[5] + a[6] * a[6]) > 0.0;
  ok = ok && (b[3] * b[3] + b[4] * b[4] + b[5] * b[5] + b[6] * b[6]) > 0.0;
  if (!ok) {
    const float nan = __builtin_nanf("");
    for (int r = 0; r < 3; ++r) tab[3 * k + r] = make_float4(nan, nan, nan, nan);
    return;
  }
  double Rm[9], Rp[9], A[9];
  quat_to_rot(a + 3, Rm);
  quat_to_rot(b + 3, Rp);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      A[3 * r + c] = s * (Rp[3 * r] * Rm[3 * c] + Rp[3 * r + 1] * Rm[3 * c + 1] + Rp[3 * r + 2] * Rm[3 * c + 2]);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double br = b[r] - (A[3 * r] * a[0] + A[3 * r + 1] * a[1] + A[3 * r + 2] * a[2]);
    tab[3 * k + r] = make_float4((float)A[3 * r], (float)A[3 * r + 1], (float)A[3 * r + 2], (float)br);
  }
}

struct Sim {
  float4 r0, r1, r2;
  __device__ __forceinline__ bool valid() const { return r0.w == r0.w; }
};

__device__ __forceinline__ Sim load_sim(const float4* __restrict__ tab, int k) {
  return Sim{tab[3 * k], tab[3 * k + 1], tab[3 * k + 2]};
}

__device__ __forceinline__ void map_mean(const Sim& S, float* m) {
  const float x = m[0], y = m[1], z = m[2];
  m[0] = fmaf(S.r0.x, x, fmaf(S.r0.y, y, fmaf(S.r0.z, z, S.r0.w)));
  m[1] = fmaf(S.r1.x, x, fmaf(S.r1.y, y, fmaf(S.r1.z, z, S.r1.w)));
  m[2] = fmaf(S.r2.x, x, fmaf(S.r2.y, y, fmaf(S.r2.z, z, S.r2.w)));
}

// c = (xx, xy, xz, yy, yz, zz) -> upper triangle of A Sigma A^T
__device__ __forceinline__ void map_cov(const Sim& S, float* c) {
  const float A[3][3] = {{S.r0.x, S.r0.y, S.r0.z}, {S.r1.x, S.r1.y, S.r1.z}, {S.r2.x, S.r2.y, S.r2.z}};
  const float M[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
  float T[3][3];  // A Sigma
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) T[r][q] = fmaf(A[r][0], M[0][q], fmaf(A[r][1], M[1][q], A[r][2] * M[2][q]));
  int e = 0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = r; q < 3; ++q) c[e++] = fmaf(T[r][0], A[q][0], fmaf(T[r][1], A[q][1], T[r][2] * A[q][2]));
}

// the Gaussian is moved when its anchor names a keyframe with a valid update;
// returns 1 when it is left unchanged (rejected)
template <bool kCov>
__device__ __forceinline__ int update_one(int k, int n_kf, const float4* __restrict__ tab, float* m, float* c) {
  if (k < 0 || k >= n_kf) return 1;
  const Sim S = load_sim(tab, k);
  if (!S.valid()) return 1;
  map_mean(S, m);
  if (kCov) map_cov(S, c);
  return 0;
}

// the four Gaussians m[0..11], c[0..23] of a quad with anchors a; returns the
// number left unchanged
template <bool kCov>
__device__ __forceinline__ int update_quad(const int4 a, int n_kf, const float4* __restrict__ tab, float* m,
                                           float* c) {
  if (a.x == a.y && a.x == a.z && a.x == a.w && a.x >= 0 && a.x < n_kf) {
    const Sim S = load_sim(tab, a.x);
    if (!S.valid()) return 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      map_mean(S, m + 3 * j);
      if (kCov) map_cov(S, c + 6 * j);
    }
    return 0;
  }
  return update_one<kCov>(a.x, n_kf, tab, m, c) + update_one<kCov>(a.y, n_kf, tab, m + 3, c + 6) +
         update_one<kCov>(a.z, n_kf, tab, m + 6, c + 12) + update_one<kCov>(a.w, n_kf, tab, m + 9, c + 18);
}

typedef float f4v __attribute__((ext_vector_type(4)));

// streaming 16-byte access that bypasses cache retention (each byte is used once)
__device__ __forceinline__ float4 ld_stream(const float* p) {
  const f4v v = __builtin_nontemporal_load((const f4v*)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_stream(float* p, const float4& v) {
  const f4v w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, (f4v*)p);
}

// A workgroup owns kGaussPerBlock consecutive Gaussians, thread t the quad
// 4t..4t+3.  kVec (every array 16-byte aligned): a full block moves its means
// and covariances between HBM and LDS as consecutive float4s, so that each
// wave-wide access covers one contiguous 1 KiB span, and every thread then
// reads its quad from LDS; the last, partial block and unaligned arrays go
// element by element.
template <bool kVec, bool kCov>
__global__ void __launch_bounds__(kGaussThreads) k_reanchor(int64_t K, int n_kf, const int32_t* __restrict__ anchor,
                                                            const float4* __restrict__ tab,
                                                            const float* mean_in, const float* cov_in,
                                                            float* mean_out, float* cov_out, int* n_rej) {
  constexpr int T = kGaussThreads;
  __shared__ float4 sm[kVec ? 3 * T : 1], sc[kVec && kCov ? 6 * T : 1];
  const int t = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * kGaussPerBlock;
  int bad = 0;
  if (kVec && b0 + kGaussPerBlock <= K) {
    const int4 a = *(const int4*)(anchor + b0 + 4 * t);
#pragma unroll
    for (int i = 0; i < 3; ++i) sm[i * T + t] = ld_stream(mean_in + 3 * b0 + 4 * (i * T + t));
    if (kCov) {
#pragma unroll
      for (int i = 0; i < 6; ++i) sc[i * T + t] = ld_stream(cov_in + 6 * b0 + 4 * (i * T + t));
    }
    __syncthreads();
    float m[12], c[24];
#pragma unroll
    for (int i = 0; i < 3; ++i) *(float4*)(m + 4 * i) = sm[3 * t + i];
    if (kCov) {
#pragma unroll
      for (int i = 0; i < 6; ++i) *(float4*)(c + 4 * i) = sc[6 * t + i];
    }
    bad = update_quad<kCov>(a, n_kf, tab, m, c);
    // each thread rewrites only the LDS slots it read
#pragma unroll
    for (int i = 0; i < 3; ++i) sm[3 * t + i] = *(const float4*)(m + 4 * i);
    if (kCov) {
#pragma unroll
      for (int i = 0; i < 6; ++i) sc[6 * t + i] = *(const float4*)(c + 4 * i);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) st_stream(mean_out + 3 * b0 + 4 * (i * T + t), sm[i * T + t]);
    if (kCov) {
#pragma unroll
      for (int i = 0; i < 6; ++i) st_stream(cov_out + 6 * b0 + 4 * (i * T + t), sc[i * T + t]);
    }
  } else {
    const int64_t g0 = b0 + 4 * t;
    const int64_t g1 = g0 + 4 < K ? g0 + 4 : K;
    for (int64_t g = g0; g < g1; ++g) {
      float m[3], c[6];
      for (int i = 0; i < 3; ++i) m[i] = mean_in[3 * g + i];
      if (kCov)
        for (int i = 0; i < 6; ++i) c[i] = cov_in[6 * g + i];
      bad += update_one<kCov>(anchor[g], n_kf, tab, m, c);
      for (int i = 0; i < 3; ++i) mean_out[3 * g + i] = m[i];
      if (kCov)
        for (int i = 0; i < 6; ++i) cov_out[6 * g + i] = c[i];
    }
  }
  // rejections are rare: the lanes that have any add them
  if (n_rej && bad != 0) atomicAdd(n_rej, bad);
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

template <bool kVec, bool kCov>
void launch_map(hipStream_t s, int64_t blocks, int64_t K, int n_kf, const int32_t* anchor, const float4* tab,
                const float* mi, const float* ci, float* mo, float* co, int* n_rej) {
  hipLaunchKernelGGL((k_reanchor<kVec, kCov>), dim3((unsigned)blocks), dim3(kGaussThreads), 0, s, K, n_kf, anchor,
                     tab, mi, ci, mo, co, n_rej);
}

}  // namespace

size_t reanchor_table_bytes(int n_kf) { return (size_t)n_kf * 3 * sizeof(float4); }

int reanchor_noalloc_max_keyframes() { return kReanchorNoAllocMaxKeyframes; }

hipError_t reanchor_scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* reanchor_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxScratchDevices) ? g_scratch_ptr[device] : nullptr;
}

int64_t reanchor_max_gaussians() { return (int64_t)kGaussPerBlock * 0x7fffffffLL; }

void launch_reanchor(hipStream_t s, int n_kf, const double* pose_pre, const double* pose_post, const double* ds,
                     void* table, int64_t K, const int32_t* anchor, const float* mean_in, const float* cov_in,
                     float* mean_out, float* cov_out, int* n_rej) {
  float4* tab = (float4*)table;
  if (n_rej) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, n_rej);
  hipLaunchKernelGGL(k_reanchor_prep, dim3((n_kf + 127) / 128), dim3(128), 0, s, n_kf, pose_pre, pose_post, ds, tab);
  if (K == 0) return;
  const int64_t blocks = (K + kGaussPerBlock - 1) / kGaussPerBlock;
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const bool cov = cov_in != nullptr;
  const bool vec = al(anchor) && al(mean_in) && al(mean_out) && (!cov || (al(cov_in) && al(cov_out)));
  if (vec && cov) launch_map<true, true>(s, blocks, K, n_kf, anchor, tab, mean_in, cov_in, mean_out, cov_out, n_rej);
  if (vec && !cov) launch_map<true, false>(s, blocks, K, n_kf, anchor, tab, mean_in, cov_in, mean_out, cov_out, n_rej);
  if (!vec && cov) launch_map<false, true>(s, blocks, K, n_kf, anchor, tab, mean_in, cov_in, mean_out, cov_out, n_rej);
  if (!vec && !cov) launch_map<false, false>(s, blocks, K, n_kf, anchor, tab, mean_in, cov_in, mean_out, cov_out, n_rej);
}

}  // namespace vi
