// Learned warm start: a four-layer 3x3 convolutional network (32 channels)
// over per-keyframe feature maps on a grid of 4 x 4-pixel cells, with a
// per-cell inverse-depth head and a pooled bias head; forward, backward,
// gradient reduction and AdamW.  The paper has no counterpart of this network;
// it proposes the starting inverse depths and biases of a window, and plain
// Gauss-Newton stays the fallback and the arbiter of the result.
//
// Numerics: activations, activation gradients and the MFMA operands are BF16;
// products accumulate in FP32 (MFMA 16x16x32 bf16 -> f32); the master weights,
// the weight gradients and the optimiser state are FP32.
//
// One 256-thread workgroup per image (keyframe).  Every image of a call sits on
// one padded canvas of hq x wq cells (its own grid is dims[img] = (h, w) in
// the top-left corner); cells outside an image's grid are zero in every layer
// and are excluded from pooling and the loss.  Activations live in LDS in
// pixel-major (HWC) layout with a one-cell zero border, so a convolution is an
// implicit GEMM whose A operand (8 consecutive channels of one tap) is one
// 16-byte LDS read:
//   M = canvas cells, N = output channels, K = 9 taps x input channels,
//   k = tap * Cin + ci.
// The MFMA operand layout: lane l supplies A[l%16][8 (l/16) + i] and
// B[8 (l/16) + i][l%16] (i = 0..7); it receives D[4 (l/16) + r][l%16].
#include <algorithm>

#include "vi_internal.h"

namespace vi {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int PS = 40;                         // bf16 per canvas cell (32 channels + pad; 80 B, 16-B aligned)

// parameter offsets (flat FP32, layout [o][ci][ky][kx] for every conv)
__host__ __device__ constexpr int w_off(int l) {     // l = 1..4
  return l == 1 ? 0 : (kWC * kWCin * 9 + kWC) + (l - 2) * (kWC * kWC * 9 + kWC);
}
__host__ __device__ constexpr int b_off(int l) { return w_off(l) + kWC * (l == 1 ? kWCin : kWC) * 9; }
constexpr int kOffWd = w_off(4) + kWC * kWC * 9 + kWC;
constexpr int kOffBd = kOffWd + kWC * 9;
constexpr int kOffWb = kOffBd + 1;
constexpr int kOffBb = kOffWb + 6 * kWC;
static_assert(kOffBb + 6 == kWParams, "parameter layout");

__device__ const float kSB[6] = {0.005f, 0.005f, 0.005f, 0.05f, 0.05f, 0.05f};

struct Canvas {
  int HQ, WQ, hq, wq;
  __device__ __forceinline__ int cell(int y, int x) const { return (y + 1) * (WQ + 2) + (x + 1); }
  __device__ __forceinline__ bool valid(int p) const {
    if (p >= HQ * WQ) return false;
    const int y = p / WQ, x = p % WQ;
    return y < hq && x < wq;
  }
};

__device__ __forceinline__ void zero_canvas(__bf16* c, int ncell) {
  for (int i = threadIdx.x; i < ncell * PS; i += kThreads) c[i] = (__bf16)0.0f;
}

// Weights of a layer into LDS as [n][k] bf16, k = tap * kpad + c (kpad: the
// padded channel count of the K axis), K padded to KP (multiple of 32), row
// stride KP + 8.  transpose: the weights of the input-gradient convolution,
// Wt[ci][tap' * Cout + o] = W[o][ci][8 - tap'].
__device__ void load_weights(__bf16* Wl, const float* W, int cout, int cin, int kpad, int KP, bool transpose) {
  const int rows = transpose ? cin : cout;
  const int rin = transpose ? cout : cin;      // real channels of the K axis
  const int kshift = kpad == 16 ? 4 : 5;       // kpad is 16 or 32
  // eight elements per thread and pass, their global loads in flight together
  constexpr int U = 8;
  const int total = rows * KP;
  for (int e0 = threadIdx.x; e0 < total; e0 += U * kThreads) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads;
      const int n = e / KP, k = e - (e / KP) * KP;
      const int tap = k >> kshift, c = k & (kpad - 1);
      v[u] = 0.0f;
      if (e < total && tap < 9 && c < rin)
        v[u] = transpose ? W[(c * cin + n) * 9 + (8 - tap)] : W[(n * cin + c) * 9 + tap];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads;
      if (e < total) Wl[(e / KP) * (KP + 8) + (e - (e / KP) * KP)] = (__bf16)v[u];
    }
  }
}

// The forward weights of layer l (1..4) as they sit in LDS: [32][KP + 8] bf16
// with KP = 160 for the first layer and 288 after; layers back to back.
__host__ __device__ constexpr int prep_kp(int l) { return l == 1 ? 160 : 288; }
__host__ __device__ constexpr int prep_off(int l) {
  return l == 1 ? 0 : kWC * (prep_kp(1) + 8) + (l - 2) * kWC * (prep_kp(2) + 8);
}

// theta -> the four layers' LDS images, one workgroup per (output row, layer)
__global__ void __launch_bounds__(kThreads) k_wnet_prep(const float* __restrict__ theta, __bf16* __restrict__ wprep) {
  const int l = blockIdx.y + 1, n = blockIdx.x;
  const int cin = l == 1 ? kWCin : kWC, kpad = l == 1 ? kWCinPad : kWC, KP = prep_kp(l);
  const int kshift = kpad == 16 ? 4 : 5;
  const int row = KP + 8;
  const float* W = theta + w_off(l);
  __bf16* out = wprep + prep_off(l) + (size_t)n * row;
  for (int k = threadIdx.x; k < row; k += kThreads) {
    const int tap = k >> kshift, c = k & (kpad - 1);
    float v = 0.0f;
    if (k < KP && tap < 9 && c < cin) v = W[(n * cin + c) * 9 + tap];
    out[k] = (__bf16)v;
  }
}

// out[cell][o] = act(sum_k in[cell + tap][ci] W[o][k] + bias[o]) for the 16 * ntile
// canvas cells; CIN = channels of the input canvas used on the K axis, COUT
// (16 or 32) output channels.  bias may be null; relu applies max(., 0).
template <int CIN, int COUT>
__device__ void conv_layer(const __bf16* in, __bf16* out, const __bf16* Wl, int KP, const float* bias, Canvas cv,
                           bool relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mrow = lane & 15, q = lane >> 4;
  const int npix = cv.HQ * cv.WQ;
  const int ntile = (npix + 15) / 16;
  constexpr int NT = COUT / 16;
  for (int t = wave; t < ntile; t += kWaves) {
    const int p = 16 * t + mrow;
    const int y = p < npix ? p / cv.WQ : 0, x = p < npix ? p % cv.WQ : 0;
    float4_t acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = float4_t{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < KP / 32; ++s) {
      const int k0 = 32 * s + 8 * q;
      const int tap = k0 / CIN, ci0 = k0 % CIN;
      bf16x8_t a;
      if (tap < 9) {
        a = *(const bf16x8_t*)(in + cv.cell(y + tap / 3 - 1, x + tap % 3 - 1) * PS + ci0);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = (__bf16)0.0f;
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8_t b = *(const bf16x8_t*)(Wl + (16 * nt + mrow) * (KP + 8) + k0);
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pp = 16 * t + 4 * q + r;
        const int o = 16 * nt + mrow;
        if (pp >= npix) continue;
        float v = acc[nt][r] + (bias ? bias[o] : 0.0f);
        if (relu) v = fmaxf(v, 0.0f);
        if (!cv.valid(pp)) v = 0.0f;
        out[cv.cell(pp / cv.WQ, pp % cv.WQ) * PS + o] = (__bf16)v;
      }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// forward: features [n][15][HQ][WQ] (FP32) -> dd [n][HQ][WQ], db [n][6]; when
// act is given, the BF16 activations [n][5][HQ*WQ][32] (layer 0 = the input)
// are kept for the backward pass.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_wnet_forward(const float* __restrict__ theta, int HQ, int WQ,
                                                           const int* __restrict__ dims, const float* __restrict__ feat,
                                                           __bf16* __restrict__ act, float* __restrict__ dd,
                                                           float* __restrict__ db, const __bf16* __restrict__ wprep) {
  extern __shared__ char smem[];
  const int img = blockIdx.x;
  const int ncell = (HQ + 2) * (WQ + 2);
  __bf16* cA = (__bf16*)smem;
  __bf16* cB = cA + ncell * PS;
  __bf16* Wl = cB + ncell * PS;                       // [32][296]
  __shared__ float bias[kWC];
  __shared__ float pool[kThreads];
  __shared__ float wd[kWC * 9];                      // depth head, rounded to bf16
  __shared__ float wb[6 * kWC + 6];                  // bias head (Wb, bb)
  const Canvas cv{HQ, WQ, dims[2 * img], dims[2 * img + 1]};
  const int npix = HQ * WQ;
  for (int e = threadIdx.x; e < kWC * 9; e += kThreads) wd[e] = (float)(__bf16)theta[kOffWd + e];
  for (int e = threadIdx.x; e < 6 * kWC + 6; e += kThreads) wb[e] = theta[kOffWb + e];
  {
    // only the border ring of the two canvases needs zeros: every interior
    // cell is written (by the input planes, channels 0..15 of cA, and by each
    // layer) before it is read
    const int W2 = WQ + 2, nb = 2 * W2 + 2 * HQ;
    for (int e = threadIdx.x; e < 2 * nb * PS; e += kThreads) {
      const int cnv = e / (nb * PS), r = e % (nb * PS), b = r / PS, ch = r % PS;
      const int cell = b < W2 ? b : (b < 2 * W2 ? (HQ + 1) * W2 + (b - W2)
                                                 : (1 + (b - 2 * W2) / 2) * W2 + ((b - 2 * W2) & 1) * (WQ + 1));
      (cnv ? cB : cA)[cell * PS + ch] = (__bf16)0.0f;
    }
  }
  __syncthreads();
  const float* f = feat + (size_t)img * kWCin * npix;
  {
    // eight planes per pass, their loads in flight together
    constexpr int U = 8;
    for (int p = threadIdx.x; p < npix; p += kThreads) {
      const bool ok = cv.valid(p);
      const int cell = cv.cell(p / WQ, p % WQ) * PS;
      for (int c0 = 0; c0 < kWCinPad; c0 += U) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = (c0 + u < kWCin && ok) ? f[(size_t)(c0 + u) * npix + p] : 0.0f;
#pragma unroll
        for (int u = 0; u < U; ++u) cA[cell + c0 + u] = (__bf16)v[u];
      }
    }
  }
  __syncthreads();
  auto save = [&](const __bf16* c, int layer, int ch) {
    if (!act) return;
    __bf16* dst = act + ((size_t)img * 5 + layer) * npix * kWC;
    for (int e = threadIdx.x; e < npix * kWC; e += kThreads) {
      const int p = e / kWC, o = e % kWC;
      dst[e] = o < ch ? c[cv.cell(p / WQ, p % WQ) * PS + o] : (__bf16)0.0f;
    }
  };
  save(cA, 0, kWCinPad);
  __bf16* in = cA;
  __bf16* out = cB;
  for (int l = 1; l <= kWLayers; ++l) {
    const int cin = l == 1 ? kWCin : kWC;
    const int KP = l == 1 ? 160 : 288;
    if (wprep) {
      // the prepared LDS image: 16-byte copies, all in flight together
      const uint4* src = (const uint4*)(wprep + prep_off(l));
      uint4* dst = (uint4*)Wl;
      const int n16 = kWC * (KP + 8) / 8;
      for (int e = threadIdx.x; e < n16; e += kThreads) dst[e] = src[e];
    } else {
      load_weights(Wl, theta + w_off(l), kWC, cin, l == 1 ? kWCinPad : kWC, KP, false);
    }
    for (int o = threadIdx.x; o < kWC; o += kThreads) bias[o] = theta[b_off(l) + o];
    __syncthreads();
    if (l == 1) conv_layer<kWCinPad, kWC>(in, out, Wl, KP, bias, cv, true);
    else conv_layer<kWC, kWC>(in, out, Wl, KP, bias, cv, true);
    __syncthreads();
    save(out, l, kWC);
    __bf16* t = in; in = out; out = t;
  }
  // heads on h4 (in): per-cell depth correction and pooled bias correction
  const float bd = theta[kOffBd];
  for (int p = threadIdx.x; p < npix; p += kThreads) {
    const int y = p / WQ, x = p % WQ;
    float v = bd;
    for (int tap = 0; tap < 9; ++tap) {
      const __bf16* h = in + cv.cell(y + tap / 3 - 1, x + tap % 3 - 1) * PS;
#pragma unroll
      for (int c = 0; c < kWC; ++c) v += wd[c * 9 + tap] * (float)h[c];
    }
    dd[(size_t)img * npix + p] = cv.valid(p) ? v : 0.0f;
  }
  // pooled channel means: thread (c, part) sums a slice of the cells
  {
    // cells p = part, part + P, ... with P = kThreads / 32, (y, x) stepped without divisions
    constexpr int P = kThreads / 32;
    const int c = threadIdx.x & 31, part = threadIdx.x >> 5;
    float s = 0.0f;
    int y = part / WQ, x = part % WQ;
    for (int p = part; p < npix; p += P) {
      if (y < cv.hq && x < cv.wq) s += (float)in[cv.cell(y, x) * PS + c];
      x += P;
      while (x >= WQ) { x -= WQ; ++y; }
    }
    pool[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x < kWC) {
    // channel means, summed over the parts in order
    const int c = threadIdx.x;
    float s = 0.0f;
    for (int part = 0; part < kThreads / 32; ++part) s += pool[part * 32 + c];
    wd[c] = s / (float)max(cv.hq * cv.wq, 1);         // the depth head's weights are no longer needed
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    float v = wb[6 * kWC + k];
    for (int c = 0; c < kWC; ++c) v += wb[k * kWC + c] * wd[c];
    db[(size_t)img * 6 + k] = v;
  }
}

// ---------------------------------------------------------------------------
// loss and output gradients (one image per workgroup):
//   L_img = sum_valid ((dd - dd*) / s_d)^2 / nv + sum_6 ((db - db*) / s_b)^2 / n
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_wnet_loss(int n, int HQ, int WQ, const int* __restrict__ dims,
                                                        float nv, const float* __restrict__ dd,
                                                        const float* __restrict__ db, const float* __restrict__ lab_dd,
                                                        const float* __restrict__ lab_db, float* __restrict__ g_dd,
                                                        float* __restrict__ g_db, float* __restrict__ loss) {
  __shared__ float red[kThreads];
  const int img = blockIdx.x;
  const Canvas cv{HQ, WQ, dims[2 * img], dims[2 * img + 1]};
  const int npix = HQ * WQ;
  const float sd2 = kWSd * kWSd;
  float s = 0.0f;
  for (int p = threadIdx.x; p < npix; p += kThreads) {
    const size_t i = (size_t)img * npix + p;
    const float e = cv.valid(p) ? dd[i] - lab_dd[i] : 0.0f;
    s += e * e / sd2 / nv;
    g_dd[i] = 2.0f * e / sd2 / nv;
  }
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    const float e = db[(size_t)img * 6 + k] - lab_db[(size_t)img * 6 + k];
    s += e * e / (kSB[k] * kSB[k]) / (float)n;
    g_db[(size_t)img * 6 + k] = 2.0f * e / (kSB[k] * kSB[k]) / (float)n;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[img] = red[0];
}

// ---------------------------------------------------------------------------
// backward (one image per workgroup): per-image gradient partials [n][P]
// ---------------------------------------------------------------------------
// part[o][ci * 9 + tap] += sum_p g[p][o] h[p + tap][ci] over the canvas cells:
// M = output channels (32), N = tap * CIN + ci, K = cells (MFMA over 32-cell slices).
template <int CIN>
__device__ void weight_grad(const __bf16* g, const __bf16* h, Canvas cv, float* part, int cin_real) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mrow = lane & 15, q = lane >> 4;
  const int npix = cv.HQ * cv.WQ;
  constexpr int NN = 9 * CIN / 16;              // N tiles
  const int ksteps = (npix + 31) / 32;
  for (int tile = wave; tile < 2 * NN; tile += kWaves) {
    const int mt = tile / NN, nt = tile % NN;
    const int o = 16 * mt + mrow;               // A row (as lane supplier)
    const int n = 16 * nt + mrow;               // B column
    const int tap = n / CIN, ci = n % CIN;
    float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ksteps; ++s) {
      bf16x8_t a, b;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = 32 * s + 8 * q + i;
        const bool ok = p < npix;
        const int y = ok ? p / cv.WQ : 0, x = ok ? p % cv.WQ : 0;
        a[i] = ok ? g[cv.cell(y, x) * PS + o] : (__bf16)0.0f;
        b[i] = ok ? h[cv.cell(y + tap / 3 - 1, x + tap % 3 - 1) * PS + ci] : (__bf16)0.0f;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int oo = 16 * mt + 4 * q + r;       // D row
      const int nn = 16 * nt + mrow;            // D column
      const int tp = nn / CIN, cc = nn % CIN;
      if (cc < cin_real) part[(oo * cin_real + cc) * 9 + tp] = acc[r];
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_wnet_backward(const float* __restrict__ theta, int HQ, int WQ,
                                                            const int* __restrict__ dims,
                                                            const __bf16* __restrict__ act,
                                                            const float* __restrict__ g_dd,
                                                            const float* __restrict__ g_db,
                                                            float* __restrict__ partial) {
  extern __shared__ char smem[];
  const int img = blockIdx.x;
  const int ncell = (HQ + 2) * (WQ + 2);
  __bf16* cH = (__bf16*)smem;                   // activation h_l / h_{l-1}
  __bf16* cG = cH + ncell * PS;                 // gradient at the layer output
  __bf16* cX = cG + ncell * PS;                 // gradient at the layer input
  __bf16* Wl = cX + ncell * PS;                 // [32][296]
  __shared__ float pooled[kWC];
  __shared__ float gpool[kWC];
  __shared__ float red[kThreads];
  const Canvas cv{HQ, WQ, dims[2 * img], dims[2 * img + 1]};
  const int npix = HQ * WQ;
  float* part = partial + (size_t)img * kWParams;
  const float cnt = (float)max(cv.hq * cv.wq, 1);
  zero_canvas(cH, ncell);
  zero_canvas(cG, ncell);
  zero_canvas(cX, ncell);
  __syncthreads();
  auto load_act = [&](int layer) {
    const __bf16* src = act + ((size_t)img * 5 + layer) * npix * kWC;
    for (int e = threadIdx.x; e < npix * kWC; e += kThreads) {
      const int p = e / kWC, o = e % kWC;
      cH[cv.cell(p / WQ, p % WQ) * PS + o] = src[e];
    }
  };
  load_act(4);
  __syncthreads();
  // bias head: pooled h4, gWb, gbb, and the pooled gradient Wb^T g_db / cnt
  if (threadIdx.x < kWC) {
    const int c = threadIdx.x;
    float s = 0.0f;
    for (int p = 0; p < npix; ++p)
      if (cv.valid(p)) s += (float)cH[cv.cell(p / WQ, p % WQ) * PS + c];
    pooled[c] = s / cnt;
    float g = 0.0f;
    for (int k = 0; k < 6; ++k) g += theta[kOffWb + k * kWC + c] * g_db[(size_t)img * 6 + k];
    gpool[c] = g / cnt;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 6 * kWC; e += kThreads)
    part[kOffWb + e] = g_db[(size_t)img * 6 + e / kWC] * pooled[e % kWC];
  if (threadIdx.x < 6) part[kOffBb + threadIdx.x] = g_db[(size_t)img * 6 + threadIdx.x];
  // depth head: gWd[c][tap] = sum_p g_dd[p] h4[p + tap][c], gbd = sum_p g_dd[p]
  const float* gd = g_dd + (size_t)img * npix;
  for (int e = threadIdx.x; e < kWC * 9; e += kThreads) {
    const int c = e / 9, tap = e % 9;
    float s = 0.0f;
    for (int p = 0; p < npix; ++p)
      s += gd[p] * (float)cH[cv.cell(p / WQ + tap / 3 - 1, p % WQ + tap % 3 - 1) * PS + c];
    part[kOffWd + c * 9 + tap] = s;
  }
  {
    float s = 0.0f;
    for (int p = threadIdx.x; p < npix; p += kThreads) s += gd[p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[kOffBd] = red[0];
  }
  // gradient at h4: transpose of the depth head plus the pooled term
  const float* Wd = theta + kOffWd;
  for (int e = threadIdx.x; e < npix * kWC; e += kThreads) {
    const int p = e / kWC, c = e % kWC;
    const int y = p / WQ, x = p % WQ;
    float v = 0.0f;
    if (cv.valid(p)) {
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + 1 - tap / 3, xx = x + 1 - tap % 3;
        if (yy >= 0 && yy < HQ && xx >= 0 && xx < WQ) v += (float)(__bf16)Wd[c * 9 + tap] * gd[yy * WQ + xx];
      }
      v += gpool[c];
    }
    cG[cv.cell(y, x) * PS + c] = (__bf16)v;
  }
  __syncthreads();
  for (int l = kWLayers; l >= 1; --l) {
    // through the ReLU (h_l is in cH) and the mask
    for (int e = threadIdx.x; e < npix * kWC; e += kThreads) {
      const int p = e / kWC, c = e % kWC;
      const int cl = cv.cell(p / WQ, p % WQ) * PS + c;
      if (!((float)cH[cl] > 0.0f) || !cv.valid(p)) cG[cl] = (__bf16)0.0f;
    }
    __syncthreads();
    // bias gradient
    {
      const int c = threadIdx.x & 31, pr = threadIdx.x >> 5;
      float s = 0.0f;
      for (int p = pr; p < npix; p += kThreads / 32) s += (float)cG[cv.cell(p / WQ, p % WQ) * PS + c];
      red[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < kWC) {
      float s = 0.0f;
      for (int pr = 0; pr < kThreads / 32; ++pr) s += red[pr * 32 + threadIdx.x];
      part[b_off(l) + threadIdx.x] = s;
    }
    // h_{l-1} into cH (layer 0: the 16-channel input)
    __syncthreads();
    load_act(l - 1);
    __syncthreads();
    if (l == 1) weight_grad<kWCinPad>(cG, cH, cv, part + w_off(1), kWCin);
    else weight_grad<kWC>(cG, cH, cv, part + w_off(l), kWC);
    if (l > 1) {
      // gradient at the layer input: convolution of g with the flipped,
      // transposed weights, then the mask (ReLU of h_{l-1} applied next round)
      load_weights(Wl, theta + w_off(l), kWC, kWC, kWC, 288, true);
      __syncthreads();
      conv_layer<kWC, kWC>(cG, cX, Wl, 288, nullptr, cv, false);
      __syncthreads();
      __bf16* t = cG; cG = cX; cX = t;
    }
    __syncthreads();
  }
}

// grads[k] = sum over images of partial[img][k], in image order
__global__ void k_wnet_reduce(int n, const float* __restrict__ partial, float* __restrict__ grads) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kWParams) return;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int i = 0;
  for (; i + 8 <= n; i += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += partial[(size_t)(i + u) * kWParams + k];
  }
  for (; i < n; ++i) acc[0] += partial[(size_t)i * kWParams + k];
  float s = 0.0f;
#pragma unroll
  for (int u = 0; u < 8; ++u) s += acc[u];
  grads[k] = s;
}

__global__ void k_wnet_adamw(int P, float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, float c1, float c2, float lr, float b1, float b2, float eps,
                             float wd) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk / c1, vh = vk / c2;
  theta[k] = theta[k] - lr * (mh / (sqrtf(vh) + eps) + wd * theta[k]);
}

size_t wnet_fwd_lds(int HQ, int WQ) {
  return sizeof(__bf16) * (2 * (size_t)(HQ + 2) * (WQ + 2) * PS + 32 * 296);
}
size_t wnet_bwd_lds(int HQ, int WQ) {
  return sizeof(__bf16) * (3 * (size_t)(HQ + 2) * (WQ + 2) * PS + 32 * 296);
}

void wnet_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_wnet_forward, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)wnet_fwd_lds(kWHQMax, kWWQMax));
  (void)hipFuncSetAttribute((const void*)k_wnet_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)wnet_bwd_lds(kWHQMax, kWWQMax));
}

void launch_wnet_forward(hipStream_t s, int n, int HQ, int WQ, const int* dims, const float* theta, const float* feat,
                         void* act, float* dd, float* db, void* wprep) {
  if (wprep) hipLaunchKernelGGL(k_wnet_prep, dim3(kWC, kWLayers), dim3(kThreads), 0, s, theta, (__bf16*)wprep);
  hipLaunchKernelGGL(k_wnet_forward, dim3(n), dim3(kThreads), wnet_fwd_lds(HQ, WQ), s, theta, HQ, WQ, dims, feat,
                     (__bf16*)act, dd, db, (const __bf16*)wprep);
}

size_t wnet_prep_bytes() { return sizeof(__bf16) * (size_t)prep_off(kWLayers + 1); }

void launch_wnet_backward(hipStream_t s, int n, int HQ, int WQ, const int* dims, const float* theta, const void* act,
                          const float* dd, const float* db, const float* lab_dd, const float* lab_db, float nv,
                          float* g_dd, float* g_db, float* loss, float* partial, float* grads) {
  hipLaunchKernelGGL(k_wnet_loss, dim3(n), dim3(kThreads), 0, s, n, HQ, WQ, dims, nv, dd, db, lab_dd, lab_db, g_dd,
                     g_db, loss);
  hipLaunchKernelGGL(k_wnet_backward, dim3(n), dim3(kThreads), wnet_bwd_lds(HQ, WQ), s, theta, HQ, WQ, dims,
                     (const __bf16*)act, g_dd, g_db, partial);
  hipLaunchKernelGGL(k_wnet_reduce, dim3((kWParams + 255) / 256), dim3(256), 0, s, n, partial, grads);
}

void launch_wnet_adamw(hipStream_t s, int P, float* theta, const float* g, float* m, float* v, int t, float lr,
                       float b1, float b2, float eps, float wd) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_wnet_adamw, dim3((P + 255) / 256), dim3(256), 0, s, P, theta, g, m, v, c1, c2, lr, b1, b2, eps,
                     wd);
}

}  // namespace vi
