// C ABI of the visual-inertial step library: argument validation, the
// per-batch plan (index tables derived from the windows' frame graphs), the
// workspace carve, the autotuner of the fused assembly tiling, HIP-graph
// capture of whole solves, and the reports.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "vi_internal.h"

using namespace vi;

namespace {

// candidate pixels-per-workgroup of the fused assembly (multiples of 64)
const int kRanges[] = {128, 192, 256, 320, 384, 448, 512, 640, 1024, 1536, 2048, 3072, 4096, 8192};
constexpr int kRangeMin = 128;
constexpr int kAssemblyWGTarget = 256;   // default tiling: about one assembly workgroup per compute unit

struct WinIn {
  const vi_camera* cam;
  const vi_state* st;
  const vi_edges* ed;
  const vi_preint* imu;
  vi_report* rep;
  double* scale = nullptr;                // pose-graph adjustment: keyframe scales
  const vi_rel_poses* rel = nullptr;      // pose-graph adjustment: relative-pose factors (marks the mode)
};

}  // namespace

struct vi_ctx {
  int device = 0;
  hipStream_t user = nullptr;      // caller's stream
  hipStream_t priv = nullptr;      // private stream (graph capture and execution)
  hipEvent_t ev_in = nullptr;
  std::string err;
  DevStatus* status = nullptr;     // device [status_cap]
  int status_cap = 0;
  int32_t* d_off = nullptr;        // device CSR for imu_preintegrate
  size_t d_off_cap = 0;
  std::vector<int32_t> off_on_dev; // what d_off holds (empty: not known), so an unchanged CSR is not sent again
  // plan
  Plan plan;
  bool have_plan = false;
  uint64_t plan_version = 0;
  std::vector<int32_t> plan_sig;   // shape signature of the planned batch
  char* d_plan = nullptr;
  size_t d_plan_cap = 0;
  DevPlan dplan{};
  WinDev* d_win = nullptr;         // device window table (inside d_plan)
  std::vector<char> win_on_dev;    // bytes d_win holds (empty: not known), so an unchanged table is not sent again
  int attr_kmax = -1;
  // autotuning
  bool autotune = false;
  double tol = 0.0;                // tolerance stop of the solves (0: off)
  std::map<std::tuple<int, int, int, int>, int> tuned;
  // graph cache
  bool have_graph = false;
  std::vector<uint64_t> gkey;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

vi_status fail(vi_ctx* ctx, vi_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, VI_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Host checks of one window.  `full` also requires the device arrays (a
// workspace-size query only needs the shapes and the frame graph).
vi_status check_window(vi_ctx* ctx, int w, const WinIn& in, const vi_opts* o, bool full) {
  const vi_camera* cam = in.cam;
  const vi_state* st = in.st;
  const vi_edges* ed = in.ed;
  if (!cam || !st || !ed) return fail(ctx, VI_EINVAL, "window %d: null argument", w);
  if (!finite_pos(cam->fx) || !finite_pos(cam->fy) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(ctx, VI_EINVAL, "window %d: intrinsics must be finite with fx, fy > 0", w);
  if (cam->H <= 0 || cam->W <= 0 || (int64_t)cam->H * cam->W > (1 << 24))
    return fail(ctx, VI_EINVAL, "window %d: bad map size %d x %d", w, cam->H, cam->W);
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(cam->gravity[k])) return fail(ctx, VI_EINVAL, "window %d: gravity must be finite", w);
  for (int k = 0; k < 7; ++k)
    if (!std::isfinite(cam->T_bc[k])) return fail(ctx, VI_EINVAL, "window %d: T_bc must be finite", w);
  if (st->n_kf < 2) return fail(ctx, VI_EINVAL, "window %d: need at least 2 keyframes (got %d)", w, st->n_kf);
  if (st->n_kf > kMaxKeyframes)
    return fail(ctx, VI_EUNSUPPORTED, "window %d: at most %d keyframes are supported (dense reduced system)", w,
                kMaxKeyframes);
  if (ed->n_edges < 1) return fail(ctx, VI_EINVAL, "window %d: need at least one edge", w);
  if (!ed->ii || !ed->jj) return fail(ctx, VI_EINVAL, "window %d: null edge index array", w);
  if (o->n_fixed > st->n_kf) return fail(ctx, VI_EINVAL, "window %d: n_fixed out of range", w);
  if (full) {
    if (!st->pose || !st->vel || !st->bias || !st->invdepth)
      return fail(ctx, VI_EINVAL, "window %d: null state array", w);
    if (!ed->target || !ed->weight) return fail(ctx, VI_EINVAL, "window %d: null edge array", w);
    if (o->use_imu && !in.imu) return fail(ctx, VI_EINVAL, "window %d: use_imu set but no IMU factors given", w);
  }
  return VI_OK;
}

vi_status check_opts(vi_ctx* ctx, const vi_opts* o) {
  if (!o) return fail(ctx, VI_EINVAL, "null options");
  if (o->n_fixed < 0) return fail(ctx, VI_EINVAL, "n_fixed out of range");
  if (o->precision != VI_PREC_FP64 && o->precision != VI_PREC_MIXED)
    return fail(ctx, VI_EINVAL, "opts.precision must be VI_PREC_FP64 or VI_PREC_MIXED");
  if (!(o->lm_lambda >= 0.0) || !(o->depth_eta >= 0.0) || !std::isfinite(o->lm_lambda) ||
      !std::isfinite(o->depth_eta))
    return fail(ctx, VI_EINVAL, "damping must be finite and >= 0");
  if (!std::isfinite(o->z_min) || !(o->d_min >= 0.0) || !std::isfinite(o->d_min))
    return fail(ctx, VI_EINVAL, "z_min must be finite and d_min finite and >= 0");
  if (o->bias_mode != VI_BIAS_PER_KF && o->bias_mode != VI_BIAS_FIXED && o->bias_mode != VI_BIAS_GLOBAL)
    return fail(ctx, VI_EINVAL, "opts.bias_mode must be VI_BIAS_PER_KF, VI_BIAS_FIXED or VI_BIAS_GLOBAL");
  if (o->invdepth_f32 != 0 && o->invdepth_f32 != 1) return fail(ctx, VI_EINVAL, "opts.invdepth_f32 must be 0 or 1");
  if (o->invdepth_f32 && o->precision != VI_PREC_MIXED)
    return fail(ctx, VI_EINVAL, "float32 inverse depths (opts.invdepth_f32) need VI_PREC_MIXED");
  if (o->reserved != 0) return fail(ctx, VI_EINVAL, "opts.reserved must be 0");
  return VI_OK;
}

// Shape signature: everything the plan depends on (sizes and the frame graphs).
std::vector<int32_t> plan_signature(const std::vector<WinIn>& wins, bool bias_global) {
  std::vector<int32_t> s;
  s.push_back((int32_t)wins.size());
  s.push_back(bias_global ? 1 : 0);
  for (const WinIn& in : wins) {
    s.push_back(in.st->n_kf);
    s.push_back(in.cam->H);
    s.push_back(in.cam->W);
    s.push_back(in.ed->n_edges);
    s.insert(s.end(), in.ed->ii, in.ed->ii + in.ed->n_edges);
    s.insert(s.end(), in.ed->jj, in.ed->jj + in.ed->n_edges);
    if (in.rel) {
      s.push_back(-7);     // pose-graph mode marker
      s.push_back(in.rel->n_rel);
      s.insert(s.end(), in.rel->ii, in.rel->ii + in.rel->n_rel);
      s.insert(s.end(), in.rel->jj, in.rel->jj + in.rel->n_rel);
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Order of the keyframes in a window's reduced system, and the envelope of S.
// The Cholesky factor of S is nonzero only inside the envelope of S (in each
// row, from the first nonzero column to the diagonal), so the tile dataflow
// only visits tiles (i, j) with fc[i] <= j, and inside a tile only the
// k >= max(fc[i], fc[j]).  Loop edges widen the envelope far beyond the band
// of nearby keyframes; a reverse Cuthill-McKee order of the keyframe coupling
// graph (breadth-first from a pseudo-peripheral keyframe, neighbours by
// increasing degree, the whole sequence reversed) narrows it again.  The
// order is taken only when it lowers the factorisation's work.
// ---------------------------------------------------------------------------
struct Coupling {
  int a, b;
  bool full;   // all unknowns of both keyframes coupled (else only the 6 pose unknowns at the head of each block)
};

std::vector<int> rcm_order(int N, const std::vector<std::vector<int>>& adj) {
  std::vector<int> deg(N), order, dist(N, -1), comp;
  for (int v = 0; v < N; ++v) deg[v] = (int)adj[v].size();
  std::vector<char> done(N, 0);
  order.reserve(N);
  auto by_degree = [&](int x, int y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; };
  // breadth-first levels from r over the component; returns the eccentricity and the last level
  auto levels = [&](int r, std::vector<int>& last) {
    for (int v : comp) dist[v] = -1;
    std::vector<int> q{r};
    dist[r] = 0;
    for (size_t h = 0; h < q.size(); ++h)
      for (int u : adj[q[h]])
        if (dist[u] < 0) {
          dist[u] = dist[q[h]] + 1;
          q.push_back(u);
        }
    const int ecc = dist[q.back()];
    last.clear();
    for (int v : q)
      if (dist[v] == ecc) last.push_back(v);
    return ecc;
  };
  for (int s0 = 0; s0 < N; ++s0) {
    if (done[s0]) continue;
    // the component of s0
    comp.assign(1, s0);
    dist[s0] = 0;
    for (size_t h = 0; h < comp.size(); ++h)
      for (int u : adj[comp[h]])
        if (dist[u] < 0) {
          dist[u] = 0;
          comp.push_back(u);
        }
    int root = *std::min_element(comp.begin(), comp.end(), by_degree);
    std::vector<int> last, last2;
    int ecc = levels(root, last);
    for (int guard = 0; guard < N; ++guard) {
      const int v = *std::min_element(last.begin(), last.end(), by_degree);
      const int e2 = levels(v, last2);
      if (e2 <= ecc) break;
      root = v;
      ecc = e2;
      last.swap(last2);
    }
    // Cuthill-McKee sequence of the component
    const size_t base = order.size();
    order.push_back(root);
    done[root] = 1;
    std::vector<int> nb;
    for (size_t h = base; h < order.size(); ++h) {
      nb.clear();
      for (int u : adj[order[h]])
        if (!done[u]) nb.push_back(u);
      std::sort(nb.begin(), nb.end(), by_degree);
      for (int u : nb) {
        done[u] = 1;
        order.push_back(u);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// first nonzero scalar column of each scalar row of S (lower triangle) with
// keyframe a at block position pos[a]
void scalar_envelope(int N, int PD, const std::vector<Coupling>& cpl, const std::vector<int>& pos,
                     std::vector<int>& fcs) {
  fcs.assign((size_t)N * PD, 0);
  for (int a = 0; a < N; ++a)
    for (int r = 0; r < PD; ++r) fcs[(size_t)pos[a] * PD + r] = pos[a] * PD;
  for (const Coupling& c : cpl) {
    int qa = pos[c.a], qb = pos[c.b];
    if (qa == qb) continue;
    if (qa < qb) std::swap(qa, qb);
    const int rows = c.full ? PD : 6;
    for (int r = 0; r < rows; ++r) fcs[(size_t)qa * PD + r] = std::min(fcs[(size_t)qa * PD + r], qb * PD);
  }
}

// tile envelope (nblk + 1 entries, the last one the right-hand-side row), the
// tile-update count of the dataflow factorisation over it and the tile band
struct Envelope {
  std::vector<int> fc;
  long long work = 0;
  int band = 0;
};

Envelope tile_envelope(const std::vector<int>& fcs, int n, int nblk) {
  Envelope E;
  E.fc.assign(nblk + 1, 0);
  int wsc = 0;
  for (int i = 0; i < nblk; ++i) {
    int f = i;
    for (int r = i * kCholNB; r < std::min(n, (i + 1) * kCholNB); ++r) {
      f = std::min(f, fcs[r] / kCholNB);
      wsc = std::max(wsc, r - fcs[r]);
    }
    E.fc[i] = f;
  }
  E.fc[nblk] = 0;
  for (int i = 0; i <= nblk; ++i)
    for (int j = E.fc[i]; j <= std::min(i, nblk - 1); ++j) E.work += 1 + (j - std::max(E.fc[i], E.fc[j]));
  E.band = std::min(nblk - 1, (wsc + kCholNB - 1) / kCholNB);
  return E;
}

vi_status build_plan(vi_ctx* ctx, const std::vector<WinIn>& wins, Plan& P, bool bias_global = false) {
  P = Plan();
  const int nw = (int)wins.size();
  // pose-graph adjustment (one window): 7 unknowns per keyframe, 7x7 blocks,
  // relative-pose factors instead of inertial ones
  const bool pg = nw > 0 && wins[0].rel != nullptr;
  const int PD = pg ? 7 : 15, ZD = pg ? 49 : 36, ZBD = pg ? 7 : 6;
  P.pdim = PD;
  P.n_win = nw;
  P.win.resize(nw);
  int kf = 0, ed = 0, fa = 0;
  long long pix = 0;
  for (int w = 0; w < nw; ++w) {
    const WinIn& in = wins[w];
    WinDev& W = P.win[w];
    std::memset(&W, 0, sizeof(W));
    W.H = in.cam->H;
    W.W = in.cam->W;
    W.HW = W.H * W.W;
    W.N = in.st->n_kf;
    W.kf_base = kf;
    W.e_base = ed;
    W.f_base = fa;
    W.F = pg ? 0 : W.N - 1;
    W.pix_base = pix;
    const int E = in.ed->n_edges;
    for (int e = 0; e < E; ++e) {
      const int i = in.ed->ii[e], j = in.ed->jj[e];
      if (i < 0 || i >= W.N || j < 0 || j >= W.N)
        return fail(ctx, VI_EINVAL, "window %d edge %d: keyframe index out of range (%d -> %d, N = %d)", w, e, i, j,
                    W.N);
      if (i == j) return fail(ctx, VI_EINVAL, "window %d edge %d: source equals target (%d)", w, e, i);
      P.ii.push_back(kf + i);
      P.jj.push_back(kf + j);
    }
    for (int l = 0; l < W.N; ++l) P.win_of_kf.push_back(w);
    for (int l = 0; l < W.F; ++l) P.win_of_f.push_back(w);
    kf += W.N;
    ed += E;
    fa += W.F;
    pix += (long long)W.N * W.HW;
    P.hw_max = std::max(P.hw_max, W.HW);
  }
  P.N = kf;
  P.kf_pos.assign(P.N, 0);
  P.kf_at.assign(P.N, 0);
  P.E = ed;
  P.F = fa;
  P.pix_total = pix;
  // edges grouped by source keyframe (input order within a source)
  std::vector<int> cnt(P.N, 0);
  for (int e = 0; e < P.E; ++e) cnt[P.ii[e]]++;
  P.src_off.assign(P.N + 1, 0);
  for (int g = 0; g < P.N; ++g) P.src_off[g + 1] = P.src_off[g] + cnt[g];
  P.src_edges.assign(P.E, 0);
  std::vector<int> fill(P.N, 0);
  for (int e = 0; e < P.E; ++e) {
    const int g = P.ii[e];
    P.src_edges[P.src_off[g] + fill[g]++] = e;
  }
  P.kmax = 0;
  for (int g = 0; g < P.N; ++g) P.kmax = std::max(P.kmax, cnt[g]);
  if (P.kmax > kMaxOutDegree)
    return fail(ctx, VI_EUNSUPPORTED, "a keyframe has %d outgoing edges; at most %d are supported", P.kmax,
                kMaxOutDegree);
  for (int g = 0; g < P.N; ++g) {
    std::vector<int> t;
    for (int s = P.src_off[g]; s < P.src_off[g + 1]; ++s) t.push_back(P.jj[P.src_edges[s]]);
    std::sort(t.begin(), t.end());
    const WinDev& W = P.win[P.win_of_kf[g]];
    for (size_t a = 1; a < t.size(); ++a)
      if (t[a] == t[a - 1])
        return fail(ctx, VI_EINVAL, "window %d: duplicate edge %d -> %d", P.win_of_kf[g], g - W.kf_base,
                    t[a] - W.kf_base);
  }
  // partial-sum layout for the smallest tiling, so any candidate fits
  P.nkr_max = (P.hw_max + kRangeMin - 1) / kRangeMin;
  P.gram_off.assign(P.N, 0);
  P.z_off.assign(P.N, 0);
  P.zb_off.assign(P.N, 0);
  size_t go = 0, zo = 0, zbo = 0;
  for (int g = 0; g < P.N; ++g) {
    const int k = cnt[g];
    const WinDev& W = P.win[P.win_of_kf[g]];
    // the fused assembly writes the tiles of (6 k + 1) columns for every
    // source, one tile (the right-hand-side column alone) when k = 0
    const int T = (6 * k + 16) / 16;
    P.gram_off[g] = (int32_t)go;
    P.z_off[g] = (int32_t)zo;
    P.zb_off[g] = (int32_t)zbo;
    go += (size_t)T * (T + 1) / 2 * 256 * ((W.HW + kRangeMin - 1) / kRangeMin);
    zo += (size_t)(k + 1) * (k + 1) * ZD;
    zbo += (size_t)ZBD * (k + 1);
  }
  if (pg) {
    // relative-pose factors: four 7x7 blocks ((i,i), (i,j), (j,i), (j,j)) and 14 diagonal / right-hand-side entries
    const vi_rel_poses* rel = wins[0].rel;
    P.R = rel->n_rel;
    for (int f = 0; f < P.R; ++f) {
      const int i = rel->ii[f], j = rel->jj[f];
      if (i < 0 || i >= P.win[0].N || j < 0 || j >= P.win[0].N || i == j)
        return fail(ctx, VI_EINVAL, "relative pose %d: bad keyframe pair (%d, %d)", f, i, j);
      P.rel_ii.push_back(i);
      P.rel_jj.push_back(j);
      P.rel_z.push_back((int32_t)zo);
      P.rel_zb.push_back((int32_t)zbo);
      zo += 4 * 49;
      zbo += 14;
    }
    P.win[0].rel_base = 0;
    P.win[0].n_rel = P.R;
  }
  if (go > INT32_MAX || zo > INT32_MAX) return fail(ctx, VI_EUNSUPPORTED, "batch too large for 32-bit offsets");
  P.gram_size = go;
  P.z_size = zo;
  P.zb_size = zbo;
  // per window: reduced system and gather lists of its assembly.  Pose block
  // (a, b) <- Z blocks of every source whose touched set contains a and b.
  size_t A_off = 0, L_off = 0, x_off = 0;
  for (int w = 0; w < nw; ++w) {
    WinDev& W = P.win[w];
    W.n = PD * W.N;
    W.npad = (W.n + kCholNB - 1) / kCholNB * kCholNB;
    W.nblk = W.npad / kCholNB;
    W.A_off = (long long)A_off;
    W.Linv_off = (long long)L_off;
    W.x_off = (long long)x_off;
    W.flag_off = (int)P.flags_size;
    W.nflags = (W.nblk + 2) * W.nblk;   // tile flags, then the back-substitution's x_b flags
    P.flags_size += (size_t)W.nflags;
    A_off += (size_t)(W.npad + kCholNB) * W.npad;
    L_off += (size_t)W.nblk * kCholNB * kCholNB;
    x_off += (size_t)W.npad;
    P.nblk_max = std::max(P.nblk_max, W.nblk);
    std::vector<std::vector<std::pair<int, int>>> items((size_t)W.N * W.N);
    for (int g = W.kf_base; g < W.kf_base + W.N; ++g) {
      const int k = cnt[g];
      std::vector<int> T(1, g - W.kf_base);
      for (int s = P.src_off[g]; s < P.src_off[g + 1]; ++s) T.push_back(P.jj[P.src_edges[s]] - W.kf_base);
      for (int ta = 0; ta <= k; ++ta)
        for (int tb = 0; tb <= k; ++tb)
          items[(size_t)T[ta] * W.N + T[tb]].push_back({P.z_off[g] + (ta * (k + 1) + tb) * ZD, P.zb_off[g] + ZBD * ta});
    }
    if (pg) {
      for (int f = 0; f < P.R; ++f) {
        const int i = P.rel_ii[f], j = P.rel_jj[f];
        const int zf = P.rel_z[f], zbf = P.rel_zb[f];
        items[(size_t)i * W.N + i].push_back({zf, zbf});
        items[(size_t)i * W.N + j].push_back({zf + 49, zbf});
        items[(size_t)j * W.N + i].push_back({zf + 98, zbf + 7});
        items[(size_t)j * W.N + j].push_back({zf + 147, zbf + 7});
      }
    }
    // couplings of S: the vision terms couple only the 6 pose unknowns at the
    // head of each keyframe's 15 in the visual-inertial layout (all 7 in the
    // pose graph); the inertial factors the full blocks of consecutive keyframes
    std::vector<Coupling> cpl;
    std::vector<std::vector<int>> adj(W.N);
    for (int a = 0; a < W.N; ++a)
      for (int b = 0; b < a; ++b)
        if (!items[(size_t)a * W.N + b].empty()) cpl.push_back({a, b, pg});
    if (!pg)
      for (int a = 0; a + 1 < W.N; ++a) cpl.push_back({a + 1, a, true});
    // one bias for the window: it sits in the last keyframe's slot and couples
    // with every keyframe that an inertial factor touches
    if (!pg && bias_global)
      for (int a = 0; a + 2 < W.N; ++a) cpl.push_back({W.N - 1, a, true});
    for (const Coupling& c : cpl) {
      adj[c.a].push_back(c.b);
      adj[c.b].push_back(c.a);
    }
    for (auto& v : adj) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    // natural order unless the reverse Cuthill-McKee order lowers the work of
    // the factorisation path this window takes (tile updates of the dataflow
    // path, the band of the one-workgroup path)
    std::vector<int> pos(W.N), fcs;
    for (int a = 0; a < W.N; ++a) pos[a] = a;
    scalar_envelope(W.N, PD, cpl, pos, fcs);
    Envelope env = tile_envelope(fcs, W.n, W.nblk);
    const std::vector<int> rcm = rcm_order(W.N, adj);
    std::vector<int> pos2(W.N);
    for (int q = 0; q < W.N; ++q) pos2[rcm[q]] = q;
    scalar_envelope(W.N, PD, cpl, pos2, fcs);
    Envelope env2 = tile_envelope(fcs, W.n, W.nblk);
    const bool small_path = W.npad <= kCholSmallMaxNpad;
    if (small_path ? env2.band < env.band : env2.work < env.work) {
      pos.swap(pos2);
      env = std::move(env2);
    }
    for (int a = 0; a < W.N; ++a) {
      P.kf_pos[W.kf_base + a] = pos[a];
      P.kf_at[W.kf_base + pos[a]] = a;
    }
    W.band = env.band;
    W.fc_off = (int)P.chol_fc.size();
    P.chol_fc.insert(P.chol_fc.end(), env.fc.begin(), env.fc.end());
    // this window's table: entries pair_base .. pair_base + N*N (the last one is its end)
    W.pair_base = (int)P.pair_off.size();
    for (size_t q = 0; q < items.size(); ++q) {
      P.pair_off.push_back((int32_t)P.pair_z.size());
      for (auto& it : items[q]) {
        P.pair_z.push_back(it.first);
        P.pair_zb.push_back(it.second);
      }
    }
    P.pair_off.push_back((int32_t)P.pair_z.size());
  }
  if (P.pair_z.empty()) { P.pair_z.push_back(0); P.pair_zb.push_back(0); }
  // Cholesky tickets of the windows too large for the one-workgroup path:
  // column j, then window, then block row i (nblk = the right-hand-side
  // block), so that every tile depends on smaller tickets only
  for (int j = 0; j < P.nblk_max; ++j)
    for (int w = 0; w < nw; ++w) {
      const WinDev& W = P.win[w];
      if (j >= W.nblk || W.npad <= kCholSmallMaxNpad) continue;
      const int32_t* fc = &P.chol_fc[W.fc_off];
      // the diagonal tile, unless the ticket of tile (j, j - 1) carries it;
      // tile (j + 1, j) then carries the diagonal tile j + 1 (kPairTicket);
      // tiles outside the envelope are zero in S and in L
      if (j == 0 || fc[j] > j - 1) {
        P.chol_tiles.push_back(w);
        P.chol_tiles.push_back((j << 16) | j);
      }
      for (int i = j + 1; i <= W.nblk; ++i) {
        if (fc[i] > j) continue;
        P.chol_tiles.push_back(w);
        P.chol_tiles.push_back((i << 16) | j | ((i == j + 1 && i < W.nblk) ? kPairTicketFlag : 0));
      }
    }
  P.n_tickets = (int)(P.chol_tiles.size() / 2);
  // then the back-substitution's block columns, last column first, two per
  // ticket (c and c - 1; the ticket of block 0 alone when nblk is odd)
  for (int c = P.nblk_max - 1; c >= 0; --c)
    for (int w = 0; w < nw; ++w) {
      const WinDev& W = P.win[w];
      if (c >= W.nblk || W.npad <= kCholSmallMaxNpad || (W.nblk - 1 - c) % 2 != 0) continue;
      P.chol_tiles.push_back(w);
      P.chol_tiles.push_back(c);
    }
  P.n_bs = (int)(P.chol_tiles.size() / 2) - P.n_tickets;
  P.A_size = A_off;
  P.Linv_size = L_off;
  P.x_size = x_off;
  return VI_OK;
}

// a coordinate of window w's reduced system (in its block order) as
// keyframe * unknowns-per-keyframe + unknown
int natural_coord(const Plan& P, int w, int c) {
  const WinDev& W = P.win[w];
  if (c < 0 || c >= W.n) return c;
  return P.kf_at[W.kf_base + c / P.pdim] * P.pdim + c % P.pdim;
}

void set_range(Plan& P, int range) {
  P.range = range;
  for (WinDev& W : P.win) W.nkr = (W.HW + range - 1) / range;
}

// default pixel range of the fused assembly: the source pixels of the batch
// over about one workgroup per compute unit (a multiple of 64, at least
// kRangeMin), so that small windows still fill the chip and large problems
// keep whole keyframes in one workgroup (one set of Gram partials each)
int default_range(const Plan& P) {
  long long px = 0;
  for (int g = 0; g < P.N; ++g)
    if (P.src_off[g + 1] > P.src_off[g]) px += P.win[P.win_of_kf[g]].HW;
  // pose graph: a source has few loop pairs (out-degree 1-3), so a chunk of
  // pixels carries little work to hide the loads behind; shorter ranges
  // (about four workgroups per compute unit) keep more chunks in flight
  const long long target = P.pdim == 7 ? 4 * kAssemblyWGTarget : kAssemblyWGTarget;
  long long r = (px + target - 1) / target;
  r = (r + 63) / 64 * 64;
  return (int)std::max<long long>(kRangeMin, std::min<long long>(r, (P.hw_max + 63) / 64 * 64));
}

struct Carve {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + off) : nullptr;
    off += align256(std::max<size_t>(count, 1) * sizeof(T));
    return p;
  }
};

Work do_carve(const Plan& P, void* base, size_t* bytes) {
  Carve c;
  c.base = (char*)base;
  Work w{};
  const size_t N = P.N, E = P.E, F = std::max(P.F, 0);
  w.Rw = c.take<double>(N * 9);
  w.rel = c.take<double>(E * 12);
  w.Cd = c.take<double>((size_t)P.pix_total);
  w.wd = c.take<double>((size_t)P.pix_total);
  w.hpart = c.take<double>(E * P.nkr_max * 32);
  w.vcost = c.take<double>(N * cost_slots(P) * 2);
  w.gpart = c.take<double>(P.gram_size);
  w.Z = c.take<double>(P.z_size);
  w.ZB = c.take<double>(P.zb_size);
  w.ZV = c.take<double>(P.zb_size);
  w.Lam = c.take<double>(F * 225);
  w.Hf = c.take<double>(F * 900);
  w.gf = c.take<double>(F * 30);
  w.icost = c.take<double>(F);
  w.A = c.take<double>(P.A_size);
  w.flags = c.take<int32_t>(P.flags_size);
  w.sync = c.take<int32_t>(4);
  w.Linv = c.take<double>(P.Linv_size);
  w.x = c.take<double>(P.x_size);
  w.trace = c.take<double>((size_t)P.n_win * kTraceLen);
  w.rcost = c.take<double>((size_t)std::max(P.R, 1));
  if (bytes) *bytes = c.off;
  return w;
}

// Upload the int tables; the window table at the front is refreshed per call.
vi_status upload_plan(vi_ctx* ctx) {
  const Plan& P = ctx->plan;
  const std::vector<int32_t>* parts[] = {&P.ii, &P.jj, &P.win_of_kf, &P.win_of_f, &P.src_off, &P.src_edges,
                                         &P.gram_off, &P.z_off, &P.zb_off, &P.pair_off, &P.pair_z, &P.pair_zb,
                                         &P.chol_tiles, &P.rel_ii, &P.rel_jj, &P.rel_z, &P.rel_zb,
                                         &P.kf_pos, &P.kf_at, &P.chol_fc};
  size_t total = align256(sizeof(WinDev) * P.n_win);
  for (auto* v : parts) total += align256(std::max<size_t>(v->size(), 1) * sizeof(int32_t));
  if (total > ctx->d_plan_cap) {
    if (ctx->d_plan) HIPCHK(ctx, hipFree(ctx->d_plan));
    ctx->d_plan = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&ctx->d_plan, total));
    ctx->d_plan_cap = total;
  }
  std::vector<char> host(total, 0);
  size_t off = align256(sizeof(WinDev) * P.n_win);
  const int32_t* dptr[20];
  int idx = 0;
  for (auto* v : parts) {
    if (!v->empty()) std::memcpy(host.data() + off, v->data(), v->size() * sizeof(int32_t));
    dptr[idx++] = (const int32_t*)(ctx->d_plan + off);
    off += align256(std::max<size_t>(v->size(), 1) * sizeof(int32_t));
  }
  ctx->win_on_dev.clear();
  HIPCHK(ctx, hipMemcpy(ctx->d_plan, host.data(), total, hipMemcpyHostToDevice));
  DevPlan& D = ctx->dplan;
  ctx->d_win = (WinDev*)ctx->d_plan;
  D.win = ctx->d_win;
  D.ii = dptr[0]; D.jj = dptr[1]; D.win_of_kf = dptr[2]; D.win_of_f = dptr[3]; D.src_off = dptr[4];
  D.src_edges = dptr[5]; D.gram_off = dptr[6]; D.z_off = dptr[7]; D.zb_off = dptr[8];
  D.pair_off = dptr[9]; D.pair_z = dptr[10]; D.pair_zb = dptr[11]; D.chol_tiles = dptr[12];
  D.rel_ii = dptr[13]; D.rel_jj = dptr[14]; D.rel_z = dptr[15]; D.rel_zb = dptr[16];
  D.kf_pos = dptr[17]; D.kf_at = dptr[18]; D.chol_fc = dptr[19];
  return VI_OK;
}

vi_status ensure_status(vi_ctx* ctx, int n) {
  if (n <= ctx->status_cap) return VI_OK;
  if (ctx->status) HIPCHK(ctx, hipFree(ctx->status));
  ctx->status = nullptr;
  HIPCHK(ctx, hipMalloc((void**)&ctx->status, sizeof(DevStatus) * n));
  ctx->status_cap = n;
  return VI_OK;
}

vi_status ensure_plan(vi_ctx* ctx, const std::vector<WinIn>& wins, bool bias_global = false) {
  std::vector<int32_t> sig = plan_signature(wins, bias_global);
  if (ctx->have_plan && sig == ctx->plan_sig) return VI_OK;
  Plan P;
  vi_status s = build_plan(ctx, wins, P, bias_global);
  if (s != VI_OK) return s;
  set_range(P, default_range(P));
  ctx->plan = std::move(P);
  ctx->plan_sig = std::move(sig);
  ctx->have_plan = false;
  s = upload_plan(ctx);
  if (s != VI_OK) return s;
  s = ensure_status(ctx, ctx->plan.n_win);
  if (s != VI_OK) return s;
  ctx->have_plan = true;
  ctx->plan_version++;
  if (ctx->plan.kmax > ctx->attr_kmax) {
    step_set_attributes(ctx->plan.kmax);
    pg_set_attributes();
    ctx->attr_kmax = ctx->plan.kmax;
  }
  return VI_OK;
}

// body-from-camera extrinsic (t, q xyzw) -> row-major R_bc, t_bc and whether
// it differs from the identity; a zero quaternion (or no extrinsic) is the identity
void extrinsic_rotation(const double* T, double* R, double* t, int* ext) {
  double q[4] = {0.0, 0.0, 0.0, 1.0};
  double n = 0.0;
  if (T)
    for (int k = 0; k < 4; ++k) n += T[3 + k] * T[3 + k];
  if (T && n > 0.0)
    for (int k = 0; k < 4; ++k) q[k] = T[3 + k] / std::sqrt(n);
  const double x = q[0], y = q[1], z = q[2], w = q[3];
  const double Rm[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w),     2 * (x * z + y * w),
                        2 * (x * y + z * w),     1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                        2 * (x * z - y * w),     2 * (y * z + x * w),     1 - 2 * (x * x + y * y)};
  for (int k = 0; k < 9; ++k) R[k] = Rm[k];
  for (int k = 0; k < 3; ++k) t[k] = T ? T[k] : 0.0;
  *ext = (T && (t[0] != 0.0 || t[1] != 0.0 || t[2] != 0.0 || (n > 0.0 && (x != 0.0 || y != 0.0 || z != 0.0)))) ? 1 : 0;
}

// this call's window pointers -> host window table -> device
vi_status refresh_windows(vi_ctx* ctx, const std::vector<WinIn>& wins, bool depth_f32 = false) {
  Plan& P = ctx->plan;
  for (int w = 0; w < P.n_win; ++w) {
    WinDev& W = P.win[w];
    const WinIn& in = wins[w];
    W.fx = in.cam->fx; W.fy = in.cam->fy; W.cx = in.cam->cx; W.cy = in.cam->cy;
    for (int k = 0; k < 3; ++k) W.g[k] = in.cam->gravity[k];
    // camera-IMU extrinsic (the pose-graph adjustment's poses are camera poses: none there)
    extrinsic_rotation(in.rel ? nullptr : in.cam->T_bc, W.Rbc, W.tbc, &W.ext);
    W.pose = in.st->pose; W.vel = in.st->vel; W.bias = in.st->bias;
    W.invdepth = depth_f32 ? nullptr : (double*)in.st->invdepth;
    W.invdepth32 = depth_f32 ? (float*)in.st->invdepth : nullptr;
    W.target = in.ed->target; W.weight = in.ed->weight; W.imu = in.imu;
    W.rep_dxi = in.rep ? in.rep->dxi : nullptr;
    W.rep_dd = in.rep ? in.rep->dd : nullptr;
    W.scale = in.scale;
    W.rel_meas = in.rel ? in.rel->meas : nullptr;
    W.rel_info = in.rel ? in.rel->info : nullptr;
  }
  // a blocking copy: send it only when the table differs from what the device holds
  const size_t nb = sizeof(WinDev) * P.n_win;
  const char* hb = (const char*)P.win.data();
  if (ctx->win_on_dev.size() == nb && std::memcmp(ctx->win_on_dev.data(), hb, nb) == 0) return VI_OK;
  ctx->win_on_dev.clear();
  HIPCHK(ctx, hipMemcpy(ctx->d_win, hb, nb, hipMemcpyHostToDevice));
  ctx->win_on_dev.assign(hb, hb + nb);
  return VI_OK;
}

struct TimingUser {
  hipStream_t s;
  hipEvent_t* ev;    // [kNumStages + 1]
};

void mark_event(void* user, int stage_done) {
  TimingUser* t = (TimingUser*)user;
  (void)hipEventRecord(t->ev[stage_done + 1], t->s);
}

// Time each candidate tiling of the fused assembly on the actual inputs and
// keep the fastest for this batch shape.  The candidates run the assembly and
// local-block stages only, which write the workspace, never the caller's state.
vi_status autotune_range(vi_ctx* ctx, const Work& w, const OptsDev& od) {
  Plan& P = ctx->plan;
  const bool pg = P.pdim == 7;
  const auto key = std::make_tuple(P.hw_max, P.kmax, P.N, P.n_win * (pg ? -1 : 1));
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    set_range(P, it->second);
    return VI_OK;
  }
  hipStream_t sp = ctx->priv;
  hipEvent_t ev[kNumStages + 1];
  for (auto& e : ev) HIPCHK(ctx, hipEventCreate(&e));
  launch_reset_status(sp, ctx->status, P.n_win);
  if (od.use_imu) launch_imu_info(sp, P, ctx->dplan, w.Lam, ctx->status);
  TimingUser tu{sp, ev};
  int best = default_range(P);
  float best_ms = 1e30f;
  std::vector<int> cand(std::begin(kRanges), std::end(kRanges));
  cand.push_back(best);
  std::sort(cand.begin(), cand.end());
  bool whole = false;            // a candidate already covers a whole keyframe
  for (int r : cand) {
    if (whole) break;
    whole = r >= P.hw_max;
    set_range(P, r);
    ctx->win_on_dev.clear();
    HIPCHK(ctx, hipMemcpy(ctx->d_win, P.win.data(), sizeof(WinDev) * P.n_win, hipMemcpyHostToDevice));
    float tot = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(ctx, hipEventRecord(ev[0], sp));
      if (pg) {
        // pose graph: the fused assembly of the loop pairs and the per-source blocks
        launch_vis_assembly(sp, P, ctx->dplan, w, od, ctx->status);
        launch_pg_local(sp, P, ctx->dplan, w, ctx->status);
        HIPCHK(ctx, hipEventRecord(ev[kStLocal + 1], sp));
      } else {
        launch_tune_stages(sp, P, ctx->dplan, w, od, mark_event, &tu);
      }
      HIPCHK(ctx, hipEventSynchronize(ev[kStLocal + 1]));
      float ms = 0.f;
      HIPCHK(ctx, hipEventElapsedTime(&ms, ev[0], ev[kStLocal + 1]));
      if (rep > 0) tot += ms;
    }
    if (tot < best_ms) {
      best_ms = tot;
      best = r;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  ctx->tuned[key] = best;
  set_range(P, best);
  return VI_OK;
}

// canvas of the warm start: the largest cell grid of the windows
void warm_canvas(const std::vector<WinIn>& wins, int* hq, int* wq) {
  *hq = 1;
  *wq = 1;
  for (const WinIn& in : wins) {
    *hq = std::max(*hq, (in.cam->H + 3) / 4);
    *wq = std::max(*wq, (in.cam->W + 3) / 4);
  }
}

// the warm start's own buffers, after the solver's workspace
struct WarmWork {
  float* feat;
  int32_t* dims;
  float* dd;
  float* db;
  double* saved_d;
  double* saved_b;
  double* trace;       // [n_win][kTraceLen]: F at the initial (slot 0) and corrected (slot 1) state
  void* wprep;         // the network's weights in their LDS layout
};

struct WarmArgs {
  const float* params;
  int hq, wq;
};

WarmWork warm_carve(const Plan& P, int hq, int wq, void* base, size_t* bytes) {
  size_t solve = 0;
  do_carve(P, nullptr, &solve);
  Carve c;
  c.base = base ? (char*)base + solve : nullptr;
  const size_t n = P.N, cells = (size_t)hq * wq;
  WarmWork ww{};
  ww.feat = c.take<float>(n * kWCin * cells);
  ww.dims = c.take<int32_t>(n * 2);
  ww.dd = c.take<float>(n * cells);
  ww.db = c.take<float>(n * 6);
  ww.saved_d = c.take<double>((size_t)P.pix_total);
  ww.saved_b = c.take<double>(n * 6);
  ww.trace = c.take<double>((size_t)P.n_win * kTraceLen);
  ww.wprep = c.take<char>(wnet_prep_bytes());
  if (bytes) *bytes = solve + c.off;
  return ww;
}

// warm start before the iterations (the corrections of a window are kept only
// where the cost falls); needs the inertial information already formed
void launch_warm_prologue(hipStream_t sp, const Plan& P, const DevPlan& D, const Work& w, const OptsDev& od,
                          const WarmArgs& wa, const WarmWork& ww) {
  launch_final_cost(sp, P, D, w, od, 0, ww.trace);
  // the input planes, with the copy of the inverse depths and biases taken on the way
  launch_warm_features(sp, P, D, od, wa.hq, wa.wq, ww.feat, ww.dims, ww.saved_d, ww.saved_b);
  launch_wnet_forward(sp, P.N, wa.hq, wa.wq, ww.dims, wa.params, ww.feat, nullptr, ww.dd, ww.db, ww.wprep);
  // the corrections are applied by the cost kernel of the corrected state
  launch_final_cost(sp, P, D, w, od, 1, ww.trace, ww.dd, ww.db, wa.hq, wa.wq, od.d_min);
  launch_warm_state(sp, P, D, ww.saved_d, ww.saved_b, ww.trace, 1);
}

// The solver: optional warm start (wa), then iters Gauss-Newton steps and the
// final cost, captured once per shape as a HIP graph (eager when stage times
// are asked for).  With a warm start, iters may be 0 and accepted[w] reports
// whether window w kept its corrections.
vi_status run(vi_ctx* ctx, const std::vector<WinIn>& wins, const vi_opts* o, int iters, void* workspace,
              size_t workspace_bytes, const WarmArgs* wa = nullptr, int32_t* accepted = nullptr) {
  if (!ctx) return VI_EINVAL;
  vi_status s = check_opts(ctx, o);
  if (s != VI_OK) return s;
  if (wins.empty()) return fail(ctx, VI_EINVAL, "no windows");
  for (size_t w = 0; w < wins.size(); ++w) {
    s = check_window(ctx, (int)w, wins[w], o, true);
    if (s != VI_OK) return s;
  }
  const int min_iters = wa ? 0 : 1;
  if (iters < min_iters || iters > kMaxIters)
    return fail(ctx, VI_EINVAL, "iters must be in [%d, %d]", min_iters, kMaxIters);
  if (wa) {
    if (!wa->params) return fail(ctx, VI_EINVAL, "null warm-start parameters");
    if (wa->hq > kWHQMax || wa->wq > kWWQMax)
      return fail(ctx, VI_EINVAL, "warm start: maps of up to %d x %d pixels only", 4 * kWHQMax, 4 * kWWQMax);
  }
  if (!workspace) return fail(ctx, VI_EINVAL, "null workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(ctx, VI_EINVAL, "workspace must be 256-byte aligned");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  s = ensure_plan(ctx, wins, o->use_imu && o->bias_mode == VI_BIAS_GLOBAL);
  if (s != VI_OK) return s;
  Plan& P = ctx->plan;
  size_t need = 0;
  if (wa)
    warm_carve(P, wa->hq, wa->wq, nullptr, &need);
  else
    do_carve(P, nullptr, &need);
  if (workspace_bytes < need)
    return fail(ctx, VI_ENOMEM, "workspace too small: %zu bytes given, %zu needed", workspace_bytes, need);
  Work w = do_carve(P, workspace, nullptr);
  const WarmWork ww = wa ? warm_carve(P, wa->hq, wa->wq, workspace, nullptr) : WarmWork{};
  OptsDev od{o->n_fixed, o->use_imu ? 1 : 0, o->bias_mode == VI_BIAS_FIXED ? 1 : 0, o->precision, o->lm_lambda, o->depth_eta,
             o->z_min, o->d_min, ctx->tol, (o->use_imu && o->bias_mode == VI_BIAS_GLOBAL) ? 1 : 0};
  const bool timing = wins[0].rep && wins[0].rep->stage_ms;

  // order after the caller's pending work
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  hipStream_t sp = ctx->priv;

  s = refresh_windows(ctx, wins, o->invdepth_f32 != 0);
  if (s != VI_OK) return s;
  if (ctx->autotune) {
    s = autotune_range(ctx, w, od);
    if (s != VI_OK) return s;
    s = refresh_windows(ctx, wins, o->invdepth_f32 != 0);
    if (s != VI_OK) return s;
  }
  const DevPlan& D = ctx->dplan;

  if (timing) {
    std::vector<hipEvent_t> ev(kNumStages + 1);
    for (auto& e : ev) HIPCHK(ctx, hipEventCreate(&e));
    std::vector<double> acc(VI_NUM_STAGES, 0.0);
    launch_reset_status(sp, ctx->status, P.n_win);
    if (od.use_imu) launch_imu_info(sp, P, D, w.Lam, ctx->status);
    if (wa) launch_warm_prologue(sp, P, D, w, od, *wa, ww);
    TimingUser tu{sp, ev.data()};
    for (int it = 0; it < iters; ++it) {
      HIPCHK(ctx, hipEventRecord(ev[0], sp));
      launch_step(sp, P, D, w, od, it, ctx->status, mark_event, &tu);
      HIPCHK(ctx, hipEventSynchronize(ev[kNumStages]));
      for (int k = 0; k < kNumStages; ++k) {
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
        acc[k] += ms;
      }
    }
    HIPCHK(ctx, hipEventRecord(ev[0], sp));
    launch_final_cost(sp, P, D, w, od, iters);
    HIPCHK(ctx, hipEventRecord(ev[1], sp));
    HIPCHK(ctx, hipEventSynchronize(ev[1]));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ev[0], ev[1]));
    acc[kNumStages] += ms;
    for (int k = 0; k < VI_NUM_STAGES; ++k) wins[0].rep->stage_ms[k] = (float)acc[k];
    for (auto& e : ev) (void)hipEventDestroy(e);
  } else {
    std::vector<uint64_t> key;
    key.push_back(ctx->plan_version);
    key.push_back((uint64_t)iters);
    key.push_back((uint64_t)P.range);
    uint64_t tb;
    std::memcpy(&tb, &od.tol, sizeof(tb));
    key.push_back(tb);
    uint64_t ob[sizeof(vi_opts) / 8];
    std::memcpy(ob, o, sizeof(vi_opts));
    key.insert(key.end(), ob, ob + sizeof(vi_opts) / 8);
    key.push_back((uint64_t)(uintptr_t)workspace);
    key.push_back((uint64_t)(uintptr_t)(wa ? wa->params : nullptr));
    key.push_back(wa ? (uint64_t)(wa->hq * 1000 + wa->wq) : 0);
    for (const WinDev& W : P.win) {
      const void* ptrs[] = {W.pose,   W.vel,    W.bias, W.invdepth, W.invdepth32, W.target,
                            W.weight, W.imu,    W.rep_dxi, W.rep_dd};
      for (const void* p : ptrs) key.push_back((uint64_t)(uintptr_t)p);
      uint64_t cam[19];
      const double cv[19] = {W.fx,     W.fy,     W.cx,     W.cy,     W.g[0],   W.g[1],   W.g[2],
                             W.Rbc[0], W.Rbc[1], W.Rbc[2], W.Rbc[3], W.Rbc[4], W.Rbc[5], W.Rbc[6],
                             W.Rbc[7], W.Rbc[8], W.tbc[0], W.tbc[1], W.tbc[2]};
      std::memcpy(cam, cv, sizeof(cv));
      key.insert(key.end(), cam, cam + 19);
    }
    if (!ctx->have_graph || key != ctx->gkey) {
      if (ctx->exec) { (void)hipGraphExecDestroy(ctx->exec); ctx->exec = nullptr; }
      if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
      ctx->have_graph = false;
      HIPCHK(ctx, hipStreamBeginCapture(sp, hipStreamCaptureModeThreadLocal));
      launch_reset_status(sp, ctx->status, P.n_win);
      if (od.use_imu) launch_imu_info(sp, P, D, w.Lam, ctx->status);
      if (wa) launch_warm_prologue(sp, P, D, w, od, *wa, ww);
      for (int it = 0; it < iters; ++it) launch_step(sp, P, D, w, od, it, ctx->status);
      launch_final_cost(sp, P, D, w, od, iters);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(sp, &g);
      if (e != hipSuccess) return fail(ctx, VI_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
      ctx->graph = g;
      HIPCHK(ctx, hipGraphInstantiate(&ctx->exec, g, nullptr, nullptr, 0));
      ctx->gkey = key;
      ctx->have_graph = true;
    }
    HIPCHK(ctx, hipGraphLaunch(ctx->exec, sp));
  }
  HIPCHK(ctx, hipGetLastError());
  std::vector<DevStatus> hs(P.n_win);
  std::vector<double> trace((size_t)P.n_win * kTraceLen);
  HIPCHK(ctx, hipMemcpyAsync(hs.data(), ctx->status, sizeof(DevStatus) * P.n_win, hipMemcpyDeviceToHost, sp));
  HIPCHK(ctx, hipMemcpyAsync(trace.data(), w.trace, sizeof(double) * trace.size(), hipMemcpyDeviceToHost, sp));
  std::vector<double> wtrace(wa ? trace.size() : 0);
  if (wa)
    HIPCHK(ctx, hipMemcpyAsync(wtrace.data(), ww.trace, sizeof(double) * wtrace.size(), hipMemcpyDeviceToHost, sp));
  HIPCHK(ctx, hipStreamSynchronize(sp));
  int first_bad = -1;
  for (int wi = 0; wi < P.n_win; ++wi) {
    if (hs[wi].code != 0 && first_bad < 0) first_bad = wi;
    vi_report* rep = wins[wi].rep;
    if (!rep) continue;
    const double* tr = trace.data() + (size_t)wi * kTraceLen;
    rep->iters_done = hs[wi].iters;
    rep->tile_px = P.range;
    const int last = std::max(0, std::min(hs[wi].iters, iters) - 1);
    rep->cost_before = tr[2 * last];
    rep->n_valid = (int64_t)tr[2 * last + 1];
    rep->cost_after = tr[2 * iters];
    if (rep->costs)
      for (int t = 0; t <= iters; ++t) rep->costs[t] = tr[2 * t];
    if (wa && iters == 0) {
      // the warm start alone: initial F, then F of the state left behind
      const double* wt = wtrace.data() + (size_t)wi * kTraceLen;
      rep->cost_before = wt[0];
      rep->n_valid = (int64_t)wt[1];
      if (rep->costs) {
        rep->costs[0] = wt[0];
        rep->costs[1] = wt[2];
      }
    }
  }
  if (wa && accepted)
    for (int wi = 0; wi < P.n_win; ++wi)
      accepted[wi] = wtrace[(size_t)wi * kTraceLen + 2] < wtrace[(size_t)wi * kTraceLen] ? 1 : 0;
  if (first_bad >= 0) {
    const DevStatus& b = hs[first_bad];
    if (b.code == VI_ENOTPD)
      return fail(ctx, VI_ENOTPD, "window %d: reduced system not positive definite at coordinate %d (step %d)",
                  first_bad, natural_coord(P, first_bad, b.detail), b.iters);
    if (b.code == VI_ENONFINITE)
      return fail(ctx, VI_ENONFINITE, "window %d: non-finite reduced system at coordinate %d (step %d)", first_bad,
                  b.detail, b.iters);
    return fail(ctx, (vi_status)b.code, "window %d: device error %d (detail %d)", first_bad, b.code, b.detail);
  }
  ctx->err.clear();
  return VI_OK;
}


// Host checks of a pose-graph problem; fills the window description.
vi_status pg_window(vi_ctx* ctx, const vi_camera* cam, int32_t n_kf, double* pose, double* scale, double* invdepth,
                    const vi_edges* loops, const vi_rel_poses* rel, const vi_opts* o, vi_report* rep, bool full,
                    vi_state& st, WinIn& in) {
  if (!cam || !loops || !rel) return fail(ctx, VI_EINVAL, "null argument");
  vi_status s = check_opts(ctx, o);
  if (s != VI_OK) return s;
  if (o->invdepth_f32) return fail(ctx, VI_EINVAL, "the pose-graph adjustment takes float64 inverse depths");
  if (rel->n_rel < 0) return fail(ctx, VI_EINVAL, "negative relative-pose count");
  if (rel->n_rel > 0 && (!rel->ii || !rel->jj)) return fail(ctx, VI_EINVAL, "null relative-pose index array");
  if (full && rel->n_rel > 0 && (!rel->meas || !rel->info))
    return fail(ctx, VI_EINVAL, "null relative-pose measurement array");
  if (full && (!pose || !scale || !invdepth)) return fail(ctx, VI_EINVAL, "null state array");
  st = vi_state{};
  st.n_kf = n_kf;
  st.pose = pose;
  st.vel = pose;          // not used by the pose-graph adjustment
  st.bias = pose;
  st.invdepth = invdepth;
  in = WinIn{cam, &st, loops, nullptr, rep};
  in.scale = scale;
  in.rel = rel;
  vi_opts oo = *o;
  oo.use_imu = 0;
  return check_window(ctx, 0, in, &oo, full);
}

// iters damped Gauss-Newton steps of the pose-graph adjustment in Sim(3),
// launched eagerly on the private stream; per step: fused vision assembly
// (loop pairs), per-source 7x7 blocks, relative-pose factors, cost of the
// linearisation point, reduced system, Cholesky, back-substitution and
// retraction; then the final cost
vi_status run_pgba(vi_ctx* ctx, const vi_camera* cam, int32_t n_kf, double* pose, double* scale, double* invdepth,
                   const vi_edges* loops, const vi_rel_poses* rel, const vi_opts* o, int iters, void* workspace,
                   size_t workspace_bytes, vi_report* rep) {
  vi_state st;
  WinIn in{nullptr, nullptr, nullptr, nullptr, nullptr};
  vi_status s = pg_window(ctx, cam, n_kf, pose, scale, invdepth, loops, rel, o, rep, true, st, in);
  if (s != VI_OK) return s;
  if (iters < 1 || iters > kMaxIters) return fail(ctx, VI_EINVAL, "iters must be in [1, %d]", kMaxIters);
  if (!workspace) return fail(ctx, VI_EINVAL, "null workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(ctx, VI_EINVAL, "workspace must be 256-byte aligned");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<WinIn> wins{in};
  s = ensure_plan(ctx, wins);
  if (s != VI_OK) return s;
  Plan& P = ctx->plan;
  size_t need = 0;
  do_carve(P, nullptr, &need);
  if (workspace_bytes < need)
    return fail(ctx, VI_ENOMEM, "workspace too small: %zu bytes given, %zu needed", workspace_bytes, need);
  Work w = do_carve(P, workspace, nullptr);
  OptsDev od{o->n_fixed, 0, 0, o->precision, o->lm_lambda, o->depth_eta, o->z_min, o->d_min, ctx->tol};
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  hipStream_t sp = ctx->priv;
  s = refresh_windows(ctx, wins);
  if (s != VI_OK) return s;
  if (ctx->autotune) {
    s = autotune_range(ctx, w, od);
    if (s != VI_OK) return s;
    s = refresh_windows(ctx, wins);
    if (s != VI_OK) return s;
  }
  const DevPlan& D = ctx->dplan;
  const int ncost = cost_slots(P);
  launch_reset_status(sp, ctx->status, P.n_win);
  for (int it = 0; it < iters; ++it) {
    launch_vis_assembly(sp, P, D, w, od, ctx->status);
    launch_pg_local(sp, P, D, w, ctx->status);
    launch_pg_relpose(sp, P, D, w, ctx->status, true);
    launch_pg_cost(sp, P, D, w, ncost, P.range, it, od.tol, ctx->status);
    launch_pg_assemble(sp, P, D, w, od.n_fixed, od.lambda, ctx->status);
    launch_chol(sp, P, D, w, ctx->status);
    launch_pg_backsub(sp, P, D, w, od, ctx->status);
  }
  launch_vis_cost(sp, P, D, w, od);
  launch_pg_relpose(sp, P, D, w, ctx->status, false);
  launch_pg_cost(sp, P, D, w, ncost, kVisBlock, iters, 0.0, nullptr);
  HIPCHK(ctx, hipGetLastError());
  DevStatus hs;
  std::vector<double> trace(kTraceLen);
  HIPCHK(ctx, hipMemcpyAsync(&hs, ctx->status, sizeof(DevStatus), hipMemcpyDeviceToHost, sp));
  HIPCHK(ctx, hipMemcpyAsync(trace.data(), w.trace, sizeof(double) * kTraceLen, hipMemcpyDeviceToHost, sp));
  HIPCHK(ctx, hipStreamSynchronize(sp));
  if (rep) {
    rep->iters_done = hs.iters;
    rep->tile_px = P.range;
    const int last = std::max(0, std::min(hs.iters, iters) - 1);
    rep->cost_before = trace[2 * last];
    rep->n_valid = (int64_t)trace[2 * last + 1];
    rep->cost_after = trace[2 * iters];
    if (rep->costs)
      for (int t = 0; t <= iters; ++t) rep->costs[t] = trace[2 * t];
    if (rep->stage_ms)
      for (int k = 0; k < VI_NUM_STAGES; ++k) rep->stage_ms[k] = 0.0f;
  }
  if (hs.code != 0) {
    if (hs.code == VI_ENOTPD)
      return fail(ctx, VI_ENOTPD, "reduced system not positive definite at coordinate %d (step %d)",
                  natural_coord(P, 0, hs.detail), hs.iters);
    if (hs.code == VI_ENONFINITE)
      return fail(ctx, VI_ENONFINITE, "non-finite reduced system at coordinate %d (step %d)", hs.detail, hs.iters);
    return fail(ctx, (vi_status)hs.code, "device error %d (detail %d)", hs.code, hs.detail);
  }
  ctx->err.clear();
  return VI_OK;
}

}  // namespace

extern "C" {

const char* vi_version(void) { return "vi-ba-mi355x 0.3 (gfx950; fp64 and mixed fp32/fp64)"; }

vi_status vi_ctx_create(int32_t device, void* stream, vi_ctx** out) {
  if (!out) return VI_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return VI_EDEVICE;
  vi_ctx* c = new vi_ctx();
  c->device = device;
  c->user = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess || reanchor_scratch_init(device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->priv, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess || ensure_status(c, 1) != VI_OK) {
    vi_ctx_destroy(c);
    return VI_EDEVICE;
  }
  wnet_set_attributes();
  DevStatus z{0, 0, 0, 0};
  if (hipMemcpy(c->status, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) {
    vi_ctx_destroy(c);
    return VI_EDEVICE;
  }
  *out = c;
  return VI_OK;
}

void vi_ctx_destroy(vi_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->priv) (void)hipStreamSynchronize(c->priv);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->d_plan) (void)hipFree(c->d_plan);
  if (c->d_off) (void)hipFree(c->d_off);
  if (c->status) (void)hipFree(c->status);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->priv) (void)hipStreamDestroy(c->priv);
  delete c;
}

vi_status vi_ctx_set_stream(vi_ctx* ctx, void* stream) {
  if (!ctx) return VI_EINVAL;
  ctx->user = (hipStream_t)stream;
  return VI_OK;
}

vi_status vi_ctx_set_autotune(vi_ctx* ctx, int32_t enable) {
  if (!ctx) return VI_EINVAL;
  ctx->autotune = enable != 0;
  return VI_OK;
}

vi_status vi_ctx_set_tolerance(vi_ctx* ctx, double rel_tol) {
  if (!ctx) return VI_EINVAL;
  if (!(rel_tol >= 0.0 && rel_tol < 1.0)) return fail(ctx, VI_EINVAL, "rel_tol must be in [0, 1)");
  ctx->tol = rel_tol;
  return VI_OK;
}

const char* vi_last_error(const vi_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

vi_status imu_preintegrate(vi_ctx* ctx, int32_t F, const int32_t* off, const double* gyro, const double* accel,
                           const double* dt, const double* bias_hat, const vi_imu_noise* noise, vi_preint* out) {
  if (!ctx) return VI_EINVAL;
  if (F < 1) return fail(ctx, VI_EINVAL, "need at least one factor");
  if (!off || !gyro || !accel || !dt || !bias_hat || !noise || !out) return fail(ctx, VI_EINVAL, "null argument");
  if (off[0] != 0) return fail(ctx, VI_EINVAL, "off[0] must be 0");
  for (int f = 0; f < F; ++f)
    if (off[f + 1] <= off[f]) return fail(ctx, VI_EINVAL, "factor %d has no samples (off not increasing)", f);
  const double nz[4] = {noise->sigma_g, noise->sigma_a, noise->sigma_bgw, noise->sigma_baw};
  for (double v : nz)
    if (!(v >= 0.0) || !std::isfinite(v)) return fail(ctx, VI_EINVAL, "noise densities must be finite and >= 0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const size_t bytes = sizeof(int32_t) * (F + 1);
  if (bytes > ctx->d_off_cap) {
    ctx->off_on_dev.clear();
    if (ctx->d_off) HIPCHK(ctx, hipFree(ctx->d_off));
    ctx->d_off = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&ctx->d_off, bytes));
    ctx->d_off_cap = bytes;
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  // the CSR is sent only when it differs from what the device holds (the
  // previous call has completed: it ends with a synchronisation)
  if (ctx->off_on_dev.size() != (size_t)F + 1 || std::memcmp(ctx->off_on_dev.data(), off, bytes) != 0) {
    ctx->off_on_dev.clear();
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_off, off, bytes, hipMemcpyHostToDevice, ctx->priv));
    ctx->off_on_dev.assign(off, off + F + 1);
  }
  launch_reset_status(ctx->priv, ctx->status, 1);
  launch_preint(ctx->priv, F, ctx->d_off, gyro, accel, dt, bias_hat, *noise, out, ctx->status);
  HIPCHK(ctx, hipGetLastError());
  DevStatus hs;
  HIPCHK(ctx, hipMemcpyAsync(&hs, ctx->status, sizeof(hs), hipMemcpyDeviceToHost, ctx->priv));
  HIPCHK(ctx, hipStreamSynchronize(ctx->priv));
  if (hs.code == VI_EINVAL) return fail(ctx, VI_EINVAL, "non-positive or non-finite dt at sample %d", hs.detail);
  if (hs.code != 0) return fail(ctx, (vi_status)hs.code, "device error %d", hs.code);
  ctx->err.clear();
  return VI_OK;
}

size_t vi_workspace_size_batched(int32_t n_windows, const vi_window* windows, const vi_opts* opts) {
  if (n_windows < 1 || !windows || !opts) return 0;
  std::vector<WinIn> wins;
  for (int w = 0; w < n_windows; ++w) {
    WinIn in{&windows[w].cam, &windows[w].state, &windows[w].edges, windows[w].imu, nullptr};
    if (check_window(nullptr, w, in, opts, false) != VI_OK) return 0;
    wins.push_back(in);
  }
  Plan P;
  if (build_plan(nullptr, wins, P) != VI_OK) return 0;
  set_range(P, default_range(P));
  size_t b = 0;
  do_carve(P, nullptr, &b);
  return b;
}

size_t vi_workspace_size(const vi_camera* cam, int32_t n_kf, const vi_edges* edges, const vi_opts* opts) {
  if (!cam || !edges || !opts) return 0;
  vi_window w;
  std::memset(&w, 0, sizeof(w));
  w.cam = *cam;
  w.state.n_kf = n_kf;
  w.edges = *edges;
  return vi_workspace_size_batched(1, &w, opts);
}

vi_status vi_ba_solve_batched(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                              int32_t iters, void* workspace, size_t workspace_bytes) {
  if (!ctx) return VI_EINVAL;
  if (n_windows < 1 || !windows) return fail(ctx, VI_EINVAL, "need at least one window");
  std::vector<WinIn> wins;
  for (int w = 0; w < n_windows; ++w)
    wins.push_back(WinIn{&windows[w].cam, &windows[w].state, &windows[w].edges, windows[w].imu, windows[w].report});
  return run(ctx, wins, opts, iters, workspace, workspace_bytes);
}

size_t vi_pgba_workspace_size(const vi_camera* cam, int32_t n_kf, const vi_edges* loops, const vi_rel_poses* rel,
                              const vi_opts* opts) {
  vi_state st;
  WinIn in{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (pg_window(nullptr, cam, n_kf, nullptr, nullptr, nullptr, loops, rel, opts, nullptr, false, st, in) != VI_OK)
    return 0;
  std::vector<WinIn> wins{in};
  Plan P;
  if (build_plan(nullptr, wins, P) != VI_OK) return 0;
  set_range(P, default_range(P));
  size_t b = 0;
  do_carve(P, nullptr, &b);
  return b;
}

vi_status vi_pgba_solve(vi_ctx* ctx, const vi_camera* cam, int32_t n_kf, double* pose, double* scale,
                        double* invdepth, const vi_edges* loops, const vi_rel_poses* rel, const vi_opts* opts,
                        int32_t iters, void* workspace, size_t workspace_bytes, vi_report* report) {
  if (!ctx) return VI_EINVAL;
  return run_pgba(ctx, cam, n_kf, pose, scale, invdepth, loops, rel, opts, iters, workspace, workspace_bytes,
                  report);
}

vi_status vi_ba_step(vi_ctx* ctx, const vi_camera* cam, vi_state* state, const vi_edges* edges,
                     const vi_preint* imu, const vi_opts* opts, void* workspace, size_t workspace_bytes,
                     vi_report* report) {
  return vi_ba_solve(ctx, cam, state, edges, imu, opts, 1, workspace, workspace_bytes, report);
}

vi_status vi_ba_solve(vi_ctx* ctx, const vi_camera* cam, vi_state* state, const vi_edges* edges,
                      const vi_preint* imu, const vi_opts* opts, int32_t iters, void* workspace,
                      size_t workspace_bytes, vi_report* report) {
  if (!ctx) return VI_EINVAL;
  if (!cam || !state || !edges) return fail(ctx, VI_EINVAL, "null argument");
  std::vector<WinIn> wins{WinIn{cam, state, edges, imu, report}};
  return run(ctx, wins, opts, iters, workspace, workspace_bytes);
}

// ---------------------------------------------------------------------------
// learned warm start
// ---------------------------------------------------------------------------
int32_t vi_warm_param_count(void) { return kWParams; }

size_t vi_warm_workspace_size(int32_t n_img, int32_t hq, int32_t wq) {
  if (n_img < 1 || hq < 1 || wq < 1 || hq > kWHQMax || wq > kWWQMax) return 0;
  const size_t n = n_img, cells = (size_t)hq * wq;
  size_t b = 0;
  b += align256(n * 5 * cells * kWC * 2);        // BF16 activations
  b += 2 * align256(n * cells * sizeof(float));  // dd, g_dd
  b += 2 * align256(n * 6 * sizeof(float));      // db, g_db
  b += align256(n * sizeof(float));              // per-image loss
  b += align256(n * kWParams * sizeof(float));   // per-image gradient partials
  return b;
}

}  // extern "C"

namespace {

vi_status warm_check_canvas(vi_ctx* ctx, int32_t n_img, int32_t hq, int32_t wq) {
  if (n_img < 1) return fail(ctx, VI_EINVAL, "need at least one image");
  if (hq < 1 || wq < 1 || hq > kWHQMax || wq > kWWQMax)
    return fail(ctx, VI_EINVAL, "canvas %d x %d cells outside [1, %d] x [1, %d]", hq, wq, kWHQMax, kWWQMax);
  return VI_OK;
}

// order the private stream after the caller's pending work
vi_status warm_begin(vi_ctx* ctx) {
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  return VI_OK;
}

vi_status warm_end(vi_ctx* ctx) {
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipStreamSynchronize(ctx->priv));
  ctx->err.clear();
  return VI_OK;
}

// windows -> plan -> device window table (shared with the solver's plan cache)
vi_status warm_windows(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* o, int32_t hq,
                       int32_t wq, std::vector<WinIn>& wins) {
  if (n_windows < 1 || !windows) return fail(ctx, VI_EINVAL, "need at least one window");
  vi_status s = check_opts(ctx, o);
  if (s != VI_OK) return s;
  for (int w = 0; w < n_windows; ++w) {
    wins.push_back(WinIn{&windows[w].cam, &windows[w].state, &windows[w].edges, windows[w].imu, nullptr});
    s = check_window(ctx, w, wins.back(), o, true);
    if (s != VI_OK) return s;
    if ((windows[w].cam.H + 3) / 4 > hq || (windows[w].cam.W + 3) / 4 > wq)
      return fail(ctx, VI_EINVAL, "window %d: its %d x %d cell grid does not fit the %d x %d canvas", w,
                  (windows[w].cam.H + 3) / 4, (windows[w].cam.W + 3) / 4, hq, wq);
  }
  s = ensure_plan(ctx, wins, o->use_imu && o->bias_mode == VI_BIAS_GLOBAL);
  if (s != VI_OK) return s;
  return refresh_windows(ctx, wins, o->invdepth_f32 != 0);
}

}  // namespace

extern "C" {

size_t vi_warm_start_workspace_size(int32_t n_windows, const vi_window* windows, const vi_opts* opts) {
  if (n_windows < 1 || !windows || !opts) return 0;
  std::vector<WinIn> wins;
  for (int w = 0; w < n_windows; ++w) {
    WinIn in{&windows[w].cam, &windows[w].state, &windows[w].edges, windows[w].imu, nullptr};
    if (check_window(nullptr, w, in, opts, false) != VI_OK) return 0;
    wins.push_back(in);
  }
  Plan P;
  if (build_plan(nullptr, wins, P) != VI_OK) return 0;
  set_range(P, default_range(P));
  int hq, wq;
  warm_canvas(wins, &hq, &wq);
  size_t b = 0;
  warm_carve(P, hq, wq, nullptr, &b);
  return b;
}

vi_status vi_warm_start(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                        const float* params, void* workspace, size_t workspace_bytes, int32_t* accepted) {
  return vi_ba_solve_warm(ctx, n_windows, windows, opts, params, 0, workspace, workspace_bytes, accepted);
}

vi_status vi_ba_solve_warm(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                           const float* params, int32_t iters, void* workspace, size_t workspace_bytes,
                           int32_t* accepted) {
  if (!ctx) return VI_EINVAL;
  if (n_windows < 1 || !windows) return fail(ctx, VI_EINVAL, "need at least one window");
  std::vector<WinIn> wins;
  for (int w = 0; w < n_windows; ++w)
    wins.push_back(WinIn{&windows[w].cam, &windows[w].state, &windows[w].edges, windows[w].imu, windows[w].report});
  WarmArgs wa{params, 1, 1};
  warm_canvas(wins, &wa.hq, &wa.wq);
  return run(ctx, wins, opts, iters, workspace, workspace_bytes, &wa, accepted);
}

vi_status vi_warm_features(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts,
                           int32_t hq, int32_t wq, float* feat, int32_t* dims) {
  if (!ctx) return VI_EINVAL;
  if (!feat || !dims) return fail(ctx, VI_EINVAL, "null output");
  vi_status s = warm_check_canvas(ctx, 1, hq, wq);
  if (s != VI_OK) return s;
  std::vector<WinIn> wins;
  s = warm_windows(ctx, n_windows, windows, opts, hq, wq, wins);
  if (s != VI_OK) return s;
  if ((s = warm_begin(ctx)) != VI_OK) return s;
  OptsDev od{opts->n_fixed, opts->use_imu ? 1 : 0, opts->bias_mode == VI_BIAS_FIXED ? 1 : 0, opts->precision, opts->lm_lambda,
             opts->depth_eta, opts->z_min, opts->d_min, 0.0,
             (opts->use_imu && opts->bias_mode == VI_BIAS_GLOBAL) ? 1 : 0};
  launch_warm_features(ctx->priv, ctx->plan, ctx->dplan, od, hq, wq, feat, dims);
  return warm_end(ctx);
}

vi_status vi_warm_forward(vi_ctx* ctx, int32_t n_img, int32_t hq, int32_t wq, const int32_t* dims,
                          const float* params, const float* feat, float* dd, float* db) {
  if (!ctx) return VI_EINVAL;
  vi_status s = warm_check_canvas(ctx, n_img, hq, wq);
  if (s != VI_OK) return s;
  if (!dims || !params || !feat || !dd || !db) return fail(ctx, VI_EINVAL, "null argument");
  if ((s = warm_begin(ctx)) != VI_OK) return s;
  launch_wnet_forward(ctx->priv, n_img, hq, wq, dims, params, feat, nullptr, dd, db);
  return warm_end(ctx);
}

vi_status vi_warm_gradients(vi_ctx* ctx, int32_t n_img, int32_t hq, int32_t wq, const int32_t* dims,
                            const float* params, const float* feat, const float* label_dd, const float* label_db,
                            float n_valid_cells, void* workspace, size_t workspace_bytes, float* grads,
                            float* loss) {
  if (!ctx) return VI_EINVAL;
  vi_status s = warm_check_canvas(ctx, n_img, hq, wq);
  if (s != VI_OK) return s;
  if (!dims || !params || !feat || !label_dd || !label_db || !grads || !loss || !workspace)
    return fail(ctx, VI_EINVAL, "null argument");
  if (!(n_valid_cells >= 1.0f)) return fail(ctx, VI_EINVAL, "n_valid_cells must be >= 1");
  const size_t need = vi_warm_workspace_size(n_img, hq, wq);
  if (workspace_bytes < need)
    return fail(ctx, VI_ENOMEM, "warm-start workspace too small: %zu bytes given, %zu needed", workspace_bytes, need);
  if (((uintptr_t)workspace & 255) != 0) return fail(ctx, VI_EINVAL, "workspace must be 256-byte aligned");
  const size_t n = n_img, cells = (size_t)hq * wq;
  char* b = (char*)workspace;
  void* act = b;                       b += align256(n * 5 * cells * kWC * 2);
  float* dd = (float*)b;               b += align256(n * cells * sizeof(float));
  float* gdd = (float*)b;              b += align256(n * cells * sizeof(float));
  float* db = (float*)b;               b += align256(n * 6 * sizeof(float));
  float* gdb = (float*)b;              b += align256(n * 6 * sizeof(float));
  float* lossv = (float*)b;            b += align256(n * sizeof(float));
  float* partial = (float*)b;
  if ((s = warm_begin(ctx)) != VI_OK) return s;
  launch_wnet_forward(ctx->priv, n_img, hq, wq, dims, params, feat, act, dd, db);
  launch_wnet_backward(ctx->priv, n_img, hq, wq, dims, params, act, dd, db, label_dd, label_db, n_valid_cells, gdd,
                       gdb, lossv, partial, grads);
  std::vector<float> hl(n);
  HIPCHK(ctx, hipMemcpyAsync(hl.data(), lossv, n * sizeof(float), hipMemcpyDeviceToHost, ctx->priv));
  s = warm_end(ctx);
  if (s != VI_OK) return s;
  double tot = 0.0;
  for (float v : hl) tot += v;
  *loss = (float)tot;
  return VI_OK;
}

vi_status vi_warm_adamw(vi_ctx* ctx, float* params, const float* grads, float* m, float* v, int32_t t, float lr,
                        float beta1, float beta2, float eps, float weight_decay) {
  if (!ctx) return VI_EINVAL;
  if (!params || !grads || !m || !v) return fail(ctx, VI_EINVAL, "null argument");
  if (t < 1) return fail(ctx, VI_EINVAL, "step t must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return fail(ctx, VI_EINVAL, "bad AdamW hyper-parameters");
  vi_status s = warm_begin(ctx);
  if (s != VI_OK) return s;
  launch_wnet_adamw(ctx->priv, kWParams, params, grads, m, v, t, lr, beta1, beta2, eps, weight_decay);
  return warm_end(ctx);
}

vi_status vi_warm_apply(vi_ctx* ctx, int32_t n_windows, const vi_window* windows, const vi_opts* opts, int32_t hq,
                        int32_t wq, const float* dd, const float* db) {
  if (!ctx) return VI_EINVAL;
  if (!dd || !db) return fail(ctx, VI_EINVAL, "null argument");
  vi_status s = warm_check_canvas(ctx, 1, hq, wq);
  if (s != VI_OK) return s;
  std::vector<WinIn> wins;
  s = warm_windows(ctx, n_windows, windows, opts, hq, wq, wins);
  if (s != VI_OK) return s;
  if ((s = warm_begin(ctx)) != VI_OK) return s;
  launch_warm_apply(ctx->priv, ctx->plan, ctx->dplan, hq, wq, dd, db, opts->d_min,
                    (opts->use_imu && opts->bias_mode == VI_BIAS_PER_KF) ? 1 : 0);
  return warm_end(ctx);
}

size_t vi_reanchor_workspace_size(int32_t n_kf) { return n_kf > 0 ? align256(reanchor_table_bytes(n_kf)) : 0; }

// host checks shared by both Gaussian-map entry points
static vi_status reanchor_check(vi_ctx* ctx, int32_t n_kf, const double* pose_pre, const double* pose_post,
                                const double* scale_change, const vi_gaussians* g) {
  if (!g || !pose_pre || !pose_post || !scale_change) return fail(ctx, VI_EINVAL, "null argument");
  if (n_kf < 1) return fail(ctx, VI_EINVAL, "need at least one keyframe");
  const int64_t K = g->n;
  if (K < 0 || K > reanchor_max_gaussians()) return fail(ctx, VI_EINVAL, "bad Gaussian count %lld", (long long)K);
  if ((g->cov_in == nullptr) != (g->cov_out == nullptr))
    return fail(ctx, VI_EINVAL, "cov_in and cov_out must both be given or both be NULL");
  if (K > 0 && (!g->anchor || !g->mean_in || !g->mean_out)) return fail(ctx, VI_EINVAL, "null Gaussian array");
  // an output is either its input (in place) or disjoint from every input
  struct Range { const char* p; size_t n; };
  auto overlap = [](Range a, Range b) { return a.p < b.p + b.n && b.p < a.p + a.n; };
  const Range mi{(const char*)g->mean_in, (size_t)K * 12}, mo{(const char*)g->mean_out, (size_t)K * 12};
  const Range ci{(const char*)g->cov_in, g->cov_in ? (size_t)K * 24 : 0};
  const Range co{(const char*)g->cov_out, g->cov_out ? (size_t)K * 24 : 0};
  const Range an{(const char*)g->anchor, (size_t)K * 4};
  if (K > 0) {
    if (mo.p != mi.p && overlap(mo, mi)) return fail(ctx, VI_EINVAL, "mean_out partly overlaps mean_in");
    if (co.n && co.p != ci.p && overlap(co, ci)) return fail(ctx, VI_EINVAL, "cov_out partly overlaps cov_in");
    if (overlap(mo, an) || (co.n && (overlap(co, an) || overlap(co, mi) || overlap(co, mo) || overlap(mo, ci))))
      return fail(ctx, VI_EINVAL, "an output overlaps another array");
  }
  return VI_OK;
}

vi_status vi_gaussian_reanchor(vi_ctx* ctx, int32_t n_kf, const double* pose_pre, const double* pose_post,
                               const double* scale_change, const vi_gaussians* g, void* workspace,
                               size_t workspace_bytes, int32_t* n_rejected) {
  if (!ctx) return VI_EINVAL;
  vi_status s = reanchor_check(ctx, n_kf, pose_pre, pose_post, scale_change, g);
  if (s != VI_OK) return s;
  if (!workspace) return fail(ctx, VI_EINVAL, "null argument");
  if (workspace_bytes < reanchor_table_bytes(n_kf)) return fail(ctx, VI_ENOMEM, "workspace too small");
  if (((uintptr_t)workspace & 15) != 0) return fail(ctx, VI_EINVAL, "workspace must be 16-byte aligned");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  launch_reanchor(ctx->user, n_kf, pose_pre, pose_post, scale_change, workspace, g->n, g->anchor, g->mean_in,
                  g->cov_in, g->mean_out, g->cov_out, n_rejected);
  HIPCHK(ctx, hipGetLastError());
  ctx->err.clear();
  return VI_OK;
}

vi_status vi_gaussian_reanchor_noalloc(vi_ctx* ctx, int32_t n_kf, const double* pose_pre, const double* pose_post,
                                       const double* scale_change, const vi_gaussians* g, int32_t* n_rejected) {
  if (!ctx) return VI_EINVAL;
  vi_status s = reanchor_check(ctx, n_kf, pose_pre, pose_post, scale_change, g);
  if (s != VI_OK) return s;
  if (n_kf > reanchor_noalloc_max_keyframes())
    return fail(ctx, VI_EINVAL, "%d keyframes exceed the allocation-free limit of %d", n_kf,
                reanchor_noalloc_max_keyframes());
  HIPCHK(ctx, hipSetDevice(ctx->device));
  void* table = reanchor_scratch(ctx->device);      // the device address, looked up when the context was created
  if (!table) return fail(ctx, VI_EDEVICE, "no keyframe table on device %d", ctx->device);
  // every row the map kernel reads (0 .. n_kf-1) is rewritten by this call first
  launch_reanchor(ctx->user, n_kf, pose_pre, pose_post, scale_change, table, g->n, g->anchor, g->mean_in,
                  g->cov_in, g->mean_out, g->cov_out, n_rejected);
  HIPCHK(ctx, hipGetLastError());
  ctx->err.clear();
  return VI_OK;
}

vi_status vi_predict_keyframe(vi_ctx* ctx, int32_t n, const double* pose_prev, const double* vel_prev,
                              const double* bias_prev, const vi_preint* imu, const double* gravity, double tau,
                              double* pose_new, double* vel_new, double* bias_new, int32_t* used_imu) {
  if (!ctx) return VI_EINVAL;
  if (n < 0) return fail(ctx, VI_EINVAL, "negative count");
  if (!gravity) return fail(ctx, VI_EINVAL, "null gravity");
  if (!(tau >= 0.0)) return fail(ctx, VI_EINVAL, "tau must be >= 0");
  if (n > 0 && (!pose_prev || !vel_prev || !bias_prev || !imu || !pose_new || !vel_new || !bias_new))
    return fail(ctx, VI_EINVAL, "null argument");
  if (n > 0) {
    struct Range { const char* p; size_t n; };
    auto overlap = [](Range a, Range b) { return a.p < b.p + b.n && b.p < a.p + a.n; };
    const Range in[4] = {{(const char*)pose_prev, 56u * n}, {(const char*)vel_prev, 24u * n},
                         {(const char*)bias_prev, 48u * n}, {(const char*)imu, sizeof(vi_preint) * n}};
    const Range out[4] = {{(const char*)pose_new, 56u * n}, {(const char*)vel_new, 24u * n},
                          {(const char*)bias_new, 48u * n}, {(const char*)used_imu, used_imu ? 4u * n : 0u}};
    for (int o = 0; o < 4; ++o)
      for (int i = 0; i < 4; ++i)
        if (out[o].n && !(o == i && out[o].p == in[i].p) && overlap(out[o], in[i]))
          return fail(ctx, VI_EINVAL, "output %d overlaps input %d", o, i);
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  launch_predict_kf(ctx->user, n, pose_prev, vel_prev, bias_prev, imu, gravity, tau, pose_new, vel_new, bias_new,
                    used_imu);
  HIPCHK(ctx, hipGetLastError());
  ctx->err.clear();
  return VI_OK;
}

size_t vi_inertial_init_workspace_size(int32_t n_problems, const vi_inertial_init* problems) {
  if (n_problems < 1 || !problems) return 0;
  size_t b = align256(sizeof(IInitDesc) * n_problems);
  for (int p = 0; p < n_problems; ++p) {
    const int N = problems[p].n_kf;
    if (N < 2 || N > kIInitMaxKeyframes) return 0;
    b += align256(iinit_whiten_doubles(N) * sizeof(double));
  }
  return b;
}

vi_status vi_inertial_init_solve(vi_ctx* ctx, int32_t n_problems, const vi_inertial_init* problems,
                                 double gravity_z, double lm_lambda, int32_t iters, void* workspace,
                                 size_t workspace_bytes) {
  if (!ctx) return VI_EINVAL;
  if (n_problems < 1 || !problems || !workspace) return fail(ctx, VI_EINVAL, "null argument or no problems");
  if (iters < 0) return fail(ctx, VI_EINVAL, "iters must be >= 0");
  if (!std::isfinite(gravity_z) || gravity_z == 0.0) return fail(ctx, VI_EINVAL, "gravity_z must be finite, non-zero");
  if (!(lm_lambda >= 0.0) || !std::isfinite(lm_lambda)) return fail(ctx, VI_EINVAL, "lm_lambda must be >= 0");
  int max_n = 2;
  for (int p = 0; p < n_problems; ++p) {
    const vi_inertial_init& q = problems[p];
    if (q.n_kf < 2 || q.n_kf > kIInitMaxKeyframes)
      return fail(ctx, VI_EINVAL, "problem %d: n_kf must be in 2..%d", p, kIInitMaxKeyframes);
    if (!q.pose_vis || !q.imu || !q.vel_vis || !q.bias || !q.rot_wg || !q.log_scale)
      return fail(ctx, VI_EINVAL, "problem %d: null array", p);
    max_n = std::max(max_n, (int)q.n_kf);
  }
  const size_t need = vi_inertial_init_workspace_size(n_problems, problems);
  if (workspace_bytes < need) return fail(ctx, VI_ENOMEM, "workspace too small (%zu < %zu)", workspace_bytes, need);
  if (((uintptr_t)workspace & 255) != 0) return fail(ctx, VI_EINVAL, "workspace must be 256-byte aligned");
  std::vector<IInitDesc> h(n_problems);
  char* wp = (char*)workspace + align256(sizeof(IInitDesc) * n_problems);
  for (int p = 0; p < n_problems; ++p) {
    const vi_inertial_init& q = problems[p];
    h[p] = IInitDesc{q.n_kf, 0, q.pose_vis, q.imu, q.vel_vis, q.bias, q.rot_wg, q.log_scale, q.cost, (double*)wp};
    wp += align256(iinit_whiten_doubles(q.n_kf) * sizeof(double));
  }
  vi_status st = ensure_status(ctx, n_problems);
  if (st != VI_OK) return st;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  HIPCHK(ctx, hipMemcpyAsync(workspace, h.data(), sizeof(IInitDesc) * n_problems, hipMemcpyHostToDevice, ctx->priv));
  launch_reset_status(ctx->priv, ctx->status, n_problems);
  launch_inertial_init(ctx->priv, n_problems, (const IInitDesc*)workspace, max_n, gravity_z, lm_lambda, iters,
                       ctx->status);
  HIPCHK(ctx, hipGetLastError());
  std::vector<DevStatus> hs(n_problems);
  HIPCHK(ctx, hipMemcpyAsync(hs.data(), ctx->status, sizeof(DevStatus) * n_problems, hipMemcpyDeviceToHost,
                             ctx->priv));
  HIPCHK(ctx, hipStreamSynchronize(ctx->priv));
  for (int p = 0; p < n_problems; ++p)
    if (hs[p].code != 0)
      return fail(ctx, (vi_status)hs[p].code, "problem %d: %s (stage %d)", p,
                  hs[p].code == VI_ENONFINITE ? "non-finite cost" : "not positive definite", hs[p].detail);
  ctx->err.clear();
  return VI_OK;
}

}  // extern "C"
