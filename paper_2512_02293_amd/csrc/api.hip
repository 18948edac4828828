// C ABI of the visual-inertial step library: argument validation, the
// per-shape plan (index tables derived from the frame graph), the workspace
// carve, HIP-graph capture of whole solves, and the report.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vi_internal.h"

using namespace vi;

struct GraphKey {
  int32_t N, E, H, W, iters;
  vi_opts opts;
  double cam[7];
  const void* ptrs[12];
  uint64_t plan_version;
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

struct vi_ctx {
  int device = 0;
  hipStream_t user = nullptr;      // caller's stream
  hipStream_t priv = nullptr;      // private stream (graph capture and execution)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::string err;
  DevStatus* status = nullptr;     // device
  int32_t* d_off = nullptr;        // device CSR for imu_preintegrate
  size_t d_off_cap = 0;
  // plan
  Plan plan;
  bool have_plan = false;
  uint64_t plan_version = 0;
  int32_t* d_plan = nullptr;
  size_t d_plan_cap = 0;
  DevPlan dplan{};
  int attr_kmax = -1;
  // graph cache
  bool have_graph = false;
  GraphKey gkey{};
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

vi_status build_plan(vi_ctx* ctx, int N, const vi_edges* ed, int H, int W, Plan& P) {
  const int E = ed->n_edges;
  P = Plan();
  P.N = N; P.E = E; P.H = H; P.W = W; P.HW = H * W; P.F = N - 1;
  P.n = 15 * N;
  P.npad = (P.n + kCholNB - 1) / kCholNB * kCholNB;
  P.nblk = P.npad / kCholNB;
  P.nkr_vis = (P.HW + kVisBlock - 1) / kVisBlock;
  P.nkr_gram = (P.HW + kGramRange - 1) / kGramRange;
  P.ii.assign(ed->ii, ed->ii + E);
  P.jj.assign(ed->jj, ed->jj + E);
  std::vector<int> cnt(N, 0);
  std::vector<char> seen;
  for (int e = 0; e < E; ++e) {
    const int i = P.ii[e], j = P.jj[e];
    if (i < 0 || i >= N || j < 0 || j >= N)
      return fail(ctx, VI_EINVAL, "edge %d: keyframe index out of range (%d -> %d, N = %d)", e, i, j, N);
    if (i == j) return fail(ctx, VI_EINVAL, "edge %d: source equals target (%d)", e, i);
    cnt[i]++;
  }
  P.src_off.assign(N + 1, 0);
  for (int i = 0; i < N; ++i) P.src_off[i + 1] = P.src_off[i] + cnt[i];
  P.src_edges.assign(E, 0);
  P.edge_slot.assign(E, 0);
  std::vector<int> fill(N, 0);
  for (int e = 0; e < E; ++e) {
    const int i = P.ii[e];
    P.edge_slot[e] = fill[i];
    P.src_edges[P.src_off[i] + fill[i]++] = e;
  }
  P.kmax = 0;
  for (int i = 0; i < N; ++i) P.kmax = std::max(P.kmax, cnt[i]);
  if (P.kmax > kMaxOutDegree)
    return fail(ctx, VI_EUNSUPPORTED, "a keyframe has %d outgoing edges; at most %d are supported", P.kmax,
                kMaxOutDegree);
  // duplicate pairs
  for (int i = 0; i < N; ++i) {
    std::vector<int> t;
    for (int s = P.src_off[i]; s < P.src_off[i + 1]; ++s) t.push_back(P.jj[P.src_edges[s]]);
    std::sort(t.begin(), t.end());
    for (size_t a = 1; a < t.size(); ++a)
      if (t[a] == t[a - 1]) return fail(ctx, VI_EINVAL, "duplicate edge %d -> %d", i, t[a]);
  }
  P.gram_off.assign(N, 0); P.q_off.assign(N, 0); P.z_off.assign(N, 0); P.zb_off.assign(N, 0);
  P.tiles.assign(N, 0);
  size_t go = 0, qo = 0, zo = 0, zbo = 0;
  for (int i = 0; i < N; ++i) {
    const int k = cnt[i];
    const int T = k > 0 ? (6 * k + 16) / 16 : 0;
    P.tiles[i] = T * (T + 1) / 2;
    P.gram_off[i] = (int32_t)go;
    P.q_off[i] = (int32_t)qo;
    P.z_off[i] = (int32_t)zo;
    P.zb_off[i] = (int32_t)zbo;
    go += (size_t)P.tiles[i] * 256 * P.nkr_gram;
    if (k > 0) qo += (size_t)(6 * k + 1) * (6 * k + 1);
    zo += (size_t)(k + 1) * (k + 1) * 36;
    zbo += (size_t)6 * (k + 1);
  }
  if (go > INT32_MAX || qo > INT32_MAX || zo > INT32_MAX)
    return fail(ctx, VI_EUNSUPPORTED, "problem too large for 32-bit plan offsets");
  P.gram_size = go; P.q_size = qo; P.z_size = zo; P.zb_size = zbo;
  P.L_size = (size_t)6 * E * P.HW;
  // gather lists of the reduced assembly: pose block (a, b) <- Z blocks of every
  // source whose touched set {i} U targets(i) contains both a and b
  std::vector<std::vector<std::pair<int, int>>> items((size_t)N * N);
  for (int i = 0; i < N; ++i) {
    const int k = cnt[i];
    std::vector<int> T(1, i);
    for (int s = P.src_off[i]; s < P.src_off[i + 1]; ++s) T.push_back(P.jj[P.src_edges[s]]);
    for (int ta = 0; ta <= k; ++ta)
      for (int tb = 0; tb <= k; ++tb)
        items[(size_t)T[ta] * N + T[tb]].push_back(
            {P.z_off[i] + (ta * (k + 1) + tb) * 36, P.zb_off[i] + 6 * ta});
  }
  P.pair_off.assign((size_t)N * N + 1, 0);
  for (size_t q = 0; q < (size_t)N * N; ++q) P.pair_off[q + 1] = P.pair_off[q] + (int32_t)items[q].size();
  P.n_pairs = P.pair_off.back();
  P.pair_z.resize(std::max<size_t>(P.n_pairs, 1));
  P.pair_zb.resize(std::max<size_t>(P.n_pairs, 1));
  for (size_t q = 0; q < (size_t)N * N; ++q)
    for (size_t u = 0; u < items[q].size(); ++u) {
      P.pair_z[P.pair_off[q] + u] = items[q][u].first;
      P.pair_zb[P.pair_off[q] + u] = items[q][u].second;
    }
  return VI_OK;
}

vi_status upload_plan(vi_ctx* ctx) {
  const Plan& P = ctx->plan;
  const std::vector<int32_t>* parts[] = {&P.ii, &P.jj, &P.src_off, &P.src_edges, &P.edge_slot,
                                         &P.gram_off, &P.q_off, &P.z_off, &P.zb_off, &P.tiles,
                                         &P.pair_off, &P.pair_z, &P.pair_zb};
  size_t total = 0;
  for (auto* v : parts) total += align256(v->size() * sizeof(int32_t));
  if (total > ctx->d_plan_cap) {
    if (ctx->d_plan) HIPCHK(ctx, hipFree(ctx->d_plan));
    ctx->d_plan = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&ctx->d_plan, total));
    ctx->d_plan_cap = total;
  }
  std::vector<char> host(total, 0);
  size_t off = 0;
  const int32_t* dptr[13];
  int idx = 0;
  for (auto* v : parts) {
    std::memcpy(host.data() + off, v->data(), v->size() * sizeof(int32_t));
    dptr[idx++] = (const int32_t*)((char*)ctx->d_plan + off);
    off += align256(v->size() * sizeof(int32_t));
  }
  HIPCHK(ctx, hipMemcpy(ctx->d_plan, host.data(), total, hipMemcpyHostToDevice));
  DevPlan& D = ctx->dplan;
  D.ii = dptr[0]; D.jj = dptr[1]; D.src_off = dptr[2]; D.src_edges = dptr[3]; D.edge_slot = dptr[4];
  D.gram_off = dptr[5]; D.q_off = dptr[6]; D.z_off = dptr[7]; D.zb_off = dptr[8]; D.tiles = dptr[9];
  D.pair_off = dptr[10]; D.pair_z = dptr[11]; D.pair_zb = dptr[12];
  return VI_OK;
}

vi_status ensure_plan(vi_ctx* ctx, int N, const vi_edges* ed, int H, int W) {
  const int E = ed->n_edges;
  if (ctx->have_plan) {
    const Plan& P = ctx->plan;
    if (P.N == N && P.E == E && P.H == H && P.W == W &&
        std::memcmp(P.ii.data(), ed->ii, sizeof(int32_t) * E) == 0 &&
        std::memcmp(P.jj.data(), ed->jj, sizeof(int32_t) * E) == 0)
      return VI_OK;
  }
  Plan P;
  vi_status s = build_plan(ctx, N, ed, H, W, P);
  if (s != VI_OK) return s;
  ctx->plan = std::move(P);
  ctx->have_plan = false;
  s = upload_plan(ctx);
  if (s != VI_OK) return s;
  ctx->have_plan = true;
  ctx->plan_version++;
  if (ctx->plan.kmax > ctx->attr_kmax) {
    step_set_attributes(ctx->plan.kmax);
    ctx->attr_kmax = ctx->plan.kmax;
  }
  return VI_OK;
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
  const size_t N = P.N, E = P.E, HW = P.HW, F = std::max(P.F, 0);
  w.Rw = c.take<double>(N * 9);
  w.rel = c.take<double>(E * 12);
  w.L = c.take<double>(P.L_size);
  w.Cd = c.take<double>(N * HW);
  w.wd = c.take<double>(N * HW);
  w.hpart = c.take<double>(E * P.nkr_vis * 32);
  w.vcost = c.take<double>(N * P.nkr_vis * 2);
  w.gpart = c.take<double>(P.gram_size);
  w.Z = c.take<double>(P.z_size);
  w.ZB = c.take<double>(P.zb_size);
  w.ZV = c.take<double>(P.zb_size);
  w.Lam = c.take<double>(F * 225);
  w.Hf = c.take<double>(F * 900);
  w.gf = c.take<double>(F * 30);
  w.icost = c.take<double>(F);
  w.A = c.take<double>((size_t)(P.npad + kCholNB) * P.npad);
  w.Linv = c.take<double>((size_t)P.nblk * kCholNB * kCholNB);
  w.x = c.take<double>(P.npad);
  w.dd = c.take<double>(N * HW);
  w.trace = c.take<double>(2 * (kMaxIters + 1));
  if (bytes) *bytes = c.off;
  return w;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

vi_status check_common(vi_ctx* ctx, const vi_camera* cam, const vi_state* st, const vi_edges* ed,
                       const vi_preint* imu, const vi_opts* o) {
  if (!ctx) return VI_EINVAL;
  if (!cam || !st || !ed || !o) return fail(ctx, VI_EINVAL, "null argument");
  if (!finite_pos(cam->fx) || !finite_pos(cam->fy) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(ctx, VI_EINVAL, "intrinsics must be finite with fx, fy > 0");
  if (cam->H <= 0 || cam->W <= 0 || (int64_t)cam->H * cam->W > (1 << 24))
    return fail(ctx, VI_EINVAL, "bad map size %d x %d", cam->H, cam->W);
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(cam->gravity[k])) return fail(ctx, VI_EINVAL, "gravity must be finite");
  if (st->n_kf < 2) return fail(ctx, VI_EINVAL, "need at least 2 keyframes (got %d)", st->n_kf);
  if (st->n_kf > 4096) return fail(ctx, VI_EUNSUPPORTED, "at most 4096 keyframes are supported");
  if (!st->pose || !st->vel || !st->bias || !st->invdepth) return fail(ctx, VI_EINVAL, "null state array");
  if (ed->n_edges < 1) return fail(ctx, VI_EINVAL, "need at least one edge");
  if (!ed->ii || !ed->jj || !ed->target || !ed->weight) return fail(ctx, VI_EINVAL, "null edge array");
  if (o->n_fixed < 0 || o->n_fixed > st->n_kf) return fail(ctx, VI_EINVAL, "n_fixed out of range");
  if (o->reserved != 0) return fail(ctx, VI_EINVAL, "opts.reserved must be 0");
  if (!(o->lm_lambda >= 0.0) || !(o->depth_eta >= 0.0) || !std::isfinite(o->lm_lambda) ||
      !std::isfinite(o->depth_eta))
    return fail(ctx, VI_EINVAL, "damping must be finite and >= 0");
  if (!std::isfinite(o->z_min) || !(o->d_min >= 0.0) || !std::isfinite(o->d_min))
    return fail(ctx, VI_EINVAL, "z_min must be finite and d_min finite and >= 0");
  if (o->use_imu && !imu) return fail(ctx, VI_EINVAL, "use_imu set but no IMU factors given");
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

vi_status run(vi_ctx* ctx, const vi_camera* cam, vi_state* st, const vi_edges* ed, const vi_preint* imu,
              const vi_opts* o, int iters, void* workspace, size_t workspace_bytes, vi_report* rep) {
  vi_status s = check_common(ctx, cam, st, ed, imu, o);
  if (s != VI_OK) return s;
  if (iters < 1 || iters > kMaxIters) return fail(ctx, VI_EINVAL, "iters must be in [1, %d]", kMaxIters);
  if (!workspace) return fail(ctx, VI_EINVAL, "null workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(ctx, VI_EINVAL, "workspace must be 256-byte aligned");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  s = ensure_plan(ctx, st->n_kf, ed, cam->H, cam->W);
  if (s != VI_OK) return s;
  const Plan& P = ctx->plan;
  size_t need = 0;
  do_carve(P, nullptr, &need);
  if (workspace_bytes < need)
    return fail(ctx, VI_ENOMEM, "workspace too small: %zu bytes given, %zu needed", workspace_bytes, need);
  Work w = do_carve(P, workspace, nullptr);
  CamDev cd{cam->fx, cam->fy, cam->cx, cam->cy, cam->H, cam->W, {cam->gravity[0], cam->gravity[1], cam->gravity[2]}};
  OptsDev od{o->n_fixed, o->use_imu ? 1 : 0, o->bias_fixed ? 1 : 0, o->lm_lambda, o->depth_eta, o->z_min, o->d_min};
  double* rep_dxi = rep ? rep->dxi : nullptr;
  double* rep_dd = rep ? rep->dd : nullptr;
  const bool timing = rep && rep->stage_ms;

  // order after the caller's pending work
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  hipStream_t sp = ctx->priv;

  auto enqueue = [&](StageMark mark, void* user) {
    launch_reset_status(sp, ctx->status);
    if (od.use_imu) launch_imu_info(sp, P.F, imu, w.Lam, ctx->status);
    for (int it = 0; it < iters; ++it)
      launch_step(sp, P, ctx->dplan, w, cd, od, *st, ed->target, ed->weight, imu, it, rep_dxi, rep_dd,
                  ctx->status, mark, user);
    launch_final_cost(sp, P, ctx->dplan, w, cd, od, *st, ed->target, ed->weight, imu, iters, ctx->status);
  };

  if (timing) {
    // eager launches with events between stages, summed over the steps
    std::vector<hipEvent_t> ev(kNumStages + 1);
    for (auto& e : ev) HIPCHK(ctx, hipEventCreate(&e));
    std::vector<double> acc(VI_NUM_STAGES, 0.0);
    launch_reset_status(sp, ctx->status);
    if (od.use_imu) launch_imu_info(sp, P.F, imu, w.Lam, ctx->status);
    TimingUser tu{sp, ev.data()};
    for (int it = 0; it < iters; ++it) {
      HIPCHK(ctx, hipEventRecord(ev[0], sp));
      launch_step(sp, P, ctx->dplan, w, cd, od, *st, ed->target, ed->weight, imu, it, rep_dxi, rep_dd,
                  ctx->status, mark_event, &tu);
      HIPCHK(ctx, hipEventSynchronize(ev[kNumStages]));
      for (int k = 0; k < kNumStages; ++k) {
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
        acc[k] += ms;
      }
    }
    HIPCHK(ctx, hipEventRecord(ev[0], sp));
    launch_final_cost(sp, P, ctx->dplan, w, cd, od, *st, ed->target, ed->weight, imu, iters, ctx->status);
    HIPCHK(ctx, hipEventRecord(ev[1], sp));
    HIPCHK(ctx, hipEventSynchronize(ev[1]));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ev[0], ev[1]));
    acc[kNumStages] += ms;
    for (int k = 0; k < VI_NUM_STAGES; ++k) rep->stage_ms[k] = (float)acc[k];
    for (auto& e : ev) (void)hipEventDestroy(e);
  } else {
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    key.N = P.N; key.E = P.E; key.H = P.H; key.W = P.W; key.iters = iters;
    key.opts = *o;
    key.cam[0] = cam->fx; key.cam[1] = cam->fy; key.cam[2] = cam->cx; key.cam[3] = cam->cy;
    key.cam[4] = cam->gravity[0]; key.cam[5] = cam->gravity[1]; key.cam[6] = cam->gravity[2];
    const void* ptrs[12] = {st->pose, st->vel, st->bias, st->invdepth, ed->target, ed->weight, imu,
                            workspace, rep_dxi, rep_dd, nullptr, nullptr};
    std::memcpy(key.ptrs, ptrs, sizeof(ptrs));
    key.plan_version = ctx->plan_version;
    if (!ctx->have_graph || !(key == ctx->gkey)) {
      if (ctx->exec) { (void)hipGraphExecDestroy(ctx->exec); ctx->exec = nullptr; }
      if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
      ctx->have_graph = false;
      HIPCHK(ctx, hipStreamBeginCapture(sp, hipStreamCaptureModeThreadLocal));
      enqueue(nullptr, nullptr);
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
  DevStatus hs;
  std::vector<double> trace(2 * (iters + 1));
  HIPCHK(ctx, hipMemcpyAsync(&hs, ctx->status, sizeof(DevStatus), hipMemcpyDeviceToHost, sp));
  HIPCHK(ctx, hipMemcpyAsync(trace.data(), w.trace, sizeof(double) * trace.size(), hipMemcpyDeviceToHost, sp));
  HIPCHK(ctx, hipStreamSynchronize(sp));
  if (rep) {
    rep->iters_done = hs.iters;
    const int last = std::max(0, std::min(hs.iters, iters) - 1);
    rep->cost_before = trace[2 * last];
    rep->n_valid = (int64_t)trace[2 * last + 1];
    rep->cost_after = trace[2 * iters];
    if (rep->costs)
      for (int t = 0; t <= iters; ++t) rep->costs[t] = trace[2 * t];
  }
  if (hs.code == VI_ENOTPD)
    return fail(ctx, VI_ENOTPD, "reduced system not positive definite at coordinate %d (step %d)", hs.detail,
                hs.iters);
  if (hs.code == VI_ENONFINITE)
    return fail(ctx, VI_ENONFINITE, "non-finite reduced system at coordinate %d (step %d)", hs.detail, hs.iters);
  if (hs.code != 0) return fail(ctx, (vi_status)hs.code, "device error %d (detail %d)", hs.code, hs.detail);
  ctx->err.clear();
  return VI_OK;
}

}  // namespace

extern "C" {

const char* vi_version(void) { return "vi-ba-mi355x 0.1 (gfx950, fp64)"; }

vi_status vi_ctx_create(int32_t device, void* stream, vi_ctx** out) {
  if (!out) return VI_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return VI_EDEVICE;
  vi_ctx* c = new vi_ctx();
  c->device = device;
  c->user = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&c->priv, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipMalloc((void**)&c->status, sizeof(DevStatus)) != hipSuccess) {
    vi_ctx_destroy(c);
    return VI_EDEVICE;
  }
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
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->priv) (void)hipStreamDestroy(c->priv);
  delete c;
}

vi_status vi_ctx_set_stream(vi_ctx* ctx, void* stream) {
  if (!ctx) return VI_EINVAL;
  ctx->user = (hipStream_t)stream;
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
    if (ctx->d_off) HIPCHK(ctx, hipFree(ctx->d_off));
    ctx->d_off = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&ctx->d_off, bytes));
    ctx->d_off_cap = bytes;
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->priv, ctx->ev_in, 0));
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_off, off, bytes, hipMemcpyHostToDevice, ctx->priv));
  launch_reset_status(ctx->priv, ctx->status);
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

size_t vi_workspace_size(const vi_camera* cam, int32_t n_kf, const vi_edges* edges, const vi_opts* opts) {
  (void)opts;
  if (!cam || !edges || n_kf < 2 || edges->n_edges < 1 || !edges->ii || !edges->jj) return 0;
  Plan P;
  if (build_plan(nullptr, n_kf, edges, cam->H, cam->W, P) != VI_OK) return 0;
  size_t b = 0;
  do_carve(P, nullptr, &b);
  return b;
}

vi_status vi_ba_step(vi_ctx* ctx, const vi_camera* cam, vi_state* state, const vi_edges* edges,
                     const vi_preint* imu, const vi_opts* opts, void* workspace, size_t workspace_bytes,
                     vi_report* report) {
  return run(ctx, cam, state, edges, imu, opts, 1, workspace, workspace_bytes, report);
}

vi_status vi_ba_solve(vi_ctx* ctx, const vi_camera* cam, vi_state* state, const vi_edges* edges,
                      const vi_preint* imu, const vi_opts* opts, int32_t iters, void* workspace,
                      size_t workspace_bytes, vi_report* report) {
  return run(ctx, cam, state, edges, imu, opts, iters, workspace, workspace_bytes, report);
}

}  // extern "C"
