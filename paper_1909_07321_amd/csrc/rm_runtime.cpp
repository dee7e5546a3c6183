// rm_runtime.cpp -- host runtime behind include/rm.h: context, resident partial
// waves, workspaces sized against the HBM budget, the staged and fused calls,
// and the serving scheduler (continuous batching over worker streams).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "rm.h"
#include "rm_internal.h"

using namespace rm;

namespace rm {
void launch_setdims(hipStream_t s, int ne, int rows, const int *nopen, int *dims);
void launch_check_inputs(hipStream_t s, int ne, int n, const double *E, const double *ethr, double thr,
                         const double *R, long ldr, long strideR, const double *fg, const double *K, long ldk,
                         long strideK, const int *nopen, int *status);
}  // namespace rm

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Slot {
  hipStream_t stream = nullptr;
  Work w;
};

struct ProfRec {
  hipEvent_t a = nullptr, b = nullptr;
  int stage = 0;
  long energies = 0;
};
const char *const kStages[] = {"rform", "nearpole", "asym", "ksolve", "somega"};
constexpr int NSTAGE = 5;

struct Req {
  uint64_t ticket = 0;
  rm_request rq{};
  std::vector<double> E;
  int next_e = 0, done_e = 0, inflight = 0;
  rm_status err = RM_OK;
  rm_req_stats st{};
  bool admitted = false;
};

}  // namespace

struct rm_ctx {
  int device = 0;
  size_t budget = 0;
  size_t resident = 0;   // bytes of resident partial waves
  size_t work_bytes = 0; // bytes of all workspaces
  hipStream_t stream = nullptr;
  Work work;  // workspace of the synchronous calls
  std::map<int32_t, DevPW> pws;
  int32_t next_id = 1;
  std::string err;
  std::mutex mu;  // guards everything below and the budget counters
  std::condition_variable cv;
  std::deque<Req *> active;  // arrival order
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_ticket = 1;
  int max_queue = 4096;
  std::atomic<int> prof_on{0};
  std::vector<ProfRec> prof;  // guarded by mu
  // rm_run alternates chunks over two streams so that one chunk's K solve
  // overlaps the next chunk's R contraction
  Slot pipe[2];
  hipEvent_t ev_in = nullptr, ev_out[2] = {nullptr, nullptr}, ev_R[2] = {nullptr, nullptr};
};

namespace {

#define HIPCHK(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                            \
      return RM_E_DEVICE;                                                                      \
    }                                                                                          \
  } while (0)

constexpr int MAX_CHUNK = 1024;

size_t per_energy_bytes(int n, int npad, int Mpad) {
  return (size_t)n * 2 * npad * 8      // aug
         + (size_t)n * npad * 8 * 2    // Kw, XK
         + (size_t)Mpad * 12           // D64 + D32
         + (size_t)n * (32 + 9)        // fg, openidx, openpos, openflag
         + (size_t)n * n * 8 / 8       // headroom
         + 64;
}

void free_work(Work &w) {
  void *ptrs[] = {w.E, w.D64, w.D32, w.win, w.status, w.nopen, w.openidx, w.openpos, w.openflag,
                  w.fg, w.aug, w.Kw, w.XK, w.dims, w.omega, w.S, w.ipiv};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  w = Work();
}

// (Re)allocates w for chunks of up to cap energies of partial wave pw.
rm_status ensure_work(rm_ctx *ctx, Work &w, const DevPW &pw, int cap, bool want_S) {
  const int n = pw.n, npad = pw.npad, Mpad = pw.Mpad;
  if (w.cap_e >= cap && w.cap_n >= n && w.cap_npad >= npad && w.cap_M >= Mpad && w.cap_nt >= pw.nt &&
      (!want_S || w.S))
    return RM_OK;
  const int ce = std::max(cap, w.cap_e), cn = std::max(n, w.cap_n), cnp = std::max(npad, w.cap_npad),
            cm = std::max(Mpad, w.cap_M), ct = std::max(pw.nt, w.cap_nt);
  const bool S = want_S || w.S != nullptr;
  size_t need = 0;
  auto sz = [&](size_t b) { need += (b + 255) / 256 * 256; return b; };
  const size_t bE = sz((size_t)ce * 8), bD64 = sz((size_t)ce * cm * 8), bD32 = sz((size_t)ce * cm * 4),
               bwin = sz((size_t)ce * 8), bst = sz((size_t)ce * 4), bno = sz((size_t)ce * 4),
               boi = sz((size_t)ce * cn * 4), bop = sz((size_t)ce * cn * 4), bof = sz((size_t)ce * cn),
               bfg = sz((size_t)ce * cn * 32), baug = sz((size_t)ce * cn * 2 * cnp * 8),
               bK = sz((size_t)ce * cn * cnp * 8), bXK = sz((size_t)ce * cn * cnp * 8),
               bdims = sz((size_t)ce * 8), bom = sz((size_t)ce * ct * ct * 8), bpiv = sz((size_t)ce * cn * 4),
               bS = S ? sz((size_t)ce * cn * cn * 16) : 0;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->resident + ctx->work_bytes - w.bytes + need > ctx->budget) {
      ctx->err = "workspace exceeds the HBM budget";
      return RM_E_NOMEM;
    }
  }
  const size_t old = w.bytes;
  free_work(w);
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->work_bytes -= old;
  }
  HIPCHK(hipMalloc(&w.E, bE));
  HIPCHK(hipMalloc(&w.D64, bD64));
  HIPCHK(hipMalloc(&w.D32, bD32));
  HIPCHK(hipMalloc(&w.win, bwin));
  HIPCHK(hipMalloc(&w.status, bst));
  HIPCHK(hipMalloc(&w.nopen, bno));
  HIPCHK(hipMalloc(&w.openidx, boi));
  HIPCHK(hipMalloc(&w.openpos, bop));
  HIPCHK(hipMalloc(&w.openflag, bof));
  HIPCHK(hipMalloc(&w.fg, bfg));
  HIPCHK(hipMalloc(&w.aug, baug));
  HIPCHK(hipMalloc(&w.Kw, bK));
  HIPCHK(hipMalloc(&w.XK, bXK));
  HIPCHK(hipMalloc(&w.dims, bdims));
  HIPCHK(hipMalloc(&w.omega, bom));
  HIPCHK(hipMalloc(&w.ipiv, bpiv));
  if (S) HIPCHK(hipMalloc(&w.S, bS));
  w.cap_e = ce;
  w.cap_n = cn;
  w.cap_npad = cnp;
  w.cap_M = cm;
  w.cap_nt = ct;
  w.bytes = need;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->work_bytes += need;
  return RM_OK;
}

// Energies per chunk for partial wave pw given `share` bytes of budget.
int chunk_cap(const DevPW &pw, size_t share, int ne) {
  const size_t per = per_energy_bytes(pw.n, pw.npad, pw.Mpad);
  long cap = (long)(share / std::max<size_t>(per, 1));
  cap = std::min<long>(cap, MAX_CHUNK);
  cap = std::min<long>(cap, ((long)ne + EB - 1) / EB * EB);
  if (cap >= EB) cap = cap / EB * EB;
  return (int)std::max<long>(cap, 1);
}

// Layout helpers: all per-energy blocks have rows of the partial wave's n
struct Lay {
  long ldaug, roff, sA, ldk, sK, ldo;
};
Lay layout(const DevPW &pw, const Work &w) {
  Lay L;
  L.ldaug = 2L * w.cap_npad;
  L.roff = w.cap_npad;
  L.sA = (long)pw.n * L.ldaug;
  L.ldk = w.cap_npad;
  L.sK = (long)pw.n * L.ldk;
  L.ldo = pw.n;
  return L;
}

// Brackets the launches issued by `body` with events when profiling is on.
template <typename F>
void timed(rm_ctx *ctx, int stage, long energies, hipStream_t s, F &&body) {
  if (!ctx || !ctx->prof_on.load()) {
    body();
    return;
  }
  ProfRec r;
  r.stage = stage;
  r.energies = energies;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
    body();
    return;
  }
  (void)hipEventRecord(r.a, s);
  body();
  (void)hipEventRecord(r.b, s);
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->prof.push_back(r);
}

void stage_R(rm_ctx *ctx, const DevPW &pw, Work &w, const Lay &L, int m, const rm_opts &o, hipStream_t s) {
  const int split = o.prec == RM_FP32_SPLIT;
  launch_dvec(s, pw, w.E, m, split, o.split_delta, w.D64, w.D32, w.win, w.status);
  timed(ctx, 0, m, s, [&] { launch_rform(s, pw, m, split, w.D64, w.D32, w.aug, L.ldaug, L.sA); });
  if (split) timed(ctx, 1, m, s, [&] { launch_nearpole(s, pw, w.E, m, w.win, w.aug, L.ldaug, L.sA); });
}

void stage_asym(rm_ctx *ctx, const DevPW &pw, Work &w, const Lay &L, int m, const rm_opts &o, hipStream_t s) {
  timed(ctx, 2, m, s, [&] {
    launch_openlist(s, pw, w.E, m, w.nopen, w.openidx, w.openpos, w.openflag, L.ldo);
    launch_asym(s, pw, w.E, m, o.thr_guard, w.fg, w.status);
  });
}

void stage_K(const DevPW &pw, Work &w, const Lay &L, int m, hipStream_t s) {
  launch_setdims(s, m, pw.n, w.nopen, w.dims);
  launch_build(s, pw, m, w.fg, w.nopen, w.openidx, L.ldo, w.aug, L.ldaug, L.sA, L.roff);
  launch_lu_solve(s, m, pw.n, pw.n, w.dims, w.aug, L.ldaug, L.sA, L.roff, w.ipiv, L.ldo, w.status);
  launch_gatherK(s, m, pw.n, w.nopen, w.openidx, L.ldo, w.aug, L.ldaug, L.sA, L.roff, w.Kw, L.ldk, L.sK);
}

void stage_SO(const DevPW &pw, Work &w, const Lay &L, int m, bool want_S, hipStream_t s) {
  // P = 1 + K K and X = P^-1 K on the same batched LU; then XK and Omega
  launch_gemm_sq(s, m, pw.n, w.nopen, w.Kw, L.ldk, L.sK, w.Kw, L.ldk, L.sK, w.aug, L.ldaug, L.sA);
  launch_formP(s, m, pw.n, w.nopen, w.Kw, L.ldk, L.sK, w.aug, L.ldaug, L.sA, L.roff, w.dims);
  launch_lu_solve(s, m, pw.n, pw.n, w.dims, w.aug, L.ldaug, L.sA, L.roff, w.ipiv, L.ldo, w.status);
  launch_gemm_sq(s, m, pw.n, w.nopen, w.aug + L.roff, L.ldaug, L.sA, w.Kw, L.ldk, L.sK, w.XK, L.ldk, L.sK);
  launch_omega(s, pw, m, w.openpos, L.ldo, w.nopen, w.aug + L.roff, L.ldaug, L.sA, w.XK, L.ldk, L.sK, w.omega,
               want_S ? w.S : nullptr);
}

hipMemcpyKind kind_out(const rm_opts &o) { return o.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }
hipMemcpyKind kind_in(const rm_opts &o) { return o.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }

rm_status get_pw(rm_ctx *ctx, int32_t id, DevPW **out) {
  auto it = ctx->pws.find(id);
  if (it == ctx->pws.end()) {
    ctx->err = "unknown partial wave id";
    return RM_E_NOTFOUND;
  }
  *out = &it->second;
  return RM_OK;
}

rm_opts fixed_opts(const rm_opts *o) {
  rm_opts r;
  rm_opts_default(&r);
  if (o) r = *o;
  if (!(r.split_delta > 0)) r.split_delta = 0.05;
  if (!(r.thr_guard >= 0)) r.thr_guard = 1e-10;
  return r;
}

hipStream_t call_stream(rm_ctx *ctx, const rm_opts &o) {
  return (o.device_ptrs && o.stream) ? (hipStream_t)o.stream : ctx->stream;
}

size_t sync_share(rm_ctx *ctx) {
  std::lock_guard<std::mutex> g(ctx->mu);
  const size_t used = ctx->resident + ctx->work_bytes - ctx->work.bytes;
  return ctx->budget > used ? ctx->budget - used : 0;
}

// Which stages a fused chunk runs and where its results go.
struct ChunkOut {
  double *omega = nullptr;   // [m][nt][nt]
  double *K = nullptr;       // [m][n][n]
  int32_t *status = nullptr; // [m]
};

// Runs all stages for energies already in w.E and copies the results out.
// before_R / after_R (optional) order the R contraction against other streams.
rm_status run_chunk(rm_ctx *ctx, const DevPW &pw, Work &w, int m, const rm_opts &o, hipStream_t s,
                    const ChunkOut &out, hipMemcpyKind ko, hipEvent_t before_R = nullptr,
                    hipEvent_t after_R = nullptr) {
  const Lay L = layout(pw, w);
  HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
  if (before_R) HIPCHK(hipStreamWaitEvent(s, before_R, 0));
  stage_R(ctx, pw, w, L, m, o, s);
  if (after_R) HIPCHK(hipEventRecord(after_R, s));
  stage_asym(ctx, pw, w, L, m, o, s);
  timed(ctx, 3, m, s, [&] { stage_K(pw, w, L, m, s); });
  timed(ctx, 4, m, s, [&] { stage_SO(pw, w, L, m, false, s); });
  launch_finalize(s, m, pw.n, pw.nt, w.status, w.omega, w.Kw, L.ldk, L.sK, nullptr);
  HIPCHK(hipMemcpyAsync(out.omega, w.omega, sizeof(double) * m * pw.nt * pw.nt, ko, s));
  if (out.K)
    HIPCHK(hipMemcpy2DAsync(out.K, sizeof(double) * pw.n, w.Kw, sizeof(double) * L.ldk, sizeof(double) * pw.n,
                            (size_t)m * pw.n, ko, s));
  HIPCHK(hipMemcpyAsync(out.status, w.status, sizeof(int) * m, ko, s));
  HIPCHK(hipGetLastError());
  return RM_OK;
}

// ------------------------------------------------------------------ serving
void worker_main(rm_ctx *ctx, Slot *slot) {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    Req *r = nullptr;
    int e0 = 0, m = 0;
    DevPW pw;
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      ctx->cv.wait(lk, [&] {
        if (ctx->stop) return true;
        for (Req *q : ctx->active)
          if (q->next_e < q->rq.ne) return true;
        return false;
      });
      if (ctx->stop) return;
      // continuous batching: the earliest request with work left that has the
      // fewest chunks in flight gets the free slot, so a newly arrived request
      // starts on the next free slot while longer ones keep progressing
      Req *best = nullptr;
      for (Req *q : ctx->active)
        if (q->next_e < q->rq.ne && (!best || q->inflight < best->inflight)) best = q;
      r = best;
      auto it = ctx->pws.find(r->rq.pw_id);
      if (it == ctx->pws.end()) {
        r->err = RM_E_NOTFOUND;
        r->next_e = r->done_e = r->rq.ne;
        r->st.t_done_ns = now_ns();
        ctx->cv.notify_all();
        continue;
      }
      pw = it->second;
      const size_t used = ctx->resident + ctx->work_bytes - slot->w.bytes;
      const size_t share = ctx->budget > used ? (ctx->budget - used) / 1 : 0;
      const int nslots = (int)ctx->slots.size();
      const int cap = chunk_cap(pw, share / std::max(1, nslots - 0), r->rq.ne - r->next_e);
      e0 = r->next_e;
      m = std::min(cap, r->rq.ne - e0);
      r->next_e += m;
      r->inflight++;
      if (!r->admitted) {
        r->admitted = true;
        r->st.t_admit_ns = now_ns();
      }
      if (!r->st.t_start_ns) r->st.t_start_ns = now_ns();
      r->st.nblocks++;
    }
    rm_ctx *c = ctx;
    rm_status st = ensure_work(c, slot->w, pw, m, false);
    if (st == RM_OK) {
      const hipStream_t s = slot->stream;
      rm_opts o = fixed_opts(&r->rq.opts);
      o.device_ptrs = 0;
      ChunkOut out;
      out.omega = r->rq.omega + (size_t)e0 * pw.nt * pw.nt;
      out.K = r->rq.K ? r->rq.K + (size_t)e0 * pw.n * pw.n : nullptr;
      out.status = r->rq.status + e0;
      if (hipMemcpyAsync(slot->w.E, r->E.data() + e0, sizeof(double) * m, hipMemcpyHostToDevice, s) != hipSuccess)
        st = RM_E_DEVICE;
      if (st == RM_OK) st = run_chunk(c, pw, slot->w, m, o, s, out, hipMemcpyDeviceToHost);
      if (st == RM_OK && hipStreamSynchronize(s) != hipSuccess) st = RM_E_DEVICE;
    }
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      r->inflight--;
      r->done_e += m;
      if (st != RM_OK) r->err = st;
      if (r->done_e >= r->rq.ne) r->st.t_done_ns = now_ns();
      ctx->cv.notify_all();
    }
  }
}

}  // namespace

// =================================================================== C ABI
extern "C" {

void rm_opts_default(rm_opts *o) {
  if (!o) return;
  o->prec = RM_FP64;
  o->split_delta = 0.05;
  o->thr_guard = 1e-10;
  o->stream = nullptr;
  o->device_ptrs = 0;
}

rm_status rm_create(int device, size_t hbm_budget_bytes, rm_ctx **out) {
  if (!out) return RM_E_ARG;
  *out = nullptr;
  rm_ctx *ctx = new (std::nothrow) rm_ctx();
  if (!ctx) return RM_E_NOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return RM_E_DEVICE;
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    delete ctx;
    return RM_E_DEVICE;
  }
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  const int nslots = 2;
  for (int i = 0; i < nslots; ++i) {
    auto sl = std::make_unique<Slot>();
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return RM_E_DEVICE;
    }
    ctx->slots.push_back(std::move(sl));
  }
  for (auto &sl : ctx->slots) ctx->workers.emplace_back(worker_main, ctx, sl.get());
  *out = ctx;
  return RM_OK;
}

rm_status rm_destroy(rm_ctx *ctx) {
  if (!ctx) return RM_E_ARG;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->stop = true;
    ctx->cv.notify_all();
  }
  for (auto &t : ctx->workers) t.join();
  (void)hipSetDevice(ctx->device);
  for (auto &sl : ctx->slots) {
    (void)hipStreamSynchronize(sl->stream);
    free_work(sl->w);
    (void)hipStreamDestroy(sl->stream);
  }
  (void)hipStreamSynchronize(ctx->stream);
  free_work(ctx->work);
  for (auto &pp : ctx->pipe) {
    if (pp.stream) {
      (void)hipStreamSynchronize(pp.stream);
      (void)hipStreamDestroy(pp.stream);
    }
    free_work(pp.w);
  }
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  for (auto &ev : ctx->ev_out)
    if (ev) (void)hipEventDestroy(ev);
  for (auto &ev : ctx->ev_R)
    if (ev) (void)hipEventDestroy(ev);
  for (auto &kv : ctx->pws) {
    DevPW &p = kv.second;
    void *ptrs[] = {p.W64, p.W32, p.Ek, p.ethr, p.l, p.target, p.tptr, p.tch};
    for (void *q : ptrs)
      if (q) (void)hipFree(q);
  }
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return RM_OK;
}

const char *rm_last_error(const rm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t rm_pw_footprint(int32_t nchan, int32_t npole) {
  const size_t npad = (size_t)round_up(std::max(nchan, 1), TILE);
  const size_t Mpad = (size_t)round_up(std::max(npole, 1), KC32);
  return Mpad * npad * 12 + Mpad * 8 + (size_t)nchan * 24 + 4096;
}

rm_status rm_pw_upload(rm_ctx *ctx, const rm_pw_desc *d, int32_t *pw_id) {
  if (!ctx || !d || !pw_id) return RM_E_ARG;
  if (d->nchan < 1 || d->npole < 1 || d->ntarget < 1 || !d->e_thr || !d->l || !d->target || !d->Ek || !d->w ||
      !(d->a > 0) || !(d->z >= 0)) {
    ctx->err = "invalid partial-wave descriptor";
    return RM_E_ARG;
  }
  for (int k = 1; k < d->npole; ++k)
    if (!(d->Ek[k] >= d->Ek[k - 1])) {
      ctx->err = "poles must be ascending";
      return RM_E_ARG;
    }
  for (int i = 0; i < d->nchan; ++i)
    if (d->target[i] < 0 || d->target[i] >= d->ntarget || d->l[i] < 0 || d->l[i] > 200) {
      ctx->err = "channel target or l out of range";
      return RM_E_ARG;
    }
  const size_t bytes = rm_pw_footprint(d->nchan, d->npole);
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->resident + ctx->work_bytes + bytes > ctx->budget) {
      ctx->err = "partial wave exceeds the HBM budget";
      return RM_E_NOMEM;
    }
  }
  (void)hipSetDevice(ctx->device);
  DevPW p;
  p.n = d->nchan;
  p.M = d->npole;
  p.nt = d->ntarget;
  p.npad = round_up(p.n, TILE);
  p.Mpad = round_up(p.M, KC32);
  p.a = d->a;
  p.b = d->b;
  p.z = d->z;
  p.g = d->g;
  p.bytes = bytes;
  std::vector<double> W64((size_t)p.Mpad * p.npad, 0.0);
  std::vector<float> W32((size_t)p.Mpad * p.npad, 0.0f);
  for (int k = 0; k < p.M; ++k)
    for (int i = 0; i < p.n; ++i) {
      const double v = d->w[(size_t)k * p.n + i];
      W64[(size_t)k * p.npad + i] = v;
      W32[(size_t)k * p.npad + i] = (float)v;
    }
  std::vector<double> Ek(p.Mpad, 1e300);
  std::memcpy(Ek.data(), d->Ek, sizeof(double) * p.M);
  std::vector<int> tptr(p.nt + 1, 0), tch(p.n);
  for (int i = 0; i < p.n; ++i) tptr[d->target[i] + 1]++;
  for (int t = 0; t < p.nt; ++t) tptr[t + 1] += tptr[t];
  {
    std::vector<int> fill(tptr.begin(), tptr.end() - 1);
    for (int i = 0; i < p.n; ++i) tch[fill[d->target[i]]++] = i;
  }
  HIPCHK(hipMalloc(&p.W64, W64.size() * 8));
  HIPCHK(hipMalloc(&p.W32, W32.size() * 4));
  HIPCHK(hipMalloc(&p.Ek, Ek.size() * 8));
  HIPCHK(hipMalloc(&p.ethr, p.n * 8));
  HIPCHK(hipMalloc(&p.l, p.n * 4));
  HIPCHK(hipMalloc(&p.target, p.n * 4));
  HIPCHK(hipMalloc(&p.tptr, (p.nt + 1) * 4));
  HIPCHK(hipMalloc(&p.tch, p.n * 4));
  HIPCHK(hipMemcpy(p.W64, W64.data(), W64.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.W32, W32.data(), W32.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.Ek, Ek.data(), Ek.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.ethr, d->e_thr, p.n * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.l, d->l, p.n * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.target, d->target, p.n * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.tptr, tptr.data(), (p.nt + 1) * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p.tch, tch.data(), p.n * 4, hipMemcpyHostToDevice));
  std::lock_guard<std::mutex> g(ctx->mu);
  const int32_t id = ctx->next_id++;
  ctx->pws[id] = p;
  ctx->resident += bytes;
  *pw_id = id;
  return RM_OK;
}

rm_status rm_pw_release(rm_ctx *ctx, int32_t pw_id) {
  if (!ctx) return RM_E_ARG;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->pws.find(pw_id);
  if (it == ctx->pws.end()) return RM_E_NOTFOUND;
  for (Req *q : ctx->active)
    if (q->rq.pw_id == pw_id && q->done_e < q->rq.ne) return RM_E_BUSY;
  DevPW p = it->second;
  ctx->pws.erase(it);
  ctx->resident -= p.bytes;
  lk.unlock();
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  void *ptrs[] = {p.W64, p.W32, p.Ek, p.ethr, p.l, p.target, p.tptr, p.tch};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  return RM_OK;
}

rm_status rm_form_R(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts, double *R,
                    int32_t *status) {
  if (!ctx || (ne > 0 && (!E || !R || !status)) || ne < 0) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  const hipStream_t s = call_stream(ctx, o);
  const int cap = chunk_cap(*pw, sync_share(ctx), ne);
  if (rm_status st = ensure_work(ctx, ctx->work, *pw, cap, false)) return st;
  Work &w = ctx->work;
  const Lay L = layout(*pw, w);
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    HIPCHK(hipMemcpyAsync(w.E, E + e0, sizeof(double) * m, kind_in(o), s));
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    stage_R(ctx, *pw, w, L, m, o, s);
    launch_nanfill_R(s, m, pw->n, w.status, w.aug, L.ldaug, L.sA);
    HIPCHK(hipMemcpy2DAsync(R + (size_t)e0 * pw->n * pw->n, sizeof(double) * pw->n, w.aug,
                            sizeof(double) * L.ldaug, sizeof(double) * pw->n, (size_t)m * pw->n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(s));
  return RM_OK;
}

rm_status rm_asymptotic(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts, double *fg,
                        int8_t *open, int32_t *nopen, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !fg || !open || !nopen || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  const hipStream_t s = call_stream(ctx, o);
  const int cap = chunk_cap(*pw, sync_share(ctx), ne);
  if (rm_status st = ensure_work(ctx, ctx->work, *pw, cap, false)) return st;
  Work &w = ctx->work;
  const Lay L = layout(*pw, w);
  const int n = pw->n;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    HIPCHK(hipMemcpyAsync(w.E, E + e0, sizeof(double) * m, kind_in(o), s));
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    stage_asym(ctx, *pw, w, L, m, o, s);
    HIPCHK(hipMemcpyAsync(fg + (size_t)e0 * n * 4, w.fg, sizeof(double) * m * n * 4, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(open + (size_t)e0 * n, w.openflag, (size_t)m * n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(nopen + e0, w.nopen, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(s));
  return RM_OK;
}

rm_status rm_solve_K(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const double *R, const double *fg,
                     const rm_opts *opts, double *K, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !R || !fg || !K || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  const hipStream_t s = call_stream(ctx, o);
  const int cap = chunk_cap(*pw, sync_share(ctx), ne);
  if (rm_status st = ensure_work(ctx, ctx->work, *pw, cap, false)) return st;
  Work &w = ctx->work;
  const Lay L = layout(*pw, w);
  const int n = pw->n;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    HIPCHK(hipMemcpyAsync(w.E, E + e0, sizeof(double) * m, kind_in(o), s));
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    HIPCHK(hipMemcpy2DAsync(w.aug, sizeof(double) * L.ldaug, R + (size_t)e0 * n * n, sizeof(double) * n,
                            sizeof(double) * n, (size_t)m * n, kind_in(o), s));
    HIPCHK(hipMemcpyAsync(w.fg, fg + (size_t)e0 * n * 4, sizeof(double) * m * n * 4, kind_in(o), s));
    launch_dvec(s, *pw, w.E, m, 0, 0.0, w.D64, w.D32, w.win, w.status);  // pole flags
    launch_openlist(s, *pw, w.E, m, w.nopen, w.openidx, w.openpos, w.openflag, L.ldo);
    launch_check_inputs(s, m, n, w.E, pw->ethr, o.thr_guard, w.aug, L.ldaug, L.sA, w.fg, nullptr, 0, 0, w.nopen,
                        w.status);
    stage_K(*pw, w, L, m, s);
    launch_finalize(s, m, n, 0, w.status, nullptr, w.Kw, L.ldk, L.sK, nullptr);
    HIPCHK(hipMemcpy2DAsync(K + (size_t)e0 * n * n, sizeof(double) * n, w.Kw, sizeof(double) * L.ldk,
                            sizeof(double) * n, (size_t)m * n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(s));
  return RM_OK;
}

rm_status rm_collision_strengths(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const double *K,
                                 const rm_opts *opts, double *omega, double *S, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !K || !omega || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  const hipStream_t s = call_stream(ctx, o);
  const int cap = chunk_cap(*pw, sync_share(ctx), ne);
  if (rm_status st = ensure_work(ctx, ctx->work, *pw, cap, S != nullptr)) return st;
  Work &w = ctx->work;
  const Lay L = layout(*pw, w);
  const int n = pw->n, nt = pw->nt;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    HIPCHK(hipMemcpyAsync(w.E, E + e0, sizeof(double) * m, kind_in(o), s));
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    HIPCHK(hipMemcpy2DAsync(w.Kw, sizeof(double) * L.ldk, K + (size_t)e0 * n * n, sizeof(double) * n,
                            sizeof(double) * n, (size_t)m * n, kind_in(o), s));
    launch_openlist(s, *pw, w.E, m, w.nopen, w.openidx, w.openpos, w.openflag, L.ldo);
    launch_check_inputs(s, m, n, w.E, pw->ethr, o.thr_guard, nullptr, 0, 0, nullptr, w.Kw, L.ldk, L.sK, w.nopen,
                        w.status);
    stage_SO(*pw, w, L, m, S != nullptr, s);
    launch_finalize(s, m, n, nt, w.status, w.omega, nullptr, 0, 0, S ? w.S : nullptr);
    HIPCHK(hipMemcpyAsync(omega + (size_t)e0 * nt * nt, w.omega, sizeof(double) * m * nt * nt, kind_out(o), s));
    if (S) HIPCHK(hipMemcpyAsync(S + (size_t)e0 * n * n * 2, w.S, sizeof(double) * m * n * n * 2, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(s));
  return RM_OK;
}

rm_status rm_run(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts, double *omega,
                 double *K, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !omega || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  const hipStream_t user = call_stream(ctx, o);
  if (!ctx->ev_in) {
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipEventCreateWithFlags(&ctx->ev_out[i], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ctx->ev_R[i], hipEventDisableTiming));
      HIPCHK(hipStreamCreateWithFlags(&ctx->pipe[i].stream, hipStreamNonBlocking));
    }
  }
  size_t share;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t used = ctx->resident + ctx->work_bytes - ctx->pipe[0].w.bytes - ctx->pipe[1].w.bytes;
    share = ctx->budget > used ? (ctx->budget - used) / 2 : 0;
  }
  // Chunks of up to 256 energies alternate over the two streams.  The R
  // contractions are chained across the streams (each waits for the previous
  // chunk's), so chunk k+1's compute-bound contraction overlaps chunk k's
  // latency-bound K solve instead of competing with chunk k's contraction.
  // The LU panel runs one workgroup per energy, so its cost grows with the
  // number of chunks rather than with their size; 256 fills the CUs.
  int cap = std::min(chunk_cap(*pw, share, ne), 256);
  if (ne > 2 * EB && cap * 2 > ne) cap = std::max(EB, (ne + 2 * EB - 1) / (2 * EB) * EB);
  const int nuse = ne > cap ? 2 : 1;
  for (int i = 0; i < nuse; ++i)
    if (rm_status st = ensure_work(ctx, ctx->pipe[i].w, *pw, cap, false)) return st;
  // the internal streams start after the caller's prior work on its stream
  HIPCHK(hipEventRecord(ctx->ev_in, user));
  for (int i = 0; i < nuse; ++i) HIPCHK(hipStreamWaitEvent(ctx->pipe[i].stream, ctx->ev_in, 0));
  int k = 0;
  for (int e0 = 0; e0 < ne; e0 += cap, ++k) {
    Slot &sl = ctx->pipe[k % nuse];
    const int m = std::min(cap, ne - e0);
    HIPCHK(hipMemcpyAsync(sl.w.E, E + e0, sizeof(double) * m, kind_in(o), sl.stream));
    ChunkOut out;
    out.omega = omega + (size_t)e0 * pw->nt * pw->nt;
    out.K = K ? K + (size_t)e0 * pw->n * pw->n : nullptr;
    out.status = status + e0;
    hipEvent_t prevR = k > 0 && nuse > 1 ? ctx->ev_R[(k - 1) % 2] : nullptr;
    if (rm_status st = run_chunk(ctx, *pw, sl.w, m, o, sl.stream, out, kind_out(o), prevR, ctx->ev_R[k % 2]))
      return st;
  }
  // and the caller's stream continues after both
  for (int i = 0; i < nuse; ++i) {
    HIPCHK(hipEventRecord(ctx->ev_out[i], ctx->pipe[i].stream));
    HIPCHK(hipStreamWaitEvent(user, ctx->ev_out[i], 0));
  }
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(user));
  return RM_OK;
}

rm_status rm_submit(rm_ctx *ctx, const rm_request *req, uint64_t *ticket) {
  if (!ctx || !req || !ticket || req->ne < 0 || (req->ne > 0 && (!req->E || !req->omega || !req->status)) ||
      req->opts.device_ptrs)
    return RM_E_ARG;
  auto r = std::make_unique<Req>();
  r->rq = *req;
  r->E.assign(req->E, req->E + req->ne);
  r->st.t_arrive_ns = now_ns();
  std::lock_guard<std::mutex> g(ctx->mu);
  if ((int)ctx->active.size() >= ctx->max_queue) return RM_E_BUSY;
  if (!ctx->pws.count(req->pw_id)) {
    ctx->err = "unknown partial wave id";
    return RM_E_NOTFOUND;
  }
  r->ticket = ctx->next_ticket++;
  *ticket = r->ticket;
  if (req->ne == 0) r->st.t_done_ns = r->st.t_arrive_ns;
  ctx->active.push_back(r.get());
  ctx->reqs[r->ticket] = std::move(r);
  ctx->cv.notify_all();
  return RM_OK;
}

rm_status rm_poll(rm_ctx *ctx, uint64_t ticket, rm_req_stats *st) {
  if (!ctx) return RM_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->reqs.find(ticket);
  if (it == ctx->reqs.end()) return RM_E_NOTFOUND;
  Req *r = it->second.get();
  if (r->done_e < r->rq.ne || r->inflight > 0) return RM_PENDING;
  if (st) *st = r->st;
  const rm_status res = r->err;
  ctx->active.erase(std::remove(ctx->active.begin(), ctx->active.end(), r), ctx->active.end());
  ctx->reqs.erase(it);
  return res;
}

rm_status rm_drain(rm_ctx *ctx) {
  if (!ctx) return RM_E_ARG;
  std::unique_lock<std::mutex> lk(ctx->mu);
  ctx->cv.wait(lk, [&] {
    for (Req *q : ctx->active)
      if (q->done_e < q->rq.ne || q->inflight > 0) return false;
    return true;
  });
  return RM_OK;
}

rm_status rm_prof_enable(rm_ctx *ctx, int32_t on) {
  if (!ctx) return RM_E_ARG;
  ctx->prof_on.store(on ? 1 : 0);
  return RM_OK;
}

rm_status rm_prof_read(rm_ctx *ctx, const char *stage, double *total_ms, int64_t *launches, int64_t *energies) {
  if (!ctx || !stage) return RM_E_ARG;
  int id = -1;
  for (int i = 0; i < NSTAGE; ++i)
    if (!std::strcmp(stage, kStages[i])) id = i;
  if (id < 0) return RM_E_NOTFOUND;
  std::vector<ProfRec> mine;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<ProfRec> rest;
    for (auto &r : ctx->prof) (r.stage == id ? mine : rest).push_back(r);
    ctx->prof.swap(rest);
  }
  double ms = 0;
  long e = 0;
  rm_status st = RM_OK;
  for (auto &r : mine) {
    float t = 0;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) st = RM_E_DEVICE;
    ms += t;
    e += r.energies;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = (int64_t)mine.size();
  if (energies) *energies = e;
  return st;
}

}  // extern "C"
