// rm_runtime.cpp -- host runtime behind include/rm.h: context, resident partial
// waves, workspaces sized against the HBM budget, chunk planning, the staged,
// fused and batched calls, and the serving scheduler.
//
// Every call is reduced to a list of segments (one partial wave, a block of
// energies, where its outputs go).  Segments are cut into chunks; a chunk may
// hold energies of several partial waves.  Per chunk the device gets a table
// of the partial waves involved, each energy's table slot, and a task list for
// the persistent R contraction (tasks ordered by cost, largest first); every
// later stage reads its energy's partial wave through the slot, so the whole
// chunk runs as one launch sequence whatever its mix of channel counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cctype>
#include <cstdlib>
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
#include "k_mqdt.h"
#include "rm_internal.h"

using namespace rm;

// Workspace of rm_run_noalloc: a file-scope device array.  Every device the
// library runs on holds its own copy until the process ends; in host code its
// name is only a stand-in, so its device address is resolved once per device
// (with that device current, by rm_create) and only that address is used.
static __device__ __align__(256) unsigned char scratch[RM_NOALLOC_SCRATCH_BYTES];

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Pinned host staging of one workspace: chunk plans are written here and copied
// to the device on the workspace's stream; `ready` marks when the copies of the
// previous chunk that used this staging have run.
struct Staging {
  double *E = nullptr;
  int *pwi = nullptr;
  DevPW *tab = nullptr;
  RTask *tasks = nullptr;
  long *off = nullptr;  // [2][cap_e + 1]: Omega and K pack offsets
  int cap_e = 0, cap_tab = 0, cap_tasks = 0;
  hipEvent_t ready = nullptr;
};

// HIP graphs of one slot's chunk pipeline, one per stage group: the captured
// launch sequence of the group for the last chunk shape (key), replayed while
// the shape repeats.  Replaced executables wait in `retired` until an event
// recorded after their last launch has completed.
constexpr int NGROUP = 9;
struct GraphCache {
  std::string key[NGROUP];
  hipGraphExec_t exec[NGROUP] = {};
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> retired;
  std::atomic<long> captures{0}, replays{0};
};

struct Slot {
  hipStream_t stream = nullptr;
  Work w;
  Staging h;
  GraphCache g;
  bool direct = false;  // launch directly, never through captured graphs
};

struct ProfRec {
  hipEvent_t a = nullptr, b = nullptr;
  int stage = 0;
  long energies = 0;
  double cost = 0, open = 0;  // chunk records: model flops and summed open fraction n_o / n
};
const char *const kStages[] = {"rform", "nearpole", "asym", "ksolve", "somega", "chunk", "prop"};
constexpr int NSTAGE = 7;
constexpr int STAGE_CHUNK = 5;
constexpr int STAGE_PROP = 6;

struct Req {
  uint64_t ticket = 0;
  rm_request rq{};
  std::vector<double> E;
  int next_e = 0, done_e = 0, inflight = 0;
  rm_status err = RM_OK;
  rm_req_stats st{};
  bool admitted = false;
};

// One partial wave's block of energies and where its results go.
struct Seg {
  const DevPW *pw = nullptr;
  const double *E = nullptr;  // host or device, see the call's opts
  int ne = 0;
  double *omega = nullptr;    // [ne][nt][nt]
  double *K = nullptr;        // [ne][n][n] or null
  int32_t *status = nullptr;  // [ne]
};

// The part [e_begin, e_begin + m) of segment `seg`, placed at chunk energy e0.
struct Part {
  int seg, e_begin, m, e0, slot;
};

struct Plan {
  std::vector<Part> parts;
  std::vector<const DevPW *> slots;
  Lay L;
  int ntasks = 0, maxtiles = 0;
  int split = 0;
  std::vector<int> pshape;  // R tile shape of each part
  RQueues q[NRTMAX]{};      // R task queues of each tile shape
};

}  // namespace

struct rm_ctx {
  int device = 0;
  int ncu = 256;
  std::string arch;  // device architecture name, for the tile cache
  size_t budget = 0;
  size_t resident = 0;    // bytes of resident partial waves
  size_t work_bytes = 0;  // bytes of all workspaces
  hipStream_t stream = nullptr;
  Slot sync;  // workspace of the staged calls
  std::map<int32_t, DevPW> pws;
  int32_t next_id = 1;
  std::string err;
  std::mutex mu;  // guards the maps, queues and budget counters
  std::condition_variable cv;
  std::deque<Req *> active;  // arrival order
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<std::unique_ptr<Slot>> slots;  // serving workers
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_ticket = 1;
  int max_queue = 4096;
  std::atomic<int> prof_on{0};
  std::vector<ProfRec> prof;  // guarded by mu
  std::map<const DevPW *, std::vector<double>> hthr;  // host copies of channel thresholds; guarded by mu
  int tile[2][NBUCKET] = {};  // R tile shape per (split, size bucket); guarded by mu
  std::atomic<int> graphs{1};  // chunk pipelines run as captured HIP graphs
  const void *mem_waiter = nullptr;  // serving slot waiting for the other slots' workspaces; guarded by mu
  // rm_run / rm_run_batch alternate chunks over two streams; the R
  // contractions are chained across them so that one chunk's K solve overlaps
  // the next chunk's contraction
  Slot pipe[2];
  // rm_run_noalloc: its slot (staging allocated by rm_create, workspace carved
  // from the device's scratch array) and the lock that serialises its calls
  Slot na;
  std::mutex na_mu;
  char *scratch = nullptr;
  // Numerov grid of the coupled waves: points between a and r1, and steps
  // between recombinations
  std::atomic<int> prop_npts{3201}, prop_stab{64};
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
// workspace bytes of a chunk beyond its per-energy blocks (wave tables, queue
// heads, the 256-byte rounding of each buffer), an upper bound for the
// admission test
constexpr size_t kChunkFixedBytes = 16u << 20;
constexpr double TUNE_MARGIN = 0.03;

// npc: padded channels of the largest coupled wave (0 if none)
size_t per_energy_bytes(int n, int npad, int Mpad, int nt, int npc = 0) {
  return (size_t)PROP_NMAT * 2 * npc * npc * 8  // propagation matrices
         + (size_t)n * 2 * npad * 8  // aug
         + (size_t)n * npad * 8 * 3  // Kw, gre, gim
         + (size_t)n * n * 8         // packed outputs
         + (size_t)Mpad * 12         // D64 + D32
         + (size_t)n * (32 + 17)     // fg, openidx, openpos, colpos, openflag, ipiv
         + (size_t)nt * nt * 8       // Omega
         + BPERM * 4 + NBU * NBU * 8 + 128
         // R tasks: a part of m energies has ceil(m / eb) <= m batches of
         // t (t + 1) / 2 tiles, most for the 16-channel tile
         + (size_t)((n + 15) / 16) * ((n + 15) / 16 + 1) / 2 * sizeof(RTask);
}

// One buffer of a chunk workspace: where its pointer goes and its byte size.
struct WorkBuf {
  void **ptr;
  size_t bytes;
};

// Every buffer of a workspace with capacities (energies, channels, padded
// channels, padded poles, targets, table slots, R tasks), in one fixed order;
// the pointers are those of w.  With S the S-matrix output buffer is included,
// with cpc > 0 the propagation matrices of coupled waves of up to cpc padded
// channels.
std::vector<WorkBuf> work_buffers(Work &w, int ce, int cn, int cnp, int cm, int ct, int ctab, int ctask, bool S,
                                  int cpc = 0) {
  auto b = [](size_t x) { return std::max<size_t>(x, 8); };
  const size_t E = (size_t)ce;
  const size_t bidx = b(E * cn * 4), bK = b(E * cn * cnp * 8), boff = b((E + 1) * 8);
  std::vector<WorkBuf> v = {
      {(void **)&w.E, b(E * 8)},           {(void **)&w.pwi, b(E * 4)},
      {(void **)&w.tab, b((size_t)ctab * sizeof(DevPW))},
      {(void **)&w.tasks, b((size_t)ctask * sizeof(RTask))},
      {(void **)&w.counter, 256},          {(void **)&w.D64, b(E * cm * 8)},
      {(void **)&w.D32, b(E * cm * 4)},    {(void **)&w.win, b(E * 8)},
      {(void **)&w.status, b(E * 4)},      {(void **)&w.nopen, b(E * 4)},
      {(void **)&w.openidx, bidx},         {(void **)&w.openpos, bidx},
      {(void **)&w.colpos, bidx},          {(void **)&w.ipiv, bidx},
      {(void **)&w.bperm, b(E * BPERM * 4)}, {(void **)&w.linv, b(E * NBU * NBU * 8)},
      {(void **)&w.openflag, b(E * cn)},   {(void **)&w.fg, b(E * cn * 32)},
      {(void **)&w.aug, b(E * cn * 2 * cnp * 8)},
      {(void **)&w.Kw, bK},                {(void **)&w.gre, bK},
      {(void **)&w.gim, bK},               {(void **)&w.dims, b(E * 8)},
      {(void **)&w.omega, b(E * ct * ct * 8)},
      {(void **)&w.pack, b(E * std::max((size_t)cn * cn, (size_t)ct * ct) * 8)},
      {(void **)&w.pack_off, 2 * boff}};
  if (S) v.push_back({(void **)&w.S, b(E * cn * cn * 16)});
  if (cpc) v.push_back({(void **)&w.pz, b(E * PROP_NMAT * 2 * cpc * cpc * 8)});
  w.cap_npc = cpc;
  w.cap_e = ce;
  w.cap_n = cn;
  w.cap_npad = cnp;
  w.cap_M = cm;
  w.cap_nt = ct;
  w.cap_tab = ctab;
  w.cap_tasks = ctask;
  return v;
}

// Device bytes of the buffers, each rounded up to 256.
size_t work_bytes(const std::vector<WorkBuf> &v) {
  size_t t = 0;
  for (const WorkBuf &b : v) t += (b.bytes + 255) / 256 * 256;
  return t;
}

void free_work(Work &w) {
  void *ptrs[] = {w.E, w.pwi, w.tab, w.tasks, w.counter, w.D64, w.D32, w.win, w.status, w.nopen, w.openidx,
                  w.openpos, w.colpos, w.openflag, w.fg, w.aug, w.Kw, w.gre, w.gim, w.dims, w.ipiv, w.bperm, w.linv, w.omega, w.pack, w.pack_off,
                  w.S, w.pz};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  w = Work();
}

void free_staging(Staging &h) {
  void *ptrs[] = {h.E, h.pwi, h.tab, h.tasks, h.off};
  for (void *p : ptrs)
    if (p) (void)hipHostFree(p);
  if (h.ready) (void)hipEventDestroy(h.ready);
  h = Staging();
}

// (Re)allocates a slot for chunks with layout L, ntab partial waves and ntasks
// R tasks.  Grows only.
rm_status ensure_slot(rm_ctx *ctx, Slot &sl, const Lay &L, int ntab, int ntasks, bool want_S) {
  Work &w = sl.w;
  Staging &h = sl.h;
  if (!h.ready) HIPCHK(hipEventCreateWithFlags(&h.ready, hipEventDisableTiming));
  const bool fits = w.cap_e >= L.ne && w.cap_n >= L.nmax && w.cap_npad >= L.npadmax && w.cap_M >= L.Mpadmax &&
                    w.cap_nt >= L.ntmax && w.cap_tab >= ntab && w.cap_tasks >= ntasks && (!want_S || w.S) &&
                    w.cap_npc >= L.npadc;
  if (!fits) {
    const int ce = std::max(L.ne, w.cap_e), cn = std::max(L.nmax, w.cap_n),
              cnp = std::max(L.npadmax, w.cap_npad), cm = std::max(L.Mpadmax, w.cap_M),
              ct = std::max(L.ntmax, w.cap_nt), ctab = std::max(ntab, w.cap_tab),
              ctask = std::max(ntasks, w.cap_tasks), cpc = std::max(L.npadc, w.cap_npc);
    const bool S = want_S || w.S != nullptr;
    Work nw;
    const std::vector<WorkBuf> bufs = work_buffers(nw, ce, cn, cnp, cm, ct, ctab, ctask, S, cpc);
    const size_t need = work_bytes(bufs);
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      if (ctx->resident + ctx->work_bytes - w.bytes + need > ctx->budget) {
        ctx->err = "workspace exceeds the HBM budget";
        return RM_E_NOMEM;
      }
    }
    HIPCHK(hipStreamSynchronize(sl.stream));
    const size_t old = w.bytes;
    free_work(w);
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->work_bytes -= old;
    }
    for (const WorkBuf &b : bufs) {
      const hipError_t e = hipMalloc(b.ptr, b.bytes);
      if (e != hipSuccess) {
        *b.ptr = nullptr;
        free_work(nw);  // the buffers allocated before this one
        ctx->err = std::string("hipMalloc (chunk workspace): ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? RM_E_NOMEM : RM_E_DEVICE;
      }
    }
    w = nw;
    w.cap_e = ce;
    w.cap_n = cn;
    w.cap_npad = cnp;
    w.cap_M = cm;
    w.cap_nt = ct;
    w.cap_tab = ctab;
    w.cap_tasks = ctask;
    w.cap_npc = cpc;
    w.bytes = need;
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->work_bytes += need;
  }
  if (h.cap_e < L.ne || h.cap_tab < ntab || h.cap_tasks < ntasks) {
    HIPCHK(hipStreamSynchronize(sl.stream));
    const int ce = std::max(L.ne, h.cap_e), ctab = std::max(ntab, h.cap_tab), ctask = std::max(ntasks, h.cap_tasks);
    hipEvent_t ev = h.ready;
    h.ready = nullptr;
    free_staging(h);
    h.ready = ev;
    HIPCHK(hipHostMalloc((void **)&h.E, sizeof(double) * ce, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&h.pwi, sizeof(int) * ce, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&h.tab, sizeof(DevPW) * ctab, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&h.tasks, sizeof(RTask) * std::max(ctask, 1), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&h.off, sizeof(long) * 2 * (ce + 1), hipHostMallocDefault));
    h.cap_e = ce;
    h.cap_tab = ctab;
    h.cap_tasks = ctask;
  }
  return RM_OK;
}

// Strides of a chunk holding the given partial waves.
Lay make_layout(const std::vector<const DevPW *> &slots, int ne) {
  Lay L;
  L.ne = ne;
  for (const DevPW *p : slots) {
    L.nmax = std::max(L.nmax, p->n);
    L.npadmax = std::max(L.npadmax, p->npad);
    L.Mpadmax = std::max(L.Mpadmax, p->Mpad);
    L.ntmax = std::max(L.ntmax, p->nt);
    if (p->lamax) {
      L.npadc = std::max(L.npadc, p->npad);
      L.lamc = std::max(L.lamc, p->lamax);
    }
  }
  L.zrb = L.npadc / TILE;
  L.sZ = 2L * L.npadc * L.npadc;
  L.ldD = L.Mpadmax;
  L.ldaug = 2L * L.npadmax;
  L.roff = L.npadmax;
  L.sA = (long)L.nmax * L.ldaug;
  L.ldk = L.npadmax;
  L.sK = (long)L.nmax * L.ldk;
  L.ldo = L.nmax;
  L.sOm = (long)L.ntmax * L.ntmax;
  return L;
}

// Energies per chunk for a chunk whose largest members are (n, npad, Mpad, nt),
// given `share` bytes of budget.
int chunk_cap(int n, int npad, int Mpad, int nt, size_t share, int limit, int npc = 0) {
  const size_t per = per_energy_bytes(n, npad, Mpad, nt, npc);
  long cap = (long)(share / std::max<size_t>(per, 1));
  cap = std::min<long>(cap, limit);
  if (cap >= EB) cap = cap / EB * EB;
  return (int)std::max<long>(cap, 1);
}

// Fills the slot's staging for the chunk (energies, slots, tasks, pack offsets)
// and queues its copies to the device.
rm_status upload_plan(rm_ctx *ctx, Slot &sl, Plan &P, const std::vector<Seg> &segs, const rm_opts &o, bool want_K) {
  Staging &h = sl.h;
  Work &w = sl.w;
  const Lay &L = P.L;
  // the previous chunk on this slot must have consumed the staging
  HIPCHK(hipEventSynchronize(h.ready));
  for (const Part &pt : P.parts)
    for (int i = 0; i < pt.m; ++i) h.pwi[pt.e0 + i] = pt.slot;
  for (size_t i = 0; i < P.slots.size(); ++i) h.tab[i] = *P.slots[i];
  // R tasks: energy batches of <= eb energies of one partial wave times its
  // tiles, per tile shape.  All batches of one (part, tile) form a unit; units
  // go, longest first, to the XCD queue with the least work so far, and each
  // queue lists its units in that order.  The shapes' task lists follow each
  // other in `tasks`.
  struct Unit {
    int part, tile;
    double cost;
  };
  int nt = 0;
  for (int sh = 0; sh < NRTMAX; ++sh) {
    std::vector<Unit> units;
    const RTile rt = rtile(P.split, std::min(sh, nrtile(P.split) - 1));
    for (size_t pi = 0; pi < P.parts.size(); ++pi) {
      if (sh >= nrtile(P.split) || P.pshape[pi] != sh) continue;
      const Part &pt = P.parts[pi];
      const DevPW *p = P.slots[pt.slot];
      const int tl = (p->n + 16 * rt.tm - 1) / (16 * rt.tm);
      const double c = (double)p->Mpad * ((pt.m + rt.eb - 1) / rt.eb) * rt.tm * rt.tm;
      for (int t = 0; t < tl * (tl + 1) / 2; ++t) units.push_back(Unit{(int)pi, t, c});
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.cost > b.cost; });
    std::vector<std::vector<int>> qu(NQ);
    double load[NQ] = {0};
    for (size_t u = 0; u < units.size(); ++u) {
      const int q = (int)(std::min_element(load, load + NQ) - load);
      qu[q].push_back((int)u);
      load[q] += units[u].cost;
    }
    for (int q = 0; q < NQ; ++q) {
      P.q[sh].start[q] = nt;
      for (int u : qu[q]) {
        const Part &pt = P.parts[units[u].part];
        for (int b = 0; b < pt.m; b += rt.eb)
          h.tasks[nt++] = RTask{pt.slot, pt.e0 + b, std::min(rt.eb, pt.m - b), units[u].tile};
      }
    }
    P.q[sh].start[NQ] = nt;
  }
  P.ntasks = nt;
  long om = 0, kk = 0;
  for (const Part &pt : P.parts) {
    const DevPW *p = P.slots[pt.slot];
    for (int i = 0; i < pt.m; ++i) {
      h.off[pt.e0 + i] = om;
      h.off[L.ne + 1 + pt.e0 + i] = kk;
      om += (long)p->nt * p->nt;
      kk += (long)p->n * p->n;
    }
  }
  h.off[L.ne] = om;
  h.off[2 * L.ne + 1] = kk;
  const hipStream_t s = sl.stream;
  HIPCHK(hipMemcpyAsync(w.pwi, h.pwi, sizeof(int) * L.ne, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w.tab, h.tab, sizeof(DevPW) * P.slots.size(), hipMemcpyHostToDevice, s));
  if (nt) HIPCHK(hipMemcpyAsync(w.tasks, h.tasks, sizeof(RTask) * nt, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w.pack_off, h.off, sizeof(long) * 2 * (L.ne + 1), hipMemcpyHostToDevice, s));
  // energies: contiguous per part
  if (o.device_ptrs) {
    for (const Part &pt : P.parts)
      HIPCHK(hipMemcpyAsync(w.E + pt.e0, segs[pt.seg].E + pt.e_begin, sizeof(double) * pt.m,
                            hipMemcpyDeviceToDevice, s));
  } else {
    for (const Part &pt : P.parts)
      std::memcpy(h.E + pt.e0, segs[pt.seg].E + pt.e_begin, sizeof(double) * pt.m);
    HIPCHK(hipMemcpyAsync(w.E, h.E, sizeof(double) * L.ne, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipEventRecord(h.ready, s));
  (void)want_K;
  return RM_OK;
}

// Opens a profile record (an event recorded on s) when profiling is on.
bool prof_begin(rm_ctx *ctx, int stage, long energies, hipStream_t s, ProfRec &r) {
  if (!ctx || !ctx->prof_on.load()) return false;
  r.stage = stage;
  r.energies = energies;
  if (hipEventCreate(&r.a) != hipSuccess) return false;
  if (hipEventCreate(&r.b) != hipSuccess) {
    (void)hipEventDestroy(r.a);
    return false;
  }
  (void)hipEventRecord(r.a, s);
  return true;
}

// Closes a record opened by prof_begin and files it.
void prof_end(rm_ctx *ctx, hipStream_t s, ProfRec &r) {
  (void)hipEventRecord(r.b, s);
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->prof.push_back(r);
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

void stage_R(rm_ctx *ctx, const Plan &P, Work &w, const rm_opts &o, hipStream_t s) {
  const Lay &L = P.L;
  const int split = o.prec == RM_FP32_SPLIT;
  launch_dvec(s, L, w.tab, w.pwi, w.E, split, o.split_delta, w.D64, w.D32, w.win, w.status);
  timed(ctx, 0, L.ne, s, [&] {
    for (int sh = 0; sh < nrtile(split); ++sh)
      launch_rform(s, L, split, sh, w.tab, w.tasks, P.q[sh], w.counter + NQ * sh, ctx->ncu, w.D64, w.D32, w.aug);
  });
  if (split)
    timed(ctx, 1, L.ne, s, [&] { launch_nearpole(s, L, P.maxtiles, w.tab, w.pwi, w.E, w.win, w.aug); });
}

void stage_asym(rm_ctx *ctx, const Plan &P, Work &w, const rm_opts &o, hipStream_t s) {
  const Lay &L = P.L;
  timed(ctx, 2, L.ne, s, [&] {
    launch_openlist(s, L, w.tab, w.pwi, w.E, w.nopen, w.openidx, w.openpos, w.colpos, w.openflag);
    launch_asym(s, L, w.tab, w.pwi, w.E, o.thr_guard, w.fg, w.status);
  });
}

void stage_K(const Plan &P, Work &w, hipStream_t s) {
  const Lay &L = P.L;
  launch_setdims(s, L, w.tab, w.pwi, w.nopen, w.dims);
  launch_build(s, L, w.tab, w.pwi, w.fg, w.nopen, w.openidx, w.colpos, w.aug);
  launch_prop_assemble(s, L, w.tab, w.pwi, w.nopen, w.pz, w.aug, w.gre, w.gim);  // coupled energies
  launch_lu_solve(s, L.ne, L.nmax, L.nmax, w.dims, w.aug, L.ldaug, L.sA, L.roff, w.ipiv, L.ldo, w.bperm, w.linv, 1,
                  w.status);
  launch_gatherK(s, L, w.tab, w.pwi, w.nopen, w.aug, w.Kw, w.dims);
}

void stage_SO(const Plan &P, Work &w, bool want_S, hipStream_t s) {
  // M = 1 - iK from K (symmetrised copy); M^-1 by a complex symmetric Cholesky
  // factorisation; then Omega (and S) from M^-1
  const Lay &L = P.L;
  launch_zs_setup(s, L, w.nopen, w.Kw, w.aug, w.gre, w.gim, w.dims);
  launch_zs_inverse(s, L, w.dims, w.aug, w.gre, w.gim, w.linv, w.status);
  launch_omega(s, L, w.tab, w.pwi, w.openpos, w.nopen, w.aug, w.aug + L.roff, w.omega, want_S ? w.S : nullptr);
}

hipMemcpyKind kind_out(const rm_opts &o) { return o.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }
hipMemcpyKind kind_in(const rm_opts &o) { return o.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }

rm_status get_pw(rm_ctx *ctx, int32_t id, const DevPW **out) {
  std::lock_guard<std::mutex> g(ctx->mu);
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

// Budget available to `sl` (its own workspace counts as available).
size_t free_share(rm_ctx *ctx, const Slot &sl) {
  std::lock_guard<std::mutex> g(ctx->mu);
  const size_t used = ctx->resident + ctx->work_bytes - sl.w.bytes;
  return ctx->budget > used ? ctx->budget - used : 0;
}

// Builds the plan for parts already chosen (slots assigned here).
void finish_plan(Plan &P, const std::vector<Seg> &segs, int ne) {
  std::vector<const DevPW *> slots;
  for (Part &pt : P.parts) {
    const DevPW *p = segs[pt.seg].pw;
    int s = -1;
    for (size_t i = 0; i < slots.size(); ++i)
      if (slots[i] == p) s = (int)i;
    if (s < 0) {
      s = (int)slots.size();
      slots.push_back(p);
    }
    pt.slot = s;
  }
  P.slots = slots;
  P.L = make_layout(slots, ne);
  P.maxtiles = 0;
  for (const DevPW *p : slots) {
    const int tl = p->npad / TILE;
    P.maxtiles = std::max(P.maxtiles, tl * (tl + 1) / 2);
  }
}

// Picks each part's R tile shape (the context's choice for its precision and
// size bucket, or `force` if it is >= 0) and returns the number of R tasks of
// the chunk.
int plan_tasks(rm_ctx *ctx, Plan &P, const rm_opts &o, int force = -1) {
  P.split = o.prec == RM_FP32_SPLIT;
  int tile[NBUCKET];
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    std::copy(ctx->tile[P.split], ctx->tile[P.split] + NBUCKET, tile);
  }
  P.pshape.assign(P.parts.size(), 0);
  int nt = 0;
  for (size_t i = 0; i < P.parts.size(); ++i) {
    const Part &pt = P.parts[i];
    const int n = P.slots[pt.slot]->n;
    P.pshape[i] = force >= 0 ? force : tile[size_bucket(n)];
    const RTile rt = rtile(P.split, P.pshape[i]);
    const int tl = (n + 16 * rt.tm - 1) / (16 * rt.tm);
    nt += (pt.m + rt.eb - 1) / rt.eb * (tl * (tl + 1) / 2);
  }
  return nt;
}

// Everything the captured launch sequence of a chunk depends on: sizes and
// strides, workspace addresses, task queues and options (the kernels read the
// chunk's tables, tasks and energies from the workspace, so chunks with equal
// keys replay the same graphs).
std::string chunk_key(rm_ctx *ctx, const Plan &P, const Work &w, const rm_opts &o, bool want_K) {
  std::string k;
  auto add = [&](const auto &v) { k.append(reinterpret_cast<const char *>(&v), sizeof v); };
  const Lay &L = P.L;
  for (long v : {(long)L.ne, (long)L.nmax, (long)L.npadmax, (long)L.Mpadmax, (long)L.ntmax, L.ldD, L.ldaug, L.roff,
                 L.sA, L.ldk, L.sK, L.ldo, L.sOm, (long)L.npadc, (long)L.lamc, L.zrb, L.sZ, (long)ctx->prop_npts.load(),
                 (long)ctx->prop_stab.load()})
    add(v);
  for (const void *p : {(const void *)w.E, (const void *)w.pwi, (const void *)w.tab, (const void *)w.tasks,
                        (const void *)w.counter, (const void *)w.D64, (const void *)w.D32, (const void *)w.win,
                        (const void *)w.status, (const void *)w.nopen, (const void *)w.openidx,
                        (const void *)w.openpos, (const void *)w.colpos, (const void *)w.openflag,
                        (const void *)w.fg, (const void *)w.aug, (const void *)w.Kw, (const void *)w.gre, (const void *)w.gim,
                        (const void *)w.dims, (const void *)w.ipiv, (const void *)w.bperm, (const void *)w.linv,
                        (const void *)w.omega, (const void *)w.pack, (const void *)w.pack_off, (const void *)w.pz})
    add(p);
  for (int sh = 0; sh < NRTMAX; ++sh) add(P.q[sh]);
  add(P.maxtiles);
  add(P.split);
  add(o.split_delta);
  add(o.thr_guard);
  add(want_K);
  add(ctx->ncu);
  return k;
}

// Runs the launches of `body` on the slot's stream: directly, or (graph mode)
// as the executable graph of stage group `grp`, captured from body when the
// slot has none for this key and replayed otherwise.
template <typename F>
rm_status launch_group(rm_ctx *ctx, Slot &sl, int grp, const std::string &key, F &&body) {
  const hipStream_t s = sl.stream;
  if (!ctx->graphs.load() || sl.direct) {
    body();
    HIPCHK(hipGetLastError());
    return RM_OK;
  }
  GraphCache &gc = sl.g;
  for (size_t i = 0; i < gc.retired.size();) {
    if (hipEventQuery(gc.retired[i].second) == hipSuccess) {
      (void)hipGraphExecDestroy(gc.retired[i].first);
      (void)hipEventDestroy(gc.retired[i].second);
      gc.retired[i] = gc.retired.back();
      gc.retired.pop_back();
    } else {
      ++i;
    }
  }
  (void)hipGetLastError();  // a query of a pending event is not an error
  if (!gc.exec[grp] || gc.key[grp] != key) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    body();
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (ec != hipSuccess || !g) {
      ctx->err = std::string("graph capture: ") + hipGetErrorString(ec);
      return RM_E_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      ctx->err = std::string("graph instantiation: ") + hipGetErrorString(ei);
      return RM_E_DEVICE;
    }
    if (gc.exec[grp]) {
      hipEvent_t ev = nullptr;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HIPCHK(hipEventRecord(ev, s));
      gc.retired.emplace_back(gc.exec[grp], ev);
    }
    gc.exec[grp] = ex;
    gc.key[grp] = key;
    ++gc.captures;
  } else {
    ++gc.replays;
  }
  HIPCHK(hipGraphLaunch(gc.exec[grp], s));
  return RM_OK;
}

// Runs every stage of a planned chunk (inputs already uploaded) and copies
// each part's results to its segment.  before_R / after_R (optional) order the
// R contraction against other streams.
rm_status run_chunk(rm_ctx *ctx, const Plan &P, Slot &sl, const std::vector<Seg> &segs, const rm_opts &o,
                    hipMemcpyKind ko, hipEvent_t before_R = nullptr, hipEvent_t after_R = nullptr) {
  const Lay &L = P.L;
  Work &w = sl.w;
  const hipStream_t s = sl.stream;
  const int split = o.prec == RM_FP32_SPLIT;
  bool want_K = false;
  for (const Part &pt : P.parts) want_K |= segs[pt.seg].K != nullptr;
  const std::string key = chunk_key(ctx, P, w, o, want_K);
  rm_status st = RM_OK;
  auto group = [&](int g, auto &&body) {
    if (st == RM_OK) st = launch_group(ctx, sl, g, key, body);
  };
  // chunk record (profiling only): model flops of the chunk's energies, per
  // energy n(n+1)M (R) + (2/3)n^3 + n^2 n_o (K solve) + 4 n_o^3 (S/Omega)
  double cost = 0, open = 0;
  if (ctx->prof_on.load()) {
    if (o.device_ptrs) {  // the chunk's energies came from device memory: bring them to the staging copy
      HIPCHK(hipMemcpyAsync(sl.h.E, w.E, sizeof(double) * L.ne, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    for (const Part &pt : P.parts) {
      const DevPW &pw = *segs[pt.seg].pw;
      auto it = ctx->hthr.find(&pw);
      const double n = pw.n, M = pw.M;
      for (int e = 0; e < pt.m; ++e) {
        double no = 0;
        if (it != ctx->hthr.end())
          for (double t : it->second) no += sl.h.E[pt.e0 + e] - t > 0.0;
        cost += n * (n + 1) * M + 2.0 / 3.0 * n * n * n + n * n * no + 4.0 * no * no * no;
        open += no / n;
      }
    }
  }
  ProfRec chunk_rec;
  const bool chunk_timed = prof_begin(ctx, STAGE_CHUNK, L.ne, s, chunk_rec);
  timed(ctx, 2, L.ne, s, [&] {
    group(0, [&] {
      launch_fill_int(s, w.status, L.ne, 0);
      launch_openlist(s, L, w.tab, w.pwi, w.E, w.nopen, w.openidx, w.openpos, w.colpos, w.openflag);
      launch_asym(s, L, w.tab, w.pwi, w.E, o.thr_guard, w.fg, w.status);
    });
  });
  if (L.npadc)
    timed(ctx, STAGE_PROP, L.ne, s, [&] {
      group(8, [&] {
        launch_prop(s, L, ctx->prop_npts.load(), ctx->prop_stab.load(), w.tab, w.pwi, w.E, w.fg, w.nopen, w.openidx, w.colpos, w.pz,
                    w.status);
      });
    });
  if (before_R) HIPCHK(hipStreamWaitEvent(s, before_R, 0));
  group(1, [&] { launch_dvec(s, L, w.tab, w.pwi, w.E, split, o.split_delta, w.D64, w.D32, w.win, w.status); });
  timed(ctx, 0, L.ne, s, [&] {
    group(2, [&] {
      for (int sh = 0; sh < nrtile(split); ++sh)
        launch_rform(s, L, split, sh, w.tab, w.tasks, P.q[sh], w.counter + NQ * sh, ctx->ncu, w.D64, w.D32, w.aug);
    });
  });
  if (split) timed(ctx, 1, L.ne, s, [&] {
      group(3, [&] { launch_nearpole(s, L, P.maxtiles, w.tab, w.pwi, w.E, w.win, w.aug); });
    });
  if (after_R) HIPCHK(hipEventRecord(after_R, s));
  timed(ctx, 3, L.ne, s, [&] { group(4, [&] { stage_K(P, w, s); }); });
  timed(ctx, 4, L.ne, s, [&] { group(5, [&] { stage_SO(P, w, false, s); }); });
  group(6, [&] {
    launch_finalize(s, L, w.tab, w.pwi, w.status, w.omega, w.Kw, nullptr);
    launch_pack(s, L, w.tab, w.pwi, 0, w.omega, w.pack_off, w.pack);
  });
  if (chunk_timed) {
    chunk_rec.cost = cost;
    chunk_rec.open = open;
    prof_end(ctx, s, chunk_rec);
  }
  if (st != RM_OK) return st;
  for (const Part &pt : P.parts) {
    const Seg &g = segs[pt.seg];
    const long o0 = sl.h.off[pt.e0], o1 = sl.h.off[pt.e0 + pt.m - 1] + (long)g.pw->nt * g.pw->nt;
    HIPCHK(hipMemcpyAsync(g.omega + (size_t)pt.e_begin * g.pw->nt * g.pw->nt, w.pack + o0, sizeof(double) * (o1 - o0),
                          ko, s));
    HIPCHK(hipMemcpyAsync(g.status + pt.e_begin, w.status + pt.e0, sizeof(int) * pt.m, ko, s));
  }
  if (want_K) {
    // K is packed into the same buffer once Omega's copies are queued
    group(7, [&] { launch_pack(s, L, w.tab, w.pwi, 1, w.Kw, w.pack_off + L.ne + 1, w.pack); });
    if (st != RM_OK) return st;
    for (const Part &pt : P.parts) {
      const Seg &g = segs[pt.seg];
      if (!g.K) continue;
      const long o0 = sl.h.off[L.ne + 1 + pt.e0], o1 = o0 + (long)pt.m * g.pw->n * g.pw->n;
      HIPCHK(hipMemcpyAsync(g.K + (size_t)pt.e_begin * g.pw->n * g.pw->n, w.pack + o0, sizeof(double) * (o1 - o0), ko,
                            s));
    }
  }
  HIPCHK(hipGetLastError());
  return RM_OK;
}

// Cuts the segments into chunks of at most `cap` energies.  With `interleave`
// every chunk takes up to EB energies from each segment in turn, so a chunk
// holds many partial waves (one persistent R launch serves them all);
// otherwise segments are cut in order.
std::vector<Plan> cut_chunks(const std::vector<Seg> &segs, int cap, bool interleave) {
  std::vector<Plan> plans;
  std::vector<int> pos(segs.size(), 0);
  size_t left = 0;
  for (const Seg &g : segs) left += g.ne;
  size_t cur = 0;
  while (left > 0) {
    Plan P;
    int ne = 0;
    if (interleave) {
      bool progress = true;
      while (ne < cap && progress) {
        progress = false;
        for (size_t g = 0; g < segs.size() && ne < cap; ++g) {
          const int take = std::min({EB, segs[g].ne - pos[g], cap - ne});
          if (take <= 0) continue;
          if (!P.parts.empty() && P.parts.back().seg == (int)g && P.parts.back().e_begin + P.parts.back().m == pos[g])
            P.parts.back().m += take;
          else
            P.parts.push_back(Part{(int)g, pos[g], take, ne, 0});
          pos[g] += take;
          ne += take;
          progress = true;
        }
      }
      // keep each segment's energies of this chunk contiguous: merge its parts
      std::vector<Part> merged;
      for (size_t g = 0; g < segs.size(); ++g) {
        int first = -1, total = 0;
        for (const Part &pt : P.parts)
          if (pt.seg == (int)g) {
            if (first < 0) first = pt.e_begin;
            total += pt.m;
          }
        if (total) merged.push_back(Part{(int)g, first, total, 0, 0});
      }
      int e0 = 0;
      for (Part &pt : merged) {
        pt.e0 = e0;
        e0 += pt.m;
      }
      P.parts = merged;
    } else {
      while (ne < cap && cur < segs.size()) {
        const int take = std::min(segs[cur].ne - pos[cur], cap - ne);
        if (take > 0) {
          P.parts.push_back(Part{(int)cur, pos[cur], take, ne, 0});
          pos[cur] += take;
          ne += take;
        }
        if (pos[cur] >= segs[cur].ne) ++cur;
      }
    }
    left -= ne;
    finish_plan(P, segs, ne);
    plans.push_back(std::move(P));
  }
  return plans;
}

// The pipelined executor behind rm_run and rm_run_batch.
rm_status run_segments(rm_ctx *ctx, const std::vector<Seg> &segs, const rm_opts &o, bool interleave) {
  const hipStream_t user = call_stream(ctx, o);
  if (!ctx->ev_in) {
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipEventCreateWithFlags(&ctx->ev_out[i], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ctx->ev_R[i], hipEventDisableTiming));
      HIPCHK(hipStreamCreateWithFlags(&ctx->pipe[i].stream, hipStreamNonBlocking));
    }
  }
  size_t total = 0;
  int n = 0, npad = 0, Mpad = 0, nt = 0, npc = 0;
  for (const Seg &g : segs) {
    total += g.ne;
    n = std::max(n, g.pw->n);
    npad = std::max(npad, g.pw->npad);
    Mpad = std::max(Mpad, g.pw->Mpad);
    nt = std::max(nt, g.pw->nt);
    if (g.pw->lamax) npc = std::max(npc, g.pw->npad);
  }
  if (!total) return RM_OK;
  size_t share;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t used = ctx->resident + ctx->work_bytes - ctx->pipe[0].w.bytes - ctx->pipe[1].w.bytes;
    share = ctx->budget > used ? (ctx->budget - used) / 2 : 0;
  }
  // Chunks of up to MAX_CHUNK energies (fewer if the HBM budget says so)
  // alternate over the two streams.  Large chunks keep every launch of the LU
  // chain wide enough to fill the device.
  const int cap = chunk_cap(n, npad, Mpad, nt, share, MAX_CHUNK, npc);
  std::vector<Plan> plans = cut_chunks(segs, cap, interleave);
  const int nuse = plans.size() > 1 ? 2 : 1;
  HIPCHK(hipEventRecord(ctx->ev_in, user));
  for (int i = 0; i < nuse; ++i) HIPCHK(hipStreamWaitEvent(ctx->pipe[i].stream, ctx->ev_in, 0));
  for (size_t k = 0; k < plans.size(); ++k) {
    Slot &sl = ctx->pipe[k % nuse];
    Plan &P = plans[k];
    if (rm_status st = ensure_slot(ctx, sl, P.L, (int)P.slots.size(), plan_tasks(ctx, P, o), false)) return st;
    if (rm_status st = upload_plan(ctx, sl, P, segs, o, false)) return st;
    hipEvent_t prevR = k > 0 && nuse > 1 ? ctx->ev_R[(k - 1) % 2] : nullptr;
    if (rm_status st = run_chunk(ctx, P, sl, segs, o, kind_out(o), prevR, ctx->ev_R[k % 2])) return st;
  }
  for (int i = 0; i < nuse; ++i) {
    HIPCHK(hipEventRecord(ctx->ev_out[i], ctx->pipe[i].stream));
    HIPCHK(hipStreamWaitEvent(user, ctx->ev_out[i], 0));
  }
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(user));
  return RM_OK;
}

// Plans one chunk of one partial wave for the staged calls (on ctx->sync).
rm_status staged_chunk(rm_ctx *ctx, const DevPW *pw, const double *E, int e0, int m, const rm_opts &o, bool want_S,
                       Plan &P, std::vector<Seg> &segs) {
  segs.assign(1, Seg{pw, E, e0 + m, nullptr, nullptr, nullptr});
  P = Plan();
  P.parts.push_back(Part{0, e0, m, 0, 0});
  finish_plan(P, segs, m);
  if (rm_status st = ensure_slot(ctx, ctx->sync, P.L, 1, plan_tasks(ctx, P, o), want_S)) return st;
  return upload_plan(ctx, ctx->sync, P, segs, o, false);
}

int staged_cap(rm_ctx *ctx, const DevPW *pw, int ne) {
  return chunk_cap(pw->n, pw->npad, pw->Mpad, pw->nt, free_share(ctx, ctx->sync), std::min(ne, 256),
                   pw->lamax ? pw->npad : 0);
}

// The staged calls run on ctx->sync.stream; with device pointers it is ordered
// after the caller's stream on entry and the caller's stream after it on exit.
rm_status staged_enter(rm_ctx *ctx, const rm_opts &o, hipEvent_t &ev) {
  if (!ctx->sync.stream) HIPCHK(hipStreamCreateWithFlags(&ctx->sync.stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, call_stream(ctx, o)));
  HIPCHK(hipStreamWaitEvent(ctx->sync.stream, ev, 0));
  return RM_OK;
}

rm_status staged_leave(rm_ctx *ctx, const rm_opts &o, hipEvent_t ev) {
  HIPCHK(hipEventRecord(ev, ctx->sync.stream));
  HIPCHK(hipStreamWaitEvent(call_stream(ctx, o), ev, 0));
  if (!o.device_ptrs) HIPCHK(hipStreamSynchronize(ctx->sync.stream));
  HIPCHK(hipEventDestroy(ev));
  return RM_OK;
}

// ------------------------------------------------------------------ serving
// A worker forms a chunk from the queued requests (continuous batching): it
// takes energies from every active request with work left, earliest arrival
// first, up to the chunk capacity, runs the chunk on its own stream, and hands
// the results back per request.  Requests that arrive while chunks run join
// the next chunk a worker forms.
//
// Admission by HBM footprint: a worker sizes its chunk to its share of the free
// budget (the free budget split over the workers).  If not even one energy of
// the chunk's shape fits, the worker becomes the memory waiter: the other
// workers finish their current chunk, release their workspaces and take no new
// work until the waiter has formed its chunk (with the whole free budget).  A
// shape that would not fit even with every other workspace released fails its
// requests with RM_E_NOMEM.
// Ends a serving chunk whose forming or run threw: waits for what the slot's
// stream already has in flight (it may still write the requests' host
// buffers), then counts the energies each request gave to the chunk as done,
// with RM_E_NOMEM.  P.parts and owners grow in step, parts first.
void chunk_failed(rm_ctx *ctx, Slot *slot, const std::vector<Req *> &owners, const Plan &P) noexcept {
  if (slot->stream) (void)hipStreamSynchronize(slot->stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (size_t i = 0; i < owners.size() && i < P.parts.size(); ++i) {
    Req *r = owners[i];
    r->inflight--;
    r->done_e += P.parts[i].m;
    r->err = RM_E_NOMEM;
    if (r->done_e >= r->rq.ne) r->st.t_done_ns = now_ns();
  }
  try {
    ctx->err = "out of host memory in a serving worker (its chunk's requests end with RM_E_NOMEM)";
  } catch (...) {
  }
  ctx->cv.notify_all();
}

void worker_main(rm_ctx *ctx, Slot *slot) {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    std::vector<Seg> segs;
    std::vector<Req *> owners;
    Plan P;
    rm_opts o;
    Work released;
    try {
      {
        std::unique_lock<std::mutex> lk(ctx->mu);
        ctx->cv.wait(lk, [&] {
          if (ctx->stop) return true;
          if (ctx->mem_waiter && ctx->mem_waiter != slot) return slot->w.bytes > 0;
          for (Req *q : ctx->active)
            if (q->next_e < q->rq.ne) return true;
          return false;
        });
        if (ctx->stop) return;
        if (ctx->mem_waiter && ctx->mem_waiter != slot) {
          // another worker waits for memory: hand this workspace back (freed
          // outside the lock; the slot's stream is idle between chunks)
          released = slot->w;
          slot->w = Work();
          ctx->work_bytes -= released.bytes;
        }
      }
      if (released.bytes) {
        free_work(released);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->cv.notify_all();
        continue;
      }
      {
        std::unique_lock<std::mutex> lk(ctx->mu);
        const Req *first = nullptr;
        for (Req *q : ctx->active)
          if (q->next_e < q->rq.ne) {
            first = q;
            break;
          }
        if (!first) continue;
        // the options of the earliest request with work decide the chunk's
        o = fixed_opts(&first->rq.opts);
        o.device_ptrs = 0;
        o.stream = nullptr;
        // requests join the chunk only if every option the chunk's kernels read
        // (precision, near-pole window, threshold guard) equals the first one's
        auto compatible = [&](const Req *q) {
          const rm_opts f = fixed_opts(&q->rq.opts);
          return f.prec == o.prec && f.split_delta == o.split_delta && f.thr_guard == o.thr_guard;
        };
        // largest member shapes decide the per-energy footprint
        const size_t used = ctx->resident + ctx->work_bytes - slot->w.bytes;
        const size_t avail = ctx->budget > used ? ctx->budget - used : 0;
        size_t share = ctx->mem_waiter == slot ? avail : avail / std::max<size_t>(ctx->slots.size(), 1);
        int n = 0, npad = 0, Mpad = 0, nt = 0, npc = 0;
        for (Req *q : ctx->active) {
          if (q->next_e >= q->rq.ne || !compatible(q)) continue;
          auto it = ctx->pws.find(q->rq.pw_id);
          if (it == ctx->pws.end()) continue;
          n = std::max(n, it->second.n);
          npad = std::max(npad, it->second.npad);
          Mpad = std::max(Mpad, it->second.Mpad);
          nt = std::max(nt, it->second.nt);
          if (it->second.lamax) npc = std::max(npc, it->second.npad);
        }
        const size_t one = n ? per_energy_bytes(n, npad, Mpad, nt, npc) + kChunkFixedBytes : 0;
        if (one > share) {
          size_t others = 0;  // releasable by the other serving workers
          for (const auto &sl : ctx->slots)
            if (sl.get() != slot) others += sl->w.bytes;
          if (one <= avail) {
            share = avail;  // fits once this worker takes the whole free budget
          } else if (one <= avail + others) {
            if (!ctx->mem_waiter) ctx->mem_waiter = slot;
            ctx->cv.notify_all();
            if (ctx->mem_waiter != slot) ctx->cv.wait(lk);
            else
              ctx->cv.wait(lk, [&] {
                return ctx->stop || ctx->resident + ctx->work_bytes - slot->w.bytes + one <= ctx->budget;
              });
            continue;
          } else {
            // cannot fit even alone: fail the compatible requests of this shape
            for (Req *q : ctx->active) {
              if (q->next_e >= q->rq.ne || !compatible(q)) continue;
              auto it = ctx->pws.find(q->rq.pw_id);
              if (it == ctx->pws.end() || it->second.n != n) continue;
              q->err = RM_E_NOMEM;
              q->done_e = q->next_e = q->rq.ne;
              q->st.t_done_ns = now_ns();
            }
            ctx->err = "a request's per-energy workspace exceeds the HBM budget";
            if (ctx->mem_waiter == slot) ctx->mem_waiter = nullptr;
            ctx->cv.notify_all();
            continue;
          }
        }
        if (ctx->mem_waiter == slot) {
          ctx->mem_waiter = nullptr;
          ctx->cv.notify_all();
        }
        int room = n ? chunk_cap(n, npad, Mpad, nt, share, 256, npc) : 0;
        for (Req *q : ctx->active) {
          if (room <= 0) break;
          if (q->next_e >= q->rq.ne || !compatible(q)) continue;
          auto it = ctx->pws.find(q->rq.pw_id);
          if (it == ctx->pws.end()) {
            q->err = RM_E_NOTFOUND;
            q->done_e = q->next_e = q->rq.ne;
            q->st.t_done_ns = now_ns();
            continue;
          }
          const int take = std::min(room, q->rq.ne - q->next_e);
          Seg g;
          g.pw = &it->second;
          g.E = q->E.data();
          g.ne = q->rq.ne;
          g.omega = q->rq.omega;
          g.K = q->rq.K;
          g.status = q->rq.status;
          P.parts.push_back(Part{(int)segs.size(), q->next_e, take, 0, 0});
          segs.push_back(g);
          owners.push_back(q);
          q->next_e += take;
          q->inflight++;
          room -= take;
          const int64_t t = now_ns();
          if (!q->admitted) {
            q->admitted = true;
            q->st.t_admit_ns = t;
          }
          if (!q->st.t_start_ns) q->st.t_start_ns = t;
          q->st.nblocks++;
        }
        ctx->cv.notify_all();
      }
      if (P.parts.empty()) continue;
      int ne = 0;
      for (Part &pt : P.parts) {
        pt.e0 = ne;
        ne += pt.m;
      }
      finish_plan(P, segs, ne);
      rm_status st = ensure_slot(ctx, *slot, P.L, (int)P.slots.size(), plan_tasks(ctx, P, o), false);
      if (st == RM_OK) st = upload_plan(ctx, *slot, P, segs, o, false);
      if (st == RM_OK) st = run_chunk(ctx, P, *slot, segs, o, hipMemcpyDeviceToHost);
      if (st == RM_OK && hipStreamSynchronize(slot->stream) != hipSuccess) st = RM_E_DEVICE;
      {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (size_t i = 0; i < owners.size(); ++i) {
          Req *r = owners[i];
          r->inflight--;
          r->done_e += P.parts[i].m;
          if (st != RM_OK) r->err = st;
          if (r->done_e >= r->rq.ne) r->st.t_done_ns = now_ns();
        }
        ctx->cv.notify_all();
      }
    } catch (...) {
      // a host allocation failed while this chunk was formed or run: its
      // requests end with RM_E_NOMEM instead of the exception ending the process
      chunk_failed(ctx, slot, owners, P);
    }
  }
}

void free_pw(DevPW &p) {
  void *ptrs[] = {p.W64, p.W32, p.Ek, p.ethr, p.l, p.target, p.tptr, p.tch, p.cft, p.cfm};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
}

void destroy_slot(Slot &sl) {
  if (sl.stream) {
    (void)hipStreamSynchronize(sl.stream);
    (void)hipStreamDestroy(sl.stream);
  }
  for (hipGraphExec_t &ex : sl.g.exec)
    if (ex) (void)hipGraphExecDestroy(ex);
  for (auto &r : sl.g.retired) {
    (void)hipGraphExecDestroy(r.first);
    (void)hipEventDestroy(r.second);
  }
  for (int g = 0; g < NGROUP; ++g) {
    sl.g.exec[g] = nullptr;
    sl.g.key[g].clear();
  }
  sl.g.retired.clear();
  free_work(sl.w);
  free_staging(sl.h);
}

// ------------------------------------------------------------ no-alloc path
// Staging capacities of the no-alloc slot (pinned, allocated by rm_create).
constexpr int NA_TASKS = 65536;

// Device address of the scratch array on `device` (resolved on first use).
rm_status scratch_address(rm_ctx *ctx, int device, char **out) {
  static std::mutex mu;
  static std::map<int, char *> addr;
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ctx->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return RM_E_DEVICE;
    }
    it = addr.emplace(device, (char *)p).first;
  }
  *out = it->second;
  return RM_OK;
}

// Points the buffers of a workspace for chunks of layout L into the scratch
// array; false if they do not fit.
bool carve_work(Work &w, char *base, const Lay &L, int ntab, int ntasks) {
  Work nw;
  const std::vector<WorkBuf> bufs =
      work_buffers(nw, L.ne, L.nmax, L.npadmax, L.Mpadmax, L.ntmax, ntab, ntasks, false, L.npadc);
  if (work_bytes(bufs) > RM_NOALLOC_SCRATCH_BYTES) return false;
  size_t off = 0;
  for (const WorkBuf &b : bufs) {
    *b.ptr = base + off;
    off += (b.bytes + 255) / 256 * 256;
  }
  nw.bytes = 0;  // not counted against the HBM budget
  w = nw;
  return true;
}

// The staging of the no-alloc slot, allocated once by rm_create.
rm_status init_noalloc(rm_ctx *ctx) {
  // a failure here disables only rm_run_noalloc (it then reports the error)
  if (scratch_address(ctx, ctx->device, &ctx->scratch) != RM_OK) ctx->scratch = nullptr;
  Staging &h = ctx->na.h;
  HIPCHK(hipEventCreateWithFlags(&h.ready, hipEventDisableTiming));
  HIPCHK(hipHostMalloc((void **)&h.E, sizeof(double) * MAX_CHUNK, hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void **)&h.pwi, sizeof(int) * MAX_CHUNK, hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void **)&h.tab, sizeof(DevPW), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void **)&h.tasks, sizeof(RTask) * NA_TASKS, hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void **)&h.off, sizeof(long) * 2 * (MAX_CHUNK + 1), hipHostMallocDefault));
  h.cap_e = MAX_CHUNK;
  h.cap_tab = 1;
  h.cap_tasks = NA_TASKS;
  ctx->na.direct = true;
  return RM_OK;
}

// Uploads a partial wave (and its multipole coupling when lamax > 0).
rm_status rm_pw_upload_coupled_impl(rm_ctx *ctx, const rm_pw_desc *d, int32_t lamax, const double *cf, double r1,
                                    int32_t *pw_id);

// Plans energies [e0, e0 + m) of the single segment.
void plan_single(Plan &P, const std::vector<Seg> &segs, int e0, int m) {
  P = Plan();
  P.parts.push_back(Part{0, e0, m, 0, 0});
  finish_plan(P, segs, m);
}

// Why the calling thread's last rm_create failed (rm_last_error(NULL)).
thread_local std::string t_create_err;

// rm_create's failure exit: records the failed call (with HIP's text, or the
// context's own message when what is null), releases what the context holds
// so far and frees it.
rm_status create_failed(rm_ctx *ctx, rm_status st, const char *what, hipError_t e) {
  t_create_err = "rm_create(device " + std::to_string(ctx->device) + "): ";
  t_create_err += what ? std::string(what) + ": " + hipGetErrorString(e) : ctx->err;
  free_staging(ctx->na.h);
  for (auto &sl : ctx->slots) destroy_slot(*sl);
  if (ctx->sync.stream) (void)hipStreamDestroy(ctx->sync.stream);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return st;
}

// An exception thrown inside an entry point (a host allocation or a thread
// start that fails) ends as RM_E_NOMEM: none may reach a C caller.
rm_status abi_failed(rm_ctx *ctx) noexcept {
  try {
    if (ctx) ctx->err = "out of host memory (an allocation or a thread start failed)";
  } catch (...) {
  }
  return RM_E_NOMEM;
}

rm_status abi_failed_create(int device) noexcept {
  try {
    t_create_err = "rm_create(device " + std::to_string(device) + "): out of host memory";
  } catch (...) {
  }
  return RM_E_NOMEM;
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

static rm_status rm_create_body(int device, size_t hbm_budget_bytes, rm_ctx **out) {
  if (!out) return RM_E_ARG;
  *out = nullptr;
  rm_ctx *ctx = new (std::nothrow) rm_ctx();
  if (!ctx) return RM_E_NOMEM;
  ctx->device = device;
  hipError_t he;
  if ((he = hipSetDevice(device)) != hipSuccess) return create_failed(ctx, RM_E_DEVICE, "hipSetDevice", he);
  if ((he = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess ||
      (he = hipStreamCreateWithFlags(&ctx->sync.stream, hipStreamNonBlocking)) != hipSuccess)
    return create_failed(ctx, RM_E_DEVICE, "hipStreamCreateWithFlags", he);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) {
    ctx->ncu = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
  }
  size_t fr = 0, tot = 0;
  if ((he = hipMemGetInfo(&fr, &tot)) != hipSuccess) return create_failed(ctx, RM_E_DEVICE, "hipMemGetInfo", he);
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  const int nslots = 2;
  for (int i = 0; i < nslots; ++i) {
    ctx->slots.push_back(std::make_unique<Slot>());
    if ((he = hipStreamCreateWithFlags(&ctx->slots.back()->stream, hipStreamNonBlocking)) != hipSuccess)
      return create_failed(ctx, RM_E_DEVICE, "hipStreamCreateWithFlags", he);
  }
  if (rm_status st = init_noalloc(ctx)) return create_failed(ctx, st, nullptr, hipSuccess);
  for (auto &sl : ctx->slots) ctx->workers.emplace_back(worker_main, ctx, sl.get());
  *out = ctx;
  return RM_OK;
}

static rm_status rm_destroy_body(rm_ctx *ctx) {
  if (!ctx) return RM_E_ARG;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->stop = true;
    ctx->cv.notify_all();
  }
  for (auto &t : ctx->workers) t.join();
  (void)hipSetDevice(ctx->device);
  for (auto &sl : ctx->slots) destroy_slot(*sl);
  destroy_slot(ctx->sync);
  for (auto &pp : ctx->pipe) destroy_slot(pp);
  free_staging(ctx->na.h);  // its workspace is the scratch array and its stream the caller's
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  for (auto &ev : ctx->ev_out)
    if (ev) (void)hipEventDestroy(ev);
  for (auto &ev : ctx->ev_R)
    if (ev) (void)hipEventDestroy(ev);
  for (auto &kv : ctx->pws) free_pw(kv.second);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return RM_OK;
}

const char *rm_last_error(const rm_ctx *ctx) {
  if (ctx) return ctx->err.c_str();
  return t_create_err.empty() ? "null context" : t_create_err.c_str();
}

size_t rm_pw_footprint(int32_t nchan, int32_t npole) {
  const size_t npad = (size_t)round_up(std::max(nchan, 1), TILE);
  const size_t Mpad = (size_t)round_up(std::max(npole, 1), MALIGN);
  return Mpad * npad * 12 + Mpad * 8 + (size_t)nchan * 24 + 4096;
}

size_t rm_work_footprint(int32_t nchan, int32_t npole, int32_t ntarget, int32_t ne) {
  if (nchan < 1 || npole < 1 || ntarget < 1 || ne < 1) return 0;
  return per_energy_bytes(nchan, round_up(nchan, TILE), round_up(npole, MALIGN), ntarget) * (size_t)ne +
         kChunkFixedBytes;
}

static rm_status rm_pw_upload_body(rm_ctx *ctx, const rm_pw_desc *d, int32_t *pw_id) {
  return rm_pw_upload_coupled_impl(ctx, d, 0, nullptr, 0.0, pw_id);
}

static rm_status rm_pw_upload_coupled_body(rm_ctx *ctx, const rm_pw_desc *d, int32_t lamax, const double *cf, double r1,
                                           int32_t *pw_id) {
  if (!ctx || !d || !pw_id) return RM_E_ARG;
  if (lamax < 1 || lamax > RM_PROP_MAX_LAMAX || !cf || d->nchan < 1 || d->nchan > RM_PROP_MAX_CHANNELS ||
      !(r1 > d->a) || !std::isfinite(r1)) {
    ctx->err = "invalid coupling: 1 <= lamax <= RM_PROP_MAX_LAMAX, nchan <= RM_PROP_MAX_CHANNELS and r1 > a needed";
    return RM_E_ARG;
  }
  for (size_t k = 0; k < (size_t)lamax * d->nchan * d->nchan; ++k)
    if (!std::isfinite(cf[k])) {
      ctx->err = "non-finite multipole coefficient";
      return RM_E_ARG;
    }
  return rm_pw_upload_coupled_impl(ctx, d, lamax, cf, r1, pw_id);
}

static rm_status rm_set_propagation_body(rm_ctx *ctx, int32_t npts, int32_t stab) {
  if (!ctx) return RM_E_ARG;
  if (npts < 4 || stab < 1) {
    ctx->err = "propagation grid: npts >= 4 and stab >= 1 needed";
    return RM_E_ARG;
  }
  ctx->prop_npts.store(npts);
  ctx->prop_stab.store(stab);
  return RM_OK;
}

}  // extern "C"

namespace {

rm_status rm_pw_upload_coupled_impl(rm_ctx *ctx, const rm_pw_desc *d, int32_t lamax, const double *cf, double r1,
                                    int32_t *pw_id) {
  if (!ctx || !d || !pw_id) return RM_E_ARG;
  if (d->nchan < 1 || d->nchan > RM_MAX_CHANNELS || d->npole < 1 || d->ntarget < 1 || !d->e_thr || !d->l || !d->target || !d->Ek || !d->w ||
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
  const size_t cfbytes = (size_t)lamax * round_up(d->nchan, TILE) * round_up(d->nchan, TILE) * 16;
  const size_t bytes = rm_pw_footprint(d->nchan, d->npole) + cfbytes;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->resident + ctx->work_bytes + bytes > ctx->budget) {
      ctx->err = "partial wave exceeds the HBM budget";
      return RM_E_NOMEM;
    }
  }
  (void)hipSetDevice(ctx->device);
  DevPW p;
  // an early return (a failed HIP call) frees what is allocated so far
  struct Unwind {
    DevPW &p;
    bool keep = false;
    ~Unwind() {
      if (!keep) free_pw(p);
    }
  } unwind{p};
  p.n = d->nchan;
  p.M = d->npole;
  p.nt = d->ntarget;
  p.npad = round_up(p.n, TILE);
  p.Mpad = round_up(p.M, MALIGN);
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
  if (lamax) {
    // transposed and fragment-major copies, zero padded
    const size_t sz = (size_t)lamax * p.npad * p.npad;
    std::vector<double> At(sz, 0.0), Am(sz, 0.0);
    const int nb = p.npad / TILE;
    for (int lam = 0; lam < lamax; ++lam)
      for (int i = 0; i < p.n; ++i)
        for (int j = 0; j < p.n; ++j) {
          const double v = cf[((size_t)lam * p.n + i) * p.n + j];
          At[((size_t)lam * p.npad + j) * p.npad + i] = v;
          Am[cfm_index(lam, i, j, nb)] = v;
        }
    HIPCHK(hipMalloc(&p.cft, sz * 8));
    HIPCHK(hipMalloc(&p.cfm, sz * 8));
    HIPCHK(hipMemcpy(p.cft, At.data(), sz * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p.cfm, Am.data(), sz * 8, hipMemcpyHostToDevice));
    p.lamax = lamax;
    p.r1 = r1;
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  const int32_t id = ctx->next_id++;
  ctx->pws[id] = p;
  unwind.keep = true;  // the context owns the buffers now
  ctx->hthr[&ctx->pws[id]].assign(d->e_thr, d->e_thr + p.n);
  ctx->resident += bytes;
  *pw_id = id;
  return RM_OK;
}

}  // namespace

extern "C" {

static rm_status rm_pw_release_body(rm_ctx *ctx, int32_t pw_id) {
  if (!ctx) return RM_E_ARG;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->pws.find(pw_id);
  if (it == ctx->pws.end()) return RM_E_NOTFOUND;
  for (Req *q : ctx->active)
    if (q->rq.pw_id == pw_id && (q->done_e < q->rq.ne || q->inflight > 0)) return RM_E_BUSY;
  DevPW p = it->second;
  ctx->hthr.erase(&it->second);
  ctx->pws.erase(it);
  ctx->resident -= p.bytes;
  lk.unlock();
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_pw(p);
  return RM_OK;
}

static rm_status rm_form_R_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts, double *R,
                                int32_t *status) {
  if (!ctx || (ne > 0 && (!E || !R || !status)) || ne < 0) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  const hipStream_t s = ctx->sync.stream;
  const int cap = staged_cap(ctx, pw, ne);
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, false, P, segs)) return st;
    Work &w = ctx->sync.w;
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    stage_R(ctx, P, w, o, s);
    launch_nanfill_R(s, P.L, w.tab, w.pwi, w.status, w.aug);
    HIPCHK(hipMemcpy2DAsync(R + (size_t)e0 * pw->n * pw->n, sizeof(double) * pw->n, w.aug,
                            sizeof(double) * P.L.ldaug, sizeof(double) * pw->n, (size_t)m * pw->n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  return staged_leave(ctx, o, ev);
}

static rm_status rm_asymptotic_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts,
                                    double *fg, int8_t *open, int32_t *nopen, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !fg || !open || !nopen || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  const hipStream_t s = ctx->sync.stream;
  const int cap = staged_cap(ctx, pw, ne);
  const int n = pw->n;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, false, P, segs)) return st;
    Work &w = ctx->sync.w;
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    stage_asym(ctx, P, w, o, s);
    HIPCHK(hipMemcpyAsync(fg + (size_t)e0 * n * 4, w.fg, sizeof(double) * m * n * 4, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(open + (size_t)e0 * n, w.openflag, (size_t)m * n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(nopen + e0, w.nopen, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  return staged_leave(ctx, o, ev);
}

static rm_status rm_propagate_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts,
                                   double *phi, double *dphi, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !phi || !dphi || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  if (!pw->lamax) {
    ctx->err = "rm_propagate: the partial wave has no multipole coupling";
    return RM_E_ARG;
  }
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  const hipStream_t s = ctx->sync.stream;
  const int cap = staged_cap(ctx, pw, ne);
  const int n = pw->n;
  const int npts = ctx->prop_npts.load(), stab = ctx->prop_stab.load();
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, false, P, segs)) return st;
    Work &w = ctx->sync.w;
    const Lay &L = P.L;
    launch_fill_int(s, w.status, m, 0);
    stage_asym(ctx, P, w, o, s);
    timed(ctx, STAGE_PROP, m, s, [&] {
      launch_prop(s, L, npts, stab, w.tab, w.pwi, w.E, w.fg, w.nopen, w.openidx, w.colpos, w.pz, w.status);
    });
    // phi, then dphi, through aug (n rows of 2 npad >= 2n columns per energy)
    double *outs[2] = {phi, dphi};
    for (int q = 0; q < 2; ++q) {
      launch_prop_gather(s, L, w.tab, w.pwi, w.nopen, w.status, w.pz, 3 + q, w.aug, L.ldaug, L.sA);
      HIPCHK(hipMemcpy2DAsync(outs[q] + (size_t)e0 * n * 2 * n, sizeof(double) * 2 * n, w.aug,
                              sizeof(double) * L.ldaug, sizeof(double) * 2 * n, (size_t)m * n, kind_out(o), s));
    }
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  return staged_leave(ctx, o, ev);
}

static rm_status rm_solve_K_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const double *R,
                                 const double *fg, const rm_opts *opts, double *K, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !R || !fg || !K || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  if (pw->lamax) {
    ctx->err = "rm_solve_K: a coupled wave is matched to its propagated solutions (rm_run)";
    return RM_E_ARG;
  }
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  const hipStream_t s = ctx->sync.stream;
  const int cap = staged_cap(ctx, pw, ne);
  const int n = pw->n;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, false, P, segs)) return st;
    Work &w = ctx->sync.w;
    const Lay &L = P.L;
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    HIPCHK(hipMemcpy2DAsync(w.aug, sizeof(double) * L.ldaug, R + (size_t)e0 * n * n, sizeof(double) * n,
                            sizeof(double) * n, (size_t)m * n, kind_in(o), s));
    HIPCHK(hipMemcpyAsync(w.fg, fg + (size_t)e0 * n * 4, sizeof(double) * m * n * 4, kind_in(o), s));
    launch_dvec(s, L, w.tab, w.pwi, w.E, 0, 0.0, w.D64, w.D32, w.win, w.status);  // pole flags
    launch_openlist(s, L, w.tab, w.pwi, w.E, w.nopen, w.openidx, w.openpos, w.colpos, w.openflag);
    launch_check_inputs(s, L, w.tab, w.pwi, w.E, o.thr_guard, w.aug, w.fg, nullptr, w.nopen, w.status);
    stage_K(P, w, s);
    launch_finalize(s, L, w.tab, w.pwi, w.status, nullptr, w.Kw, nullptr);
    HIPCHK(hipMemcpy2DAsync(K + (size_t)e0 * n * n, sizeof(double) * n, w.Kw, sizeof(double) * L.ldk,
                            sizeof(double) * n, (size_t)m * n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  return staged_leave(ctx, o, ev);
}

static rm_status rm_collision_strengths_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const double *K,
                                             const rm_opts *opts, double *omega, double *S, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !K || !omega || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  const hipStream_t s = ctx->sync.stream;
  const int cap = staged_cap(ctx, pw, ne);
  const int n = pw->n, nt = pw->nt;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, S != nullptr, P, segs)) return st;
    Work &w = ctx->sync.w;
    const Lay &L = P.L;
    HIPCHK(hipMemsetAsync(w.status, 0, sizeof(int) * m, s));
    HIPCHK(hipMemcpy2DAsync(w.Kw, sizeof(double) * L.ldk, K + (size_t)e0 * n * n, sizeof(double) * n,
                            sizeof(double) * n, (size_t)m * n, kind_in(o), s));
    launch_openlist(s, L, w.tab, w.pwi, w.E, w.nopen, w.openidx, w.openpos, w.colpos, w.openflag);
    launch_check_inputs(s, L, w.tab, w.pwi, w.E, o.thr_guard, nullptr, nullptr, w.Kw, w.nopen, w.status);
    stage_SO(P, w, S != nullptr, s);
    launch_finalize(s, L, w.tab, w.pwi, w.status, w.omega, nullptr, S ? w.S : nullptr);
    HIPCHK(hipMemcpyAsync(omega + (size_t)e0 * nt * nt, w.omega, sizeof(double) * m * nt * nt, kind_out(o), s));
    if (S) HIPCHK(hipMemcpyAsync(S + (size_t)e0 * n * n * 2, w.S, sizeof(double) * m * n * n * 2, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  return staged_leave(ctx, o, ev);
}

static rm_status rm_run_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts, double *omega,
                             double *K, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !omega || !status))) return RM_E_ARG;
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  std::vector<Seg> segs(1, Seg{pw, E, ne, omega, K, status});
  return run_segments(ctx, segs, o, false);
}

static rm_status rm_run_noalloc_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_opts *opts,
                                     double *omega, double *K, int32_t *status) {
  if (!ctx || !opts || ne < 0 || (ne > 0 && (!E || !omega || !status))) return RM_E_ARG;
  if (!opts->device_ptrs) {
    ctx->err = "rm_run_noalloc takes device pointers (opts->device_ptrs = 1)";
    return RM_E_ARG;
  }
  if (ne == 0) return RM_OK;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  if (!ctx->scratch) {
    if (ctx->err.empty()) ctx->err = "the no-alloc scratch array has no device address";
    return RM_E_DEVICE;
  }
  std::lock_guard<std::mutex> serial(ctx->na_mu);
  Slot &sl = ctx->na;
  sl.stream = call_stream(ctx, o);
  const std::vector<Seg> segs(1, Seg{pw, E, ne, omega, K, status});
  // the largest chunk whose workspace fits the scratch array and whose R tasks
  // fit the staging
  Plan P;
  int m = std::min(ne, MAX_CHUNK);
  for (;;) {
    plan_single(P, segs, 0, m);
    const int ntasks = plan_tasks(ctx, P, o);
    Work probe;
    if (ntasks <= NA_TASKS && carve_work(probe, ctx->scratch, P.L, 1, ntasks)) break;
    if (m == 1) {
      Work one;
      const size_t need = work_bytes(
          work_buffers(one, 1, pw->n, pw->npad, pw->Mpad, pw->nt, 1, ntasks, false, pw->lamax ? pw->npad : 0));
      ctx->err = "one energy of this partial wave needs " + std::to_string(need) +
                 " bytes of workspace, more than the no-alloc scratch of " +
                 std::to_string((size_t)RM_NOALLOC_SCRATCH_BYTES) + " bytes";
      return RM_E_NOMEM;
    }
    m = std::max(1, m / 2);
  }
  for (int e0 = 0; e0 < ne; e0 += m) {
    const int mm = std::min(m, ne - e0);
    plan_single(P, segs, e0, mm);
    const int ntasks = plan_tasks(ctx, P, o);
    if (!carve_work(sl.w, ctx->scratch, P.L, 1, ntasks)) {  // cannot happen: a smaller chunk of the same wave
      ctx->err = "no-alloc workspace layout";
      return RM_E_NOMEM;
    }
    if (rm_status st = upload_plan(ctx, sl, P, segs, o, false)) return st;
    if (rm_status st = run_chunk(ctx, P, sl, segs, o, hipMemcpyDeviceToDevice)) return st;
  }
  return RM_OK;
}

static rm_status rm_run_batch_body(rm_ctx *ctx, const rm_batch_item *items, int32_t nitems, const rm_opts *opts) {
  if (!ctx || nitems < 0 || (nitems > 0 && !items)) return RM_E_ARG;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  std::vector<Seg> segs;
  for (int i = 0; i < nitems; ++i) {
    const rm_batch_item &it = items[i];
    if (it.ne < 0 || (it.ne > 0 && (!it.E || !it.omega || !it.status))) return RM_E_ARG;
    const DevPW *pw;
    if (rm_status st = get_pw(ctx, it.pw_id, &pw)) return st;
    if (it.ne) segs.push_back(Seg{pw, it.E, it.ne, it.omega, it.K, it.status});
  }
  if (segs.empty()) return RM_OK;
  return run_segments(ctx, segs, o, true);
}

static rm_status rm_run_sum_body(rm_ctx *ctx, const int32_t *pw_ids, int32_t npw, const double *E, int32_t ne,
                                 int32_t order, const rm_opts *opts, double *omega, int32_t *status) {
  if (!ctx || npw < 1 || !pw_ids || ne < 0 || (ne > 0 && (!E || !omega || !status)) ||
      (order != RM_ORDER_WAVE && order != RM_ORDER_PERMUTED))
    return RM_E_ARG;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  std::vector<const DevPW *> pws(npw);
  for (int w = 0; w < npw; ++w) {
    if (rm_status st = get_pw(ctx, pw_ids[w], &pws[w])) return st;
    if (pws[w]->nt != pws[0]->nt) {
      ctx->err = "partial waves of a sum must share their targets (same ntarget)";
      return RM_E_ARG;
    }
  }
  if (ne == 0) return RM_OK;
  const int nt = pws[0]->nt;
  const size_t per = (size_t)ne * nt * nt;
  const hipStream_t user = call_stream(ctx, o);
  // device temporaries: every wave's Omega and status, the energies, the sum
  struct Tmp {
    hipStream_t s = nullptr;
    void *p[3] = {nullptr, nullptr, nullptr};
    ~Tmp() {
      if (s) (void)hipStreamSynchronize(s);  // no buffer is freed under running work
      for (void *q : p)
        if (q) (void)hipFree(q);
    }
  } tmp;
  tmp.s = user;
  double *tom, *dE, *sum;
  int32_t *tst, *sst;
  HIPCHK(hipMalloc(&tmp.p[0], sizeof(double) * per * npw + sizeof(int32_t) * (size_t)ne * npw));
  tom = static_cast<double *>(tmp.p[0]);
  tst = reinterpret_cast<int32_t *>(tom + per * npw);
  if (o.device_ptrs) {
    dE = const_cast<double *>(E);
    sum = omega;
    sst = status;
  } else {
    HIPCHK(hipMalloc(&tmp.p[1], sizeof(double) * ne));
    HIPCHK(hipMalloc(&tmp.p[2], sizeof(double) * per + sizeof(int32_t) * ne));
    dE = static_cast<double *>(tmp.p[1]);
    sum = static_cast<double *>(tmp.p[2]);
    sst = reinterpret_cast<int32_t *>(sum + per);
    HIPCHK(hipMemcpyAsync(dE, E, sizeof(double) * ne, hipMemcpyHostToDevice, user));
  }
  std::vector<Seg> segs;
  for (int w = 0; w < npw; ++w) segs.push_back(Seg{pws[w], dE, ne, tom + per * w, nullptr, tst + (size_t)ne * w});
  rm_opts od = o;
  od.device_ptrs = 1;
  od.stream = user;
  if (rm_status st = run_segments(ctx, segs, od, order == RM_ORDER_PERMUTED)) {
    (void)hipStreamSynchronize(user);
    return st;
  }
  launch_sum_waves(user, npw, ne, nt, tom, tst, sum, sst);
  if (!o.device_ptrs) {
    HIPCHK(hipMemcpyAsync(omega, sum, sizeof(double) * per, hipMemcpyDeviceToHost, user));
    HIPCHK(hipMemcpyAsync(status, sst, sizeof(int32_t) * ne, hipMemcpyDeviceToHost, user));
  }
  HIPCHK(hipStreamSynchronize(user));
  return RM_OK;
}

static rm_status rm_set_graph_body(rm_ctx *ctx, int32_t on) {
  if (!ctx) return RM_E_ARG;
  ctx->graphs.store(on ? 1 : 0);
  return RM_OK;
}

static rm_status rm_graph_stats_body(rm_ctx *ctx, int64_t *captures, int64_t *replays) {
  if (!ctx || !captures || !replays) return RM_E_ARG;
  int64_t c = ctx->sync.g.captures + ctx->pipe[0].g.captures + ctx->pipe[1].g.captures;
  int64_t r = ctx->sync.g.replays + ctx->pipe[0].g.replays + ctx->pipe[1].g.replays;
  for (auto &sl : ctx->slots) {
    c += sl->g.captures;
    r += sl->g.replays;
  }
  *captures = c;
  *replays = r;
  return RM_OK;
}

// ------------------------------------------------------------ tile autotuner
int32_t rm_tile_bucket(int32_t nchan) { return size_bucket(nchan); }

int32_t rm_tile_count(int32_t prec) {
  if (prec != RM_FP64 && prec != RM_FP32_SPLIT) return 0;
  return nrtile(prec == RM_FP32_SPLIT);
}

static rm_status rm_tile_shape_body(int32_t prec, int32_t shape, int32_t *tile, int32_t *energies) {
  if (shape < 0 || shape >= rm_tile_count(prec) || !tile || !energies) return RM_E_ARG;
  const RTile t = rtile(prec == RM_FP32_SPLIT, shape);
  *tile = 16 * t.tm;
  *energies = t.eb;
  return RM_OK;
}

static rm_status rm_get_tile_body(rm_ctx *ctx, int32_t prec, int32_t bucket, int32_t *shape) {
  if (!ctx || !shape || rm_tile_count(prec) == 0 || bucket < 0 || bucket >= NBUCKET) return RM_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  *shape = ctx->tile[prec == RM_FP32_SPLIT][bucket];
  return RM_OK;
}

static rm_status rm_set_tile_body(rm_ctx *ctx, int32_t prec, int32_t bucket, int32_t shape) {
  if (!ctx || shape < 0 || shape >= rm_tile_count(prec) || bucket < 0 || bucket >= NBUCKET) return RM_E_ARG;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->tile[prec == RM_FP32_SPLIT][bucket] = shape;
  return RM_OK;
}

static rm_status rm_tune_body(rm_ctx *ctx, int32_t prec, const int32_t *pw_ids, int32_t npw, const double *E,
                              int32_t ne, int32_t reps, const char *cache_path, double *ms) {
  if (!ctx || rm_tile_count(prec) == 0 || !pw_ids || npw < 1 || !E || ne < 1 || reps < 1) return RM_E_ARG;
  (void)hipSetDevice(ctx->device);
  const int split = prec == RM_FP32_SPLIT, ns = nrtile(split);
  rm_opts o;
  rm_opts_default(&o);
  o.prec = (rm_precision)prec;
  std::vector<double> tot((size_t)NBUCKET * ns, 0.0), best_ms((size_t)npw * ns, 0.0);
  bool seen[NBUCKET] = {false};
  hipEvent_t ea = nullptr, eb = nullptr;
  HIPCHK(hipEventCreate(&ea));
  HIPCHK(hipEventCreate(&eb));
  rm_status st = RM_OK;
  for (int w = 0; w < npw && st == RM_OK; ++w) {
    const DevPW *pw;
    if ((st = get_pw(ctx, pw_ids[w], &pw))) break;
    const int m = std::min(ne, staged_cap(ctx, pw, ne));
    const int bk = size_bucket(pw->n);
    seen[bk] = true;
    for (int sh = 0; sh < ns && st == RM_OK; ++sh) {
      std::vector<Seg> segs(1, Seg{pw, E, m, nullptr, nullptr, nullptr});
      Plan P;
      P.parts.push_back(Part{0, 0, m, 0, 0});
      finish_plan(P, segs, m);
      const int ntask = plan_tasks(ctx, P, o, sh);
      if ((st = ensure_slot(ctx, ctx->sync, P.L, 1, ntask, false))) break;
      if ((st = upload_plan(ctx, ctx->sync, P, segs, o, false))) break;
      Work &wk = ctx->sync.w;
      const hipStream_t s = ctx->sync.stream;
      double best = 1e300;
      for (int r = 0; r <= reps; ++r) {
        if (hipEventRecord(ea, s) != hipSuccess) { st = RM_E_DEVICE; break; }
        launch_dvec(s, P.L, wk.tab, wk.pwi, wk.E, split, o.split_delta, wk.D64, wk.D32, wk.win, wk.status);
        launch_rform(s, P.L, split, sh, wk.tab, wk.tasks, P.q[sh], wk.counter + NQ * sh, ctx->ncu, wk.D64, wk.D32,
                     wk.aug);
        float t = 0;
        if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
            hipEventElapsedTime(&t, ea, eb) != hipSuccess) {
          st = RM_E_DEVICE;
          break;
        }
        if (r > 0) best = std::min(best, (double)t);
      }
      best_ms[(size_t)w * ns + sh] = best;
      tot[(size_t)bk * ns + sh] += best;
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (st != RM_OK) {
    if (st == RM_E_DEVICE) ctx->err = "device error while tuning";
    return st;
  }
  if (ms) std::copy(best_ms.begin(), best_ms.end(), ms);
  int choice[NBUCKET];
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    // another shape must beat the default by TUNE_MARGIN: a chunk launches the
    // contraction once per shape it uses, so a near tie is not worth a launch
    for (int b = 0; b < NBUCKET; ++b) {
      if (seen[b]) {
        const double *t = tot.data() + (size_t)b * ns;
        int best = 0;
        for (int sh = 1; sh < ns; ++sh)
          if (t[sh] < t[best] && t[sh] < (1.0 - TUNE_MARGIN) * t[0]) best = sh;
        ctx->tile[split][b] = best;
      }
      choice[b] = ctx->tile[split][b];
    }
  }
  if (cache_path) {
    FILE *f = std::fopen(cache_path, "w");
    if (!f) {
      ctx->err = "cannot write the tile cache";
      return RM_E_DEVICE;
    }
    std::fprintf(f, "{\"rm_tile_cache\": 1, \"arch\": \"%s\", \"cus\": %d, \"entries\": [\n", ctx->arch.c_str(),
                 ctx->ncu);
    bool first = true;
    for (int b = 0; b < NBUCKET; ++b) {
      if (!seen[b]) continue;
      const RTile t = rtile(split, choice[b]);
      std::fprintf(f, "%s {\"prec\": %d, \"bucket\": %d, \"shape\": %d, \"tile\": %d, \"energies\": %d, \"ms\": [",
                   first ? "" : ",\n", prec, b, choice[b], 16 * t.tm, t.eb);
      for (int sh = 0; sh < ns; ++sh) std::fprintf(f, "%s%.4f", sh ? ", " : "", tot[(size_t)b * ns + sh]);
      std::fprintf(f, "]}");
      first = false;
    }
    std::fprintf(f, "\n]}\n");
    if (std::fclose(f) != 0) {
      ctx->err = "cannot write the tile cache";
      return RM_E_DEVICE;
    }
  }
  return RM_OK;
}

static rm_status rm_tune_load_body(rm_ctx *ctx, const char *cache_path) {
  if (!ctx || !cache_path) return RM_E_ARG;
  FILE *f = std::fopen(cache_path, "r");
  if (!f) {
    ctx->err = "cannot read the tile cache";
    return RM_E_NOTFOUND;
  }
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 20)) text.append(buf, got);
  std::fclose(f);
  auto bad = [&](const char *why) {
    ctx->err = std::string("tile cache: ") + why;
    return RM_E_ARG;
  };
  // integer value of "key" (JSON: optional blanks around the colon) within
  // [from, to); false if absent
  auto intval = [&](const char *key, size_t from, size_t to, long &out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = text.find(k, from);
    if (at == std::string::npos || at >= to) return false;
    size_t p = at + k.size();
    while (p < to && std::isspace((unsigned char)text[p])) ++p;
    if (p >= to || text[p] != ':') return false;
    const char *c = text.c_str() + p + 1;
    char *end = nullptr;
    out = std::strtol(c, &end, 10);
    return end != c && (size_t)(end - text.c_str()) <= to;
  };
  // string value of "key"
  auto strval = [&](const char *key, std::string &out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = text.find(k);
    if (at == std::string::npos) return false;
    size_t p = at + k.size();
    while (p < text.size() && std::isspace((unsigned char)text[p])) ++p;
    if (p >= text.size() || text[p] != ':') return false;
    p = text.find('"', p + 1);
    if (p == std::string::npos) return false;
    const size_t q = text.find('"', p + 1);
    if (q == std::string::npos) return false;
    out = text.substr(p + 1, q - p - 1);
    return true;
  };
  long v = 0;
  if (!intval("rm_tile_cache", 0, text.size(), v) || v != 1) return bad("not a tile cache of this version");
  std::string arch;
  if (!strval("arch", arch)) return bad("no architecture");
  if (arch != ctx->arch) return bad("made on a device of another architecture");
  if (!intval("cus", 0, text.size(), v) || v != ctx->ncu) return bad("made on a device with another compute-unit count");
  // entries: every object that holds a "prec" key
  std::vector<std::array<int, 3>> set;
  for (size_t pos = text.find("\"prec\""); pos != std::string::npos; pos = text.find("\"prec\"", pos + 1)) {
    const size_t b = text.rfind('{', pos), end = text.find('}', pos);
    if (b == std::string::npos || end == std::string::npos) return bad("entry outside an object");
    long prec, bucket, shape;
    if (!intval("prec", b, end, prec) || !intval("bucket", b, end, bucket) || !intval("shape", b, end, shape))
      return bad("entry without prec, bucket or shape");
    if (rm_tile_count((int32_t)prec) == 0 || bucket < 0 || bucket >= NBUCKET || shape < 0 ||
        shape >= rm_tile_count((int32_t)prec))
      return bad("entry out of range");
    set.push_back({(int)prec, (int)bucket, (int)shape});
  }
  if (set.empty()) return bad("no entries");
  std::lock_guard<std::mutex> g(ctx->mu);
  for (const auto &e : set) ctx->tile[e[0] == RM_FP32_SPLIT][e[1]] = e[2];
  return RM_OK;
}

static rm_status rm_submit_body(rm_ctx *ctx, const rm_request *req, uint64_t *ticket) {
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
  if (req->ne == 0) r->st.t_admit_ns = r->st.t_start_ns = r->st.t_done_ns = r->st.t_arrive_ns;
  ctx->active.push_back(r.get());
  ctx->reqs[r->ticket] = std::move(r);
  ctx->cv.notify_all();
  return RM_OK;
}

static rm_status rm_poll_body(rm_ctx *ctx, uint64_t ticket, rm_req_stats *st) {
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

static rm_status rm_drain_body(rm_ctx *ctx) {
  if (!ctx) return RM_E_ARG;
  std::unique_lock<std::mutex> lk(ctx->mu);
  ctx->cv.wait(lk, [&] {
    for (Req *q : ctx->active)
      if (q->done_e < q->rq.ne || q->inflight > 0) return false;
    return true;
  });
  return RM_OK;
}

static rm_status rm_prof_enable_body(rm_ctx *ctx, int32_t on) {
  if (!ctx) return RM_E_ARG;
  ctx->prof_on.store(on ? 1 : 0);
  return RM_OK;
}

static rm_status rm_prof_read_body(rm_ctx *ctx, const char *stage, double *total_ms, int64_t *launches,
                                   int64_t *energies) {
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

static rm_status rm_prof_chunks_body(rm_ctx *ctx, int64_t cap, double *ms, double *model_flops, double *open_frac,
                                     int64_t *energies, int64_t *count) {
  if (!ctx || !count || cap < 0 || (cap > 0 && (!ms || !model_flops || !open_frac || !energies))) return RM_E_ARG;
  std::vector<ProfRec> mine;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<ProfRec> rest;
    for (auto &r : ctx->prof) (r.stage == STAGE_CHUNK && (int64_t)mine.size() < cap ? mine : rest).push_back(r);
    ctx->prof.swap(rest);
  }
  rm_status st = RM_OK;
  for (size_t i = 0; i < mine.size(); ++i) {
    ProfRec &r = mine[i];
    float t = 0;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) st = RM_E_DEVICE;
    ms[i] = t;
    model_flops[i] = r.cost;
    open_frac[i] = r.energies ? r.open / (double)r.energies : 0.0;
    energies[i] = r.energies;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  *count = (int64_t)mine.size();
  return st;
}


}  // extern "C"

// ------------------------------------------------- quantum-defect operation
namespace {

// Device temporaries of one call, freed on every return path.
struct DevTmp {
  std::vector<void *> p;
  template <typename T>
  T *get(size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    p.push_back(q);
    return (T *)q;
  }
  ~DevTmp() {
    for (void *q : p) (void)hipFree(q);
  }
};

rm_status mqdt_check(rm_ctx *ctx, const DevPW *pw, double fnumin) {
  if (pw->lamax) {
    ctx->err = "quantum-defect operation: waves with a long-range coupling are not supported";
    return RM_E_ARG;
  }
  if (!(pw->z > 0)) {
    ctx->err = "quantum-defect operation needs a charged target (z > 0)";
    return RM_E_ARG;
  }
  if (!(fnumin >= 0) || !std::isfinite(fnumin)) {
    ctx->err = "fnumin must be finite and >= 0";
    return RM_E_ARG;
  }
  return RM_OK;
}

// Unphysical K at energies E (host or device as o says) on ctx->sync: the
// physical pipeline with the channel split and the asymptotic functions in
// quantum-defect mode.  Ku [ne][n][n] and nmember / status [ne] are written
// with the copy kinds given.  With Xp, Yp (device, [ne][n][n]) also the real
// and imaginary parts of (1 - i Ku)^-1, from the complex symmetric
// factorisation of the S/Omega stage (valid on the member block).
rm_status mqdt_coarse(rm_ctx *ctx, const DevPW *pw, const double *E, int ne, const rm_opts &o, double fnumin,
                      double *Ku, hipMemcpyKind kK, int32_t *nmember, int32_t *status, hipMemcpyKind kS,
                      double *Xp = nullptr, double *Yp = nullptr) {
  const hipStream_t s = ctx->sync.stream;
  const int cap = staged_cap(ctx, pw, ne);
  const int n = pw->n;
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, false, P, segs)) return st;
    P.L.mqdt = 1;
    P.L.fnumin = fnumin;
    Work &w = ctx->sync.w;
    const Lay &L = P.L;
    launch_fill_int(s, w.status, m, 0);
    launch_openlist(s, L, w.tab, w.pwi, w.E, w.nopen, w.openidx, w.openpos, w.colpos, w.openflag);
    launch_asym(s, L, w.tab, w.pwi, w.E, o.thr_guard, w.fg, w.status);
    stage_R(ctx, P, w, o, s);
    stage_K(P, w, s);
    launch_finalize(s, L, w.tab, w.pwi, w.status, nullptr, w.Kw, nullptr);
    HIPCHK(hipMemcpy2DAsync(Ku + (size_t)e0 * n * n, sizeof(double) * n, w.Kw, sizeof(double) * L.ldk,
                            sizeof(double) * n, (size_t)m * n, kK, s));
    if (Xp) {
      launch_zs_setup(s, L, w.nopen, w.Kw, w.aug, w.gre, w.gim, w.dims);
      launch_zs_inverse(s, L, w.dims, w.aug, w.gre, w.gim, w.linv, w.status);
      HIPCHK(hipMemcpy2DAsync(Xp + (size_t)e0 * n * n, sizeof(double) * n, w.aug, sizeof(double) * L.ldaug,
                              sizeof(double) * n, (size_t)m * n, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpy2DAsync(Yp + (size_t)e0 * n * n, sizeof(double) * n, w.aug + L.roff, sizeof(double) * L.ldaug,
                              sizeof(double) * n, (size_t)m * n, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(nmember + e0, w.nopen, sizeof(int) * m, kS, s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kS, s));
    HIPCHK(hipGetLastError());
  }
  return RM_OK;
}

}  // namespace

extern "C" {

static rm_status rm_mqdt_unphysical_K_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, double fnumin,
                                           const rm_opts *opts, double *Ku, int32_t *nmember, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !Ku || !nmember || !status))) return RM_E_ARG;
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  if (rm_status st = mqdt_check(ctx, pw, fnumin)) return st;
  if (ne == 0) return RM_OK;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  if (rm_status st = mqdt_coarse(ctx, pw, E, ne, o, fnumin, Ku, kind_out(o), nmember, status, kind_out(o))) return st;
  return staged_leave(ctx, o, ev);
}

void rm_mqdt_opts_default(rm_mqdt_opts *o) {
  if (!o) return;
  o->ieq = 1;
  o->iqdt = 1;
  o->fnumin = 0.0;
  o->qetest = 1e-7;
}

static rm_status rm_run_mqdt_body(rm_ctx *ctx, int32_t pwid, const double *E, int32_t ne, const rm_mqdt_opts *mq,
                                  const rm_opts *opts, double *omega, double *K, int8_t *coarse, int32_t *status) {
  if (!ctx || ne < 0 || (ne > 0 && (!E || !omega || !status))) return RM_E_ARG;
  rm_mqdt_opts q;
  rm_mqdt_opts_default(&q);
  if (mq) q = *mq;
  const int ieq = q.ieq, iqdt = q.iqdt;
  const double fnumin = q.fnumin;
  if (ieq < 1 || (iqdt != 1 && iqdt != 2) || !(q.qetest >= 0) || !std::isfinite(q.qetest)) {
    ctx->err = "rm_run_mqdt: ieq >= 1, iqdt 1 or 2 and a finite qetest >= 0 are needed";
    return RM_E_ARG;
  }
  const DevPW *pw;
  if (rm_status st = get_pw(ctx, pwid, &pw)) return st;
  if (rm_status st = mqdt_check(ctx, pw, fnumin)) return st;
  if (ne == 0) return RM_OK;
  (void)hipSetDevice(ctx->device);
  const rm_opts o = fixed_opts(opts);
  hipEvent_t ev;
  if (rm_status st = staged_enter(ctx, o, ev)) return st;
  const hipStream_t s = ctx->sync.stream;
  const int n = pw->n, nt = pw->nt;
  DevTmp tmp;
  // 1. the mesh on the host and the device; member counts and flags
  std::vector<double> hE(ne);
  HIPCHK(hipMemcpyAsync(hE.data(), E, sizeof(double) * ne, o.device_ptrs ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                        s));
  HIPCHK(hipStreamSynchronize(s));
  for (int e = 1; e < ne; ++e)
    if (!(hE[e] > hE[e - 1])) {
      ctx->err = "rm_run_mqdt: the energy mesh must be strictly ascending";
      (void)hipEventDestroy(ev);
      return RM_E_ARG;
    }
  double *dE = tmp.get<double>(ne);
  int *dcnt = tmp.get<int>(2 * (size_t)ne);
  if (!dE || !dcnt) {
    ctx->err = "rm_run_mqdt: device temporaries";
    return RM_E_NOMEM;
  }
  HIPCHK(hipMemcpyAsync(dE, hE.data(), sizeof(double) * ne, hipMemcpyHostToDevice, s));
  launch_mqdt_count(s, pw, dE, ne, fnumin, o.thr_guard, dcnt, dcnt + ne);
  std::vector<int> nm(ne), flag(ne), avoid(ne);
  HIPCHK(hipMemcpyAsync(nm.data(), dcnt, sizeof(int) * ne, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(flag.data(), dcnt + ne, sizeof(int) * ne, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int e = 0; e < ne; ++e) {
    avoid[e] = (flag[e] & MQDT_NEAR_INT) != 0;
    flag[e] &= ~MQDT_NEAR_INT;
  }
  // 2. runs of equal member count (the member set only grows with E) and
  // their coarse points: every ieq-th point from the run's first and the
  // run's last, unflagged and not at an integer nu of a closed member; a run
  // whose coarse candidates all fail that has every such point coarse
  std::vector<int> run0(ne), run1(ne);
  std::vector<char> isc(ne, 0);
  for (int s0 = 0; s0 < ne;) {
    int s1 = s0 + 1;
    while (s1 < ne && nm[s1] == nm[s0]) ++s1;
    bool any = false;
    for (int j = s0; j < s1; ++j) {
      run0[j] = s0;
      run1[j] = s1;
      if (((j - s0) % ieq == 0 || j == s1 - 1) && !flag[j] && !avoid[j]) isc[j] = 1, any = true;
    }
    if (!any)
      for (int j = s0; j < s1; ++j)
        if (!flag[j] && !avoid[j]) isc[j] = 1;
    s0 = s1;
  }
  std::vector<int> cpos(ne, -1);
  std::vector<double> cE;
  for (int e = 0; e < ne; ++e)
    if (isc[e]) {
      cpos[e] = (int)cE.size();
      cE.push_back(hE[e]);
    }
  const int nc = (int)cE.size();
  // 3. unphysical K at the coarse points, and Re, Im of (1 - i Ku)^-1 kept on
  // the device (the interpolated quantity: bounded where Ku has a pole)
  const size_t cpl = (size_t)std::max(nc, 1) * n * n;
  double *Kc = tmp.get<double>(cpl), *Xc = tmp.get<double>(cpl), *Yc = tmp.get<double>(cpl);
  if (!Kc || !Xc || !Yc) {
    ctx->err = "rm_run_mqdt: device memory for the coarse unphysical K";
    return RM_E_NOMEM;
  }
  std::vector<int32_t> cnm(nc), cst(nc);
  if (nc) {
    rm_opts oc = o;
    oc.device_ptrs = 0;
    if (rm_status st = mqdt_coarse(ctx, pw, cE.data(), nc, oc, fnumin, Kc, hipMemcpyDeviceToDevice, cnm.data(),
                                   cst.data(), hipMemcpyDeviceToHost, Xc, Yc))
      return st;
    HIPCHK(hipStreamSynchronize(s));
  }
  // energy at which each point's interpolant is evaluated (qetest): walking
  // each run, a point within qetest z^2 of the last point evaluated at its own
  // energy reuses that energy; coarse points are their own
  std::vector<double> hEv(ne);
  {
    const double tol = q.qetest * pw->z * pw->z;
    double last = 0.0;
    bool have = false;
    for (int e = 0; e < ne; ++e) {
      if (e == 0 || nm[e] != nm[e - 1]) have = false;
      if (!isc[e] && have && std::fabs(hE[e] - last) <= tol) {
        hEv[e] = last;
      } else {
        hEv[e] = hE[e];
        if (!flag[e]) last = hE[e], have = true;
      }
    }
  }
  // 4. stencils: the four coarse points of the run around each point (window
  // from the coarse point before the last one at or below it, clamped to the
  // run), Lagrange weights, and the flags of the point and of its coarse points
  std::vector<int> hc(4 * (size_t)ne, -1);
  std::vector<double> hw(4 * (size_t)ne, 0.0);
  std::vector<int> st0(ne);
  for (int e = 0; e < ne; ++e) {
    int st = flag[e];
    if (!st) {
      std::vector<int> cl;
      for (int j = run0[e]; j < run1[e]; ++j)
        if (isc[j]) cl.push_back(j);
      const int m = (int)cl.size();
      int k = 0;
      for (int q = 0; q < m; ++q)
        if (cl[q] <= e) k = q;
      if (m == 0) st |= RM_PT_NOCONV;  // a run without a usable coarse point
      const int w = std::min(m, 4);
      const int a0 = std::max(0, std::min(k - 1, m - w));
      for (int q = 0; q < w; ++q) {
        const int cq = cl[a0 + q];
        double wt = 1.0;
        for (int r = 0; r < w; ++r)
          if (r != q) wt *= (hEv[e] - hE[cl[a0 + r]]) / (hE[cq] - hE[cl[a0 + r]]);
        hc[4 * e + q] = cpos[cq];
        hw[4 * e + q] = wt;
        st |= cst[cpos[cq]];
      }
    }
    st0[e] = st;
  }
  if (coarse) {
    std::vector<int8_t> c8(isc.begin(), isc.end());
    HIPCHK(hipMemcpyAsync(coarse, c8.data(), ne, kind_out(o) == hipMemcpyDeviceToDevice ? hipMemcpyHostToDevice
                                                                                       : hipMemcpyHostToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
  }
  int *dci = tmp.get<int>(4 * (size_t)ne + ne);
  double *dcw = tmp.get<double>(4 * (size_t)ne);
  const int cap = staged_cap(ctx, pw, ne);
  const long ldo = n;
  int *dsys = tmp.get<int>(2 * (size_t)cap * ldo + cap);
  double *dtan = tmp.get<double>((size_t)cap * ldo);
  if (!dci || !dcw || !dsys || !dtan) {
    ctx->err = "rm_run_mqdt: device temporaries";
    return RM_E_NOMEM;
  }
  // Omega only, iqdt = 1 and at most MQDT_SMAX closed members at every point:
  // the closed members are eliminated in S form (no K is formed)
  bool sroute = iqdt == 1 && !K;
  if (sroute) {
    std::vector<double> thr;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      auto it = ctx->hthr.find(pw);
      if (it != ctx->hthr.end()) thr = it->second;
    }
    if (thr.size() != (size_t)n) sroute = false;
    for (int e = 0; e < ne && sroute; ++e) {
      int no = 0;
      for (double tv : thr) no += hE[e] - tv > 0.0;
      if (!flag[e] && nm[e] - no > MQDT_SMAX) sroute = false;
    }
  }
  int *dlist = nullptr;
  double *dW = nullptr, *dZ = nullptr;
  if (sroute) {
    dlist = tmp.get<int>(3 * (size_t)cap * ldo);
    dW = tmp.get<double>(2 * (size_t)cap * MQDT_SMAX * MQDT_SMAX);
    dZ = tmp.get<double>(2 * (size_t)cap * ldo * MQDT_SMAX);
    if (!dlist || !dW || !dZ) {
      ctx->err = "rm_run_mqdt: device temporaries";
      return RM_E_NOMEM;
    }
  }
  HIPCHK(hipMemcpyAsync(dci, hc.data(), sizeof(int) * 4 * ne, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dci + 4 * (size_t)ne, st0.data(), sizeof(int) * ne, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dcw, hw.data(), sizeof(double) * 4 * ne, hipMemcpyHostToDevice, s));
  // 5. the fine mesh in chunks: interpolate, eliminate the closed members
  // through the batched LU, then S and Omega as in the physical path
  for (int e0 = 0; e0 < ne; e0 += cap) {
    const int m = std::min(cap, ne - e0);
    Plan P;
    std::vector<Seg> segs;
    if (rm_status st = staged_chunk(ctx, pw, E, e0, m, o, false, P, segs)) return st;
    Work &w = ctx->sync.w;
    const Lay &L = P.L;
    Lay Lq = L;
    Lq.mqdt = 1;
    Lq.fnumin = fnumin;
    int *syspos = dsys, *spos = dsys + (size_t)cap * ldo, *nsys = dsys + 2 * (size_t)cap * ldo;
    HIPCHK(hipMemcpyAsync(w.status, dci + 4 * (size_t)ne + e0, sizeof(int) * m, hipMemcpyDeviceToDevice, s));
    launch_openlist(s, L, w.tab, w.pwi, w.E, w.nopen, w.openidx, w.openpos, w.colpos, w.openflag);
    if (sroute) {
      int *clist = dlist, *olist = dlist + (size_t)cap * ldo, *cch = dlist + 2 * (size_t)cap * ldo;
      launch_mqdt_setup_lists(s, Lq, w.tab, w.pwi, w.E, o.thr_guard, syspos, spos, dtan, w.dims, nsys, w.status,
                              clist, olist, cch);
      launch_mqdt_sform(s, L, w.tab, w.pwi, w.E, nsys, w.nopen, clist, olist, cch, Xc, Yc, dci + 4 * (size_t)e0,
                        dcw + 4 * (size_t)e0, w.status, dW, dW + (size_t)cap * MQDT_SMAX * MQDT_SMAX, dZ,
                        dZ + (size_t)cap * ldo * MQDT_SMAX, w.aug);
      launch_omega(s, L, w.tab, w.pwi, w.openpos, w.nopen, w.aug, w.aug + L.roff, w.omega, nullptr);
      launch_finalize(s, L, w.tab, w.pwi, w.status, w.omega, nullptr, nullptr);
      HIPCHK(hipMemcpyAsync(omega + (size_t)e0 * nt * nt, w.omega, sizeof(double) * m * nt * nt, kind_out(o), s));
      HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
      HIPCHK(hipGetLastError());
      continue;
    }
    launch_mqdt_setup(s, Lq, w.tab, w.pwi, w.E, o.thr_guard, syspos, spos, dtan, w.dims, nsys, w.status);
    if (iqdt == 1) {
      // Ku = Y X^-1 from the interpolated X, Y: [X | Y] solved in full, transposed into Kw
      launch_mqdt_interp(s, L, 1, w.tab, w.pwi, spos, nsys, Xc, Yc, dci + 4 * (size_t)e0, dcw + 4 * (size_t)e0,
                         w.status, w.dims, w.aug, w.Kw);
      launch_lu_solve(s, L.ne, L.nmax, L.nmax, w.dims, w.aug, L.ldaug, L.sA, L.roff, w.ipiv, L.ldo, w.bperm, w.linv,
                      0, w.status);
      launch_mqdt_take(s, L, nsys, w.aug, w.Kw);
    } else {
      // the interpolated Ku itself, into Kw
      launch_mqdt_interp(s, L, 2, w.tab, w.pwi, spos, nsys, Kc, nullptr, dci + 4 * (size_t)e0, dcw + 4 * (size_t)e0,
                         w.status, w.dims, w.aug, w.Kw);
    }
    // closed members eliminated: the tail of the block system is K
    launch_mqdt_build(s, L, w.tab, w.pwi, syspos, spos, dtan, w.nopen, nsys, w.Kw, w.status, w.dims, w.aug);
    launch_lu_solve(s, L.ne, L.nmax, L.nmax, w.dims, w.aug, L.ldaug, L.sA, L.roff, w.ipiv, L.ldo, w.bperm, w.linv, 1,
                    w.status);
    launch_mqdt_gather(s, L, nsys, w.nopen, w.aug, w.Kw, w.dims);
    stage_SO(P, w, false, s);
    launch_finalize(s, L, w.tab, w.pwi, w.status, w.omega, K ? w.Kw : nullptr, nullptr);
    HIPCHK(hipMemcpyAsync(omega + (size_t)e0 * nt * nt, w.omega, sizeof(double) * m * nt * nt, kind_out(o), s));
    if (K)
      HIPCHK(hipMemcpy2DAsync(K + (size_t)e0 * n * n, sizeof(double) * n, w.Kw, sizeof(double) * L.ldk,
                              sizeof(double) * n, (size_t)m * n, kind_out(o), s));
    HIPCHK(hipMemcpyAsync(status + e0, w.status, sizeof(int) * m, kind_out(o), s));
    HIPCHK(hipGetLastError());
  }
  // the temporaries are freed on return: the work that reads them completes first
  HIPCHK(hipStreamSynchronize(s));
  return staged_leave(ctx, o, ev);
}

}  // extern "C"

// ===================================================== C ABI entry points
// Each forwards to its body above; an exception never crosses into a C caller.
extern "C" {

rm_status rm_create(int device, size_t hbm_budget_bytes, rm_ctx **out) {
  try {
    return rm_create_body(device, hbm_budget_bytes, out);
  } catch (...) {
    return abi_failed_create(device);
  }
}

rm_status rm_destroy(rm_ctx *ctx) {
  try {
    return rm_destroy_body(ctx);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_pw_upload(rm_ctx *ctx, const rm_pw_desc *desc, int32_t *pw_id) {
  try {
    return rm_pw_upload_body(ctx, desc, pw_id);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_pw_release(rm_ctx *ctx, int32_t pw_id) {
  try {
    return rm_pw_release_body(ctx, pw_id);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_pw_upload_coupled(rm_ctx *ctx, const rm_pw_desc *desc, int32_t lamax, const double *cf, double r1,
                               int32_t *pw_id) {
  try {
    return rm_pw_upload_coupled_body(ctx, desc, lamax, cf, r1, pw_id);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_set_propagation(rm_ctx *ctx, int32_t npts, int32_t stab) {
  try {
    return rm_set_propagation_body(ctx, npts, stab);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_propagate(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts, double *phi,
                       double *dphi, int32_t *status) {
  try {
    return rm_propagate_body(ctx, pw, E, ne, opts, phi, dphi, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_mqdt_unphysical_K(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, double fnumin, const rm_opts *opts,
                               double *Ku, int32_t *nmember, int32_t *status) {
  try {
    return rm_mqdt_unphysical_K_body(ctx, pw, E, ne, fnumin, opts, Ku, nmember, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_run_mqdt(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_mqdt_opts *mq, const rm_opts *opts,
                      double *omega, double *K, int8_t *coarse, int32_t *status) {
  try {
    return rm_run_mqdt_body(ctx, pw, E, ne, mq, opts, omega, K, coarse, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_form_R(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts, double *R,
                    int32_t *status) {
  try {
    return rm_form_R_body(ctx, pw, E, ne, opts, R, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_asymptotic(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts, double *fg,
                        int8_t *open, int32_t *nopen, int32_t *status) {
  try {
    return rm_asymptotic_body(ctx, pw, E, ne, opts, fg, open, nopen, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_solve_K(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const double *R, const double *fg,
                     const rm_opts *opts, double *K, int32_t *status) {
  try {
    return rm_solve_K_body(ctx, pw, E, ne, R, fg, opts, K, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_collision_strengths(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const double *K,
                                 const rm_opts *opts, double *omega, double *S, int32_t *status) {
  try {
    return rm_collision_strengths_body(ctx, pw, E, ne, K, opts, omega, S, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_run(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts, double *omega, double *K,
                 int32_t *status) {
  try {
    return rm_run_body(ctx, pw, E, ne, opts, omega, K, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_run_noalloc(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts, double *omega,
                         double *K, int32_t *status) {
  try {
    return rm_run_noalloc_body(ctx, pw, E, ne, opts, omega, K, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_run_batch(rm_ctx *ctx, const rm_batch_item *items, int32_t nitems, const rm_opts *opts) {
  try {
    return rm_run_batch_body(ctx, items, nitems, opts);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_set_graph(rm_ctx *ctx, int32_t on) {
  try {
    return rm_set_graph_body(ctx, on);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_graph_stats(rm_ctx *ctx, int64_t *captures, int64_t *replays) {
  try {
    return rm_graph_stats_body(ctx, captures, replays);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_run_sum(rm_ctx *ctx, const int32_t *pw_ids, int32_t npw, const double *E, int32_t ne, int32_t order,
                     const rm_opts *opts, double *omega, int32_t *status) {
  try {
    return rm_run_sum_body(ctx, pw_ids, npw, E, ne, order, opts, omega, status);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_tile_shape(int32_t prec, int32_t shape, int32_t *tile, int32_t *energies) {
  try {
    return rm_tile_shape_body(prec, shape, tile, energies);
  } catch (...) {
    return abi_failed(nullptr);
  }
}

rm_status rm_get_tile(rm_ctx *ctx, int32_t prec, int32_t bucket, int32_t *shape) {
  try {
    return rm_get_tile_body(ctx, prec, bucket, shape);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_set_tile(rm_ctx *ctx, int32_t prec, int32_t bucket, int32_t shape) {
  try {
    return rm_set_tile_body(ctx, prec, bucket, shape);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_tune(rm_ctx *ctx, int32_t prec, const int32_t *pw_ids, int32_t npw, const double *E, int32_t ne,
                  int32_t reps, const char *cache_path, double *ms) {
  try {
    return rm_tune_body(ctx, prec, pw_ids, npw, E, ne, reps, cache_path, ms);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_tune_load(rm_ctx *ctx, const char *cache_path) {
  try {
    return rm_tune_load_body(ctx, cache_path);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_submit(rm_ctx *ctx, const rm_request *req, uint64_t *ticket) {
  try {
    return rm_submit_body(ctx, req, ticket);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_poll(rm_ctx *ctx, uint64_t ticket, rm_req_stats *st) {
  try {
    return rm_poll_body(ctx, ticket, st);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_drain(rm_ctx *ctx) {
  try {
    return rm_drain_body(ctx);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_prof_enable(rm_ctx *ctx, int32_t on) {
  try {
    return rm_prof_enable_body(ctx, on);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_prof_read(rm_ctx *ctx, const char *stage, double *total_ms, int64_t *launches, int64_t *energies) {
  try {
    return rm_prof_read_body(ctx, stage, total_ms, launches, energies);
  } catch (...) {
    return abi_failed(ctx);
  }
}

rm_status rm_prof_chunks(rm_ctx *ctx, int64_t cap, double *ms, double *model_flops, double *open_frac,
                         int64_t *energies, int64_t *count) {
  try {
    return rm_prof_chunks_body(ctx, cap, ms, model_flops, open_frac, energies, count);
  } catch (...) {
    return abi_failed(ctx);
  }
}

}  // extern "C"
