// C ABI of the TEM library (include/tem.h): context, validation and the
// orchestration of the device kernels in tem_kernels.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/tem.h"
#include "tem_internal.h"

using tem::GridArgs;
using tem::SolveState;
// the pinned head buffer holds two heads (two solver blocks in flight)
constexpr size_t kHeadStride = 4096;
static_assert(sizeof(tem::SolveHead) <= kHeadStride, "pinned head buffer");

// Device memory of tem_apply_noalloc: a fixed array in the code object, one
// copy per GPU the library is loaded on, held until the process ends.  Its
// host-side name is only a stand-in: host code uses the device address that
// hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t kNoAllocScratchBytes = 64ull << 20;  // 64 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_global_error;

// Per-device address of `scratch`, looked up once per device with that device
// current (each GPU holds its own copy of the array at its own address).
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  *out = p;
  return hipSuccess;
}
// Adjoint by one multi-shift solve per receiver row up to this many receivers
// (about n_rx seed sweeps); beyond it one batched COCG over the J shifted
// systems (about J complex solves).  Measured on the 64^3 differentiation
// workload (30 receivers, J = 22): the rows took 364 s (12.1 s each, four at
// a time); the COCG had not finished after 1044 s (6 of 22 systems still
// active at 490k iterations), so the rows are cheaper below 1044 / 12.1 = 86
// receivers at least.
constexpr int kAdjointMultishiftMaxRx = 86;
// precision 1: the sweep (FP64 iterates y_j, complex FP32 directions p_j) stops
// at the recursive tolerance kSweepTolFP32, below the M-norm error that the
// FP32 directions leave (a few 1e-8); FP64 residual refinement then drives
// every shift to the requested rtol (default kRefineTarget) on its FP64
// residual, each pass reducing the correction system's residual by
// kRefinePassTol.  The FP32 rounding noise of the stiff (air) modes dominates
// that residual: each pass cuts it about 100x, down to a floor near 1e-6 on
// grids with 1e-8 S/m air, where FP32 corrections stop helping.
constexpr double kSweepTolFP32 = 1e-10;
constexpr double kRefineTarget = 1e-5;
constexpr double kRefinePassTol = 1e-2;
constexpr int kRefinePassCap = 8192;  // COCG iterations per shift in one refinement pass
constexpr int kRefineStall = 1024;    // ... and without a 10% residual reduction

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Up to this many independent multi-shift solves (loop sources of a forward
// call, receiver rows of an adjoint) run at once, each on its own stream: the
// seed kernels of one solve are latency-bound, and concurrent solves fill the
// device between each other's reduction boundaries.
constexpr int kMaxConcurrentSolves = 4;
constexpr int kMaxSinglePoles = 32;  // pole representatives of a single-time approximant

// Workspace of one multi-shift solve.
struct SolveSlot {
  DevBuf R, pbuf, q, partials, gvec, P;  // ring, seed p (2), q, partial sums, g, per-shift p_j
  tem::SolveState* d_state = nullptr;
  void* head = nullptr;          // pinned copies of the solver head, one per block in flight
  hipStream_t stream = nullptr;  // library-owned, default priority
  hipStream_t stream2 = nullptr; // block updates overlapped with the next blocks' seed iterations
  hipEvent_t ev = nullptr;       // orders the library stream after this slot
  hipEvent_t head_ev[2] = {nullptr, nullptr};  // head copy of block b done (b mod 2)
  hipEvent_t sb_ev[tem::kPhases] = {};         // shift recurrences of block b done (b mod 3)
  hipEvent_t bu_ev[tem::kPhases] = {};         // block update of block b done (b mod 3)
};

}  // namespace

struct tem_ctx {
  int device = 0;
  tem_engine* engine = nullptr;     // solve engine the multi-shift solves are submitted to (or none)
  hipStream_t stream = nullptr;       // caller's stream (may be the null stream)
  hipStream_t work = nullptr;         // library-owned stream: every kernel runs here
  hipEvent_t order_ev = nullptr;      // orders work after the caller's stream
  hipEvent_t done_ev = nullptr;       // orders the caller's stream after work (stream-ordered calls)
  void* scratch = nullptr;            // this device's address of the fixed no-allocation array
  int nx = 0, ny = 0, nz = 0, ks = 0;
  std::vector<double> hx, hy, hz;
  GridArgs g{};
  long long n3 = 0, nstore = 0, nunk = 0;
  // operator data
  double* d_axis = nullptr;  // 9 arrays of length max(n)+1
  double* d_sigma = nullptr;
  double* d_mass = nullptr;
  double* d_dinv = nullptr;
  double* d_sqrtm = nullptr;
  bool has_sigma = false;
  // solver workspace
  std::vector<SolveSlot> slots;
  hipEvent_t work_ev = nullptr;       // orders the slot streams after the library stream
  unsigned int* d_counters = nullptr;
  DevBuf gc, f, P, C, rx, data, res, cpart, sh;
  DevBuf refine, cst, cocg_part;       // precision 1: refinement COCG vectors and state
  DevBuf refine64, refdot;             // precision 1: FP64 corrections d_j and (A + s_j) d_j; step lengths
  std::vector<DevBuf> Y;  // per source (kept) or one
  // stored forward state for the adjoint
  bool seed_one_kernel = true;  // seed CG form (seed_one_kernel_for)
  bool engine_batches = false;  // solves go to an attached engine (uses_engine)
  bool fwd_meta = false;   // the last forward's sources, receivers, poles and options are recorded
  bool fwd_valid = false;  // ... and its solutions are kept on the device
  int fwd_J = 0, fwd_T = 0, fwd_nsrc = 0, fwd_nrx = 0;
  double fwd_s0 = 0.0;
  std::vector<double> fwd_xi, fwd_c;
  std::vector<tem_receiver> fwd_rx;
  std::vector<tem_loop> fwd_src;
  tem_solve_opts fwd_opts{};
  std::string err;
  // kernel timing (opts.profile)
  double prof_ms[4] = {0, 0, 0, 0};
  long long prof_n[4] = {0, 0, 0, 0};
};

namespace {

// Overlap of each block's deferred update with the next block's seed
// iterations (second stream per solve), TEM_OVERLAP=1.  Off by default: at
// 64^3 the concurrent update slowed the latency-bound seed kernels by more
// than it hid (5.90 s against 5.78 s per model, same box).
// TEM_OVERLAP_BLOCKS caps the overlapped update's workgroups.
bool overlap_updates() {
  static const bool v = [] {
    const char* e = getenv("TEM_OVERLAP");
    return e && *e == '1';
  }();
  return v;
}
int overlap_blocks() {
  static const int v = [] {
    const char* e = getenv("TEM_OVERLAP_BLOCKS");
    const int b = e ? atoi(e) : 0;
    return b > 0 ? b : 4096;
  }();
  return v;
}

// Seed CG form of a context's solves, fixed when the context is created: one
// kernel per iteration (the update fused with the next stencil, on unscaled
// vectors M^-1/2 v) when its tiles fit on the device's compute units in one
// round, else the two-kernel stencil + update form.  With one tile per CU
// the iteration is a chain of latencies and one kernel saves a launch and a
// round trip (64^3: 5.14 s against 5.60 s per model); with several rounds
// of tiles the two-plane tile's 2 waves per SIMD hide less than the
// two-kernel form's stencil at 4 waves per SIMD plus a streaming update
// (128^3: 169 us against 148 us per iteration).  TEM_SEED=hs or =one forces
// a form.  The batched engine, whose jobs fill the device together, uses the
// two-kernel form.
// Whether a context's FP64 multi-shift solves go to its attached engine:
// only when one solve's tiles leave compute units idle (32^3, 48^3 here),
// where sharing launches with other solves fills the device.  A solve that
// fills the device alone runs faster on its own streams: 30 adjoint receiver
// rows at 64^3 took 557 s as 16 batched jobs of the engine's two-kernel
// iteration, 364 s as four concurrent one-kernel solves.
bool uses_engine(const tem_ctx* ctx) { return ctx->engine != nullptr && ctx->engine_batches; }

bool seed_one_kernel_for(const GridArgs& g, int n_cu) {
  const char* e = getenv("TEM_SEED");
  if (e && !strcmp(e, "hs")) return false;
  if (e && !strcmp(e, "one")) return true;
  return n_cu > 0 && tem::seed_step_blocks(g) <= n_cu;
}

// TEM_VERBOSE=1: progress lines on stderr from long solves
bool verbose() {
  static const bool v = [] {
    const char* e = getenv("TEM_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

int fail(tem_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_global_error = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, TEM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

int ensure(tem_ctx* ctx, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return TEM_OK;
  if (b.p) {
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, TEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  if (hipMemsetAsync(b.p, 0, bytes, ctx->work) != hipSuccess)
    return fail(ctx, TEM_EHIP, "hipMemsetAsync failed");
  b.bytes = bytes;
  return TEM_OK;
}

void release(DevBuf& b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

bool finite_pos(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!(std::isfinite(a[i]) && a[i] > 0.0)) return false;
  return true;
}

long long node_index(const tem_ctx* c, int i, int j, int k) {
  return ((long long)k * (c->ny + 1) + j) * (c->nx + 1) + i;
}

// Source vector f_e = I l_e (+-1) on the loop edges, node-padded layout.
void loop_source(const tem_ctx* c, const tem_loop& L, std::vector<double>& f) {
  const long long nn = c->g.nn;
  std::fill(f.begin(), f.end(), 0.0);
  for (int i = L.i0; i < L.i1; ++i) {
    f[0 * nn + node_index(c, i, L.j0, c->ks)] += L.current * c->hx[i];
    f[0 * nn + node_index(c, i, L.j1, c->ks)] -= L.current * c->hx[i];
  }
  for (int j = L.j0; j < L.j1; ++j) {
    f[1 * nn + node_index(c, L.i1, j, c->ks)] += L.current * c->hy[j];
    f[1 * nn + node_index(c, L.i0, j, c->ks)] -= L.current * c->hy[j];
  }
}

// Receiver row q (dB_z/dt = q . u) in the node-padded layout: minus the
// circulation around the surface z-face of column (i, j) over its area.
void receiver_row(const tem_ctx* c, const tem_receiver& r, std::vector<double>& q) {
  const long long nn = c->g.nn;
  std::fill(q.begin(), q.end(), 0.0);
  const double hx = c->hx[r.i], hy = c->hy[r.j], inva = -1.0 / (hx * hy);
  q[0 * nn + node_index(c, r.i, r.j, c->ks)] += hx * inva;
  q[1 * nn + node_index(c, r.i + 1, r.j, c->ks)] += hy * inva;
  q[0 * nn + node_index(c, r.i, r.j + 1, c->ks)] -= hx * inva;
  q[1 * nn + node_index(c, r.i, r.j, c->ks)] -= hy * inva;
}

int check_loops(tem_ctx* ctx, const tem_loop* src, int n_src) {
  if (n_src < 1 || src == nullptr) return fail(ctx, TEM_EINVAL, "need at least one loop source");
  for (int s = 0; s < n_src; ++s) {
    const tem_loop& L = src[s];
    if (!(0 < L.i0 && L.i0 < L.i1 && L.i1 < ctx->nx && 0 < L.j0 && L.j0 < L.j1 && L.j1 < ctx->ny))
      return fail(ctx, TEM_EINVAL, "loop " + std::to_string(s) + " is not on interior node lines");
    if (!std::isfinite(L.current) || L.current == 0.0)
      return fail(ctx, TEM_EINVAL, "loop current must be finite and nonzero");
  }
  return TEM_OK;
}

// Make the library stream wait for everything already queued on the caller's stream.
int order_after_caller(tem_ctx* ctx) {
  HIPCHK(ctx, hipEventRecord(ctx->order_ev, ctx->stream));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->work, ctx->order_ev, 0));
  return TEM_OK;
}

tem_solve_opts resolve_opts(const tem_solve_opts* o) {
  tem_solve_opts r{};
  if (o) r = *o;
  if (!(r.rtol > 0.0)) r.rtol = r.precision == 1 ? kRefineTarget : 1e-12;
  if (r.max_iter <= 0) r.max_iter = 2000000;
  if (r.block <= 0) r.block = 64;
  if (r.refine_max <= 0) r.refine_max = 8;
  return r;
}

// the compiled block lengths
int block_length(int requested) {
  return requested >= 64 ? 64 : requested >= 32 ? 32 : requested >= 16 ? 16 : 8;
}

// Create solve slots 0..n-1 (stream, state, pinned head) if they do not exist.
int ensure_slots(tem_ctx* ctx, int n) {
  while ((int)ctx->slots.size() < n) {
    ctx->slots.emplace_back();
    SolveSlot& sl = ctx->slots.back();
    HIPCHK(ctx, hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    HIPCHK(ctx, hipStreamCreateWithFlags(&sl.stream2, hipStreamNonBlocking));
    HIPCHK(ctx, hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    for (hipEvent_t& e : sl.sb_ev) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t& e : sl.bu_ev) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(ctx, hipMalloc(&sl.d_state, sizeof(SolveState)));
    HIPCHK(ctx, hipHostMalloc(&sl.head, 2 * kHeadStride, hipHostMallocDefault));
    for (hipEvent_t& e : sl.head_ev) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  return TEM_OK;
}

void release_slot(SolveSlot& sl) {
  for (DevBuf* b : {&sl.R, &sl.pbuf, &sl.q, &sl.partials, &sl.gvec, &sl.P}) release(*b);
  if (sl.d_state) (void)hipFree(sl.d_state);
  if (sl.head) (void)hipHostFree(sl.head);
  if (sl.ev) (void)hipEventDestroy(sl.ev);
  for (hipEvent_t e : sl.head_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : sl.sb_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : sl.bu_ev)
    if (e) (void)hipEventDestroy(e);
  if (sl.stream2) (void)hipStreamDestroy(sl.stream2);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
}

// ---------------------------------------------------------------------------
// Solve engine: one worker thread per engine advances the multi-shift solves
// submitted by every attached context (the loop sources and adjoint receiver
// rows of all admitted requests) together, 64 seed iterations at a time, as a
// HIP graph of batched launches: per iteration one seed stencil launch and one
// seed update launch cover every job's tiles, then one shift-block and one
// block-update launch cover every job's shifts.  Jobs join at block
// boundaries (their seed initialisation is queued before the next block) and
// leave when all their shifts have converged; the graph is rebuilt when the
// set of jobs changes.  Two blocks stay in flight: the worker reads the heads
// of block b while block b+1 runs.  The poles are independent work (Sec. 5.3
// parallelizes over them across processes); here the poles of several
// requests share every launch.
// ---------------------------------------------------------------------------
struct EngineJob {
  tem_ctx* ctx = nullptr;
  int slot = 0;
  double2* Y = nullptr;
  int J = 0;
  double s0 = 0.0;
  int max_iter = 0;
  std::unique_ptr<SolveState> init;    // initial device state (host copy)
  hipEvent_t ready = nullptr;          // right-hand side and buffers ready (context stream)
  hipEvent_t done = nullptr;           // every block of this job and its final state copy done (engine stream)
  SolveState* final_state = nullptr;   // pinned
  int checked = 0;                     // blocks whose head the worker has read
  int k = 0;                           // seed iterations of those blocks
  bool breakdown = false;
  bool retired = false;                // worker: no longer in the batch
  bool finished = false;               // guarded by the engine mutex
};

}  // namespace

struct tem_engine {
  int device = 0;
  int max_jobs = tem::kMaxBatchJobs;
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;       // wakes the worker: new jobs or stop
  std::condition_variable done_cv;  // wakes submitters: a job finished
  std::deque<EngineJob*> pending;
  bool stop = false;
  hipError_t error = hipSuccess;    // first HIP failure of the worker; every job then fails
  static constexpr int kGens = 4;   // job tables in flight (a table is reused 4 generations later)
  tem::BatchJob* d_tables = nullptr;
  tem::BatchJob* h_tables = nullptr;  // pinned staging of the tables
  tem::SolveHead* d_heads = nullptr;
  tem::SolveHead* h_heads = nullptr;  // pinned, one set per block in flight
  hipEvent_t head_ev[2] = {nullptr, nullptr};
  // statistics (guarded by mu)
  long long blocks = 0, job_blocks = 0;
  int max_jobs_seen = 0, max_ctx_seen = 0;
};

namespace {

constexpr int kEngineBlock = 64;  // seed iterations per batched block

void engine_worker(tem_engine* E) {
  (void)hipSetDevice(E->device);
  constexpr int B = kEngineBlock;
  struct Gen {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<EngineJob*> jobs;
    ~Gen() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
    }
  };
  std::vector<EngineJob*> active;
  std::deque<std::pair<int, std::shared_ptr<Gen>>> inflight;
  std::shared_ptr<Gen> cur;
  int next_table = 0, parity = 0;
  bool dirty = true;
  hipError_t err = hipSuccess;
  const auto t_start = std::chrono::steady_clock::now();
  double next_report = 10.0;
  long long blocks_done = 0;
  auto finish = [&](EngineJob* jb) {
    // queued after every block issued so far, which includes the job's last one
    SolveSlot& sl = jb->ctx->slots[jb->slot];
    if (err == hipSuccess)
      err = hipMemcpyAsync(jb->final_state, sl.d_state, sizeof(SolveState), hipMemcpyDeviceToHost, E->stream);
    if (err == hipSuccess) err = hipEventRecord(jb->done, E->stream);
    jb->retired = true;
    active.erase(std::remove(active.begin(), active.end(), jb), active.end());
    dirty = true;
    std::lock_guard<std::mutex> lk(E->mu);
    jb->finished = true;
  };
  for (;;) {
    std::vector<EngineJob*> fresh;
    {
      std::unique_lock<std::mutex> lk(E->mu);
      E->cv.wait(lk, [&] { return E->stop || !E->pending.empty() || !active.empty() || !inflight.empty(); });
      if (E->stop && E->pending.empty() && active.empty() && inflight.empty()) break;
      while (!E->pending.empty() && (int)active.size() + (int)fresh.size() < E->max_jobs) {
        fresh.push_back(E->pending.front());
        E->pending.pop_front();
      }
      if (err != hipSuccess) E->error = err;
    }
    if (err != hipSuccess) {
      // fail every job: nothing more is launched
      std::lock_guard<std::mutex> lk(E->mu);
      for (EngineJob* jb : fresh) jb->finished = true;
      for (EngineJob* jb : active) jb->finished = true;
      active.clear();
      inflight.clear();
      E->done_cv.notify_all();
      continue;
    }
    for (EngineJob* jb : fresh) {
      SolveSlot& sl = jb->ctx->slots[jb->slot];
      const size_t n3 = jb->ctx->n3;
      if (err == hipSuccess) err = hipStreamWaitEvent(E->stream, jb->ready, 0);
      if (err == hipSuccess)
        err = hipMemcpyAsync(sl.d_state, jb->init.get(), sizeof(SolveState), hipMemcpyHostToDevice, E->stream);
      if (err == hipSuccess) {
        const tem::Reduce red{(double*)sl.partials.p, jb->ctx->d_counters};
        tem::launch_seed_init(jb->ctx->g, (const double*)sl.gvec.p, (double*)sl.R.p, (double*)sl.pbuf.p + n3, jb->Y,
                              (double2*)sl.P.p, jb->J, red, sl.d_state, E->stream);
        err = hipGetLastError();
      }
      active.push_back(jb);
      dirty = true;
    }
    if (err != hipSuccess) continue;
    if (!active.empty() && inflight.size() < 2) {
      if (dirty) {
        // the batch's job table and graph for the current set of jobs
        auto gen = std::make_shared<Gen>();
        gen->jobs = active;
        const int n = (int)active.size();
        const int slot = next_table;
        next_table = (next_table + 1) % tem_engine::kGens;
        tem::BatchJob* ht = E->h_tables + (size_t)slot * tem::kMaxBatchJobs;
        tem::BatchJob* dt = E->d_tables + (size_t)slot * tem::kMaxBatchJobs;
        int tiles = 0, bus = 0, maxJ = 1;
        for (int i = 0; i < n; ++i) {
          EngineJob* jb = active[i];
          SolveSlot& sl = jb->ctx->slots[jb->slot];
          tem::BatchJob& b = ht[i];
          b = tem::BatchJob{};
          b.g = jb->ctx->g;
          b.dinv = jb->ctx->d_dinv;
          b.s0 = jb->s0;
          b.R = (double*)sl.R.p;
          b.pbuf = (double*)sl.pbuf.p;
          b.q = (double*)sl.q.p;
          b.part_st = (double*)sl.partials.p;
          b.part_up = (double*)sl.partials.p + tem::kReduceSlots;
          b.st = sl.d_state;
          b.Y = jb->Y;
          b.P = (double2*)sl.P.p;
          b.J = jb->J;
          b.tile0 = tiles;
          b.ntiles = tem::batch_tiles(b.g, &b.ntx, &b.nty);
          b.bu0 = bus;
          b.nbu = tem::block_update_blocks(b.g);
          tiles += b.ntiles;
          bus += b.nbu;
          maxJ = std::max(maxJ, jb->J);
        }
        err = hipMemcpyAsync(dt, ht, n * sizeof(tem::BatchJob), hipMemcpyHostToDevice, E->stream);
        if (err == hipSuccess) err = hipGraphCreate(&gen->graph, 0);
        if (err == hipSuccess) {
          tem::Sink k;
          k.graph = gen->graph;
          for (int l = 0; l < B; ++l) {
            tem::launch_seed_stencil_batch(dt, n, tiles, B, l, k);
            tem::launch_seed_update_batch(dt, n, B, l, k);
          }
          tem::launch_shift_block_batch(dt, n, maxJ, k);
          tem::launch_block_update_batch(dt, n, bus, B, k);
          tem::launch_gather_heads(dt, n, E->d_heads, k);
          err = k.err;
        }
        if (err == hipSuccess) err = hipGraphInstantiate(&gen->exec, gen->graph, nullptr, nullptr, 0);
        if (err != hipSuccess) continue;
        cur = gen;
        dirty = false;
      }
      const int n = (int)cur->jobs.size();
      err = hipGraphLaunch(cur->exec, E->stream);
      if (err == hipSuccess)
        err = hipMemcpyAsync(E->h_heads + (size_t)parity * tem::kMaxBatchJobs, E->d_heads,
                             n * sizeof(tem::SolveHead), hipMemcpyDeviceToHost, E->stream);
      if (err == hipSuccess) err = hipEventRecord(E->head_ev[parity], E->stream);
      if (err != hipSuccess) continue;
      inflight.emplace_back(parity, cur);
      parity ^= 1;
      {
        std::lock_guard<std::mutex> lk(E->mu);
        std::vector<const tem_ctx*> ctxs;
        for (EngineJob* jb : cur->jobs)
          if (std::find(ctxs.begin(), ctxs.end(), jb->ctx) == ctxs.end()) ctxs.push_back(jb->ctx);
        ++E->blocks;
        E->job_blocks += n;
        E->max_jobs_seen = std::max(E->max_jobs_seen, n);
        E->max_ctx_seen = std::max(E->max_ctx_seen, (int)ctxs.size());
      }
      continue;
    }
    // read the heads of the oldest block in flight
    const int par = inflight.front().first;
    std::shared_ptr<Gen> gen = inflight.front().second;
    inflight.pop_front();
    err = hipEventSynchronize(E->head_ev[par]);
    if (err != hipSuccess) continue;
    bool any = false;
    for (size_t i = 0; i < gen->jobs.size(); ++i) {
      EngineJob* jb = gen->jobs[i];
      if (jb->retired) continue;
      const tem::SolveHead& h = E->h_heads[(size_t)par * tem::kMaxBatchJobs + i];
      ++jb->checked;
      jb->k = jb->checked * B;
      int n_active = 0;
      for (int j = 0; j < jb->J; ++j) n_active += h.active[j];
      if (h.breakdown) jb->breakdown = true;
      if (h.breakdown || n_active == 0 || jb->k >= jb->max_iter) {
        finish(jb);
        any = true;
      }
    }
    if (any) E->done_cv.notify_all();
    ++blocks_done;
    if (verbose()) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      if (el >= next_report) {
        fprintf(stderr, "[tem] engine: %lld blocks read, %d jobs in the batch, %.1f s\n", blocks_done,
                (int)active.size(), el);
        next_report = el + 10.0;
      }
    }
  }
  // drain: nothing in flight is left behind
  (void)hipStreamSynchronize(E->stream);
}

// The multi-shift solves of multishift_solve, submitted to the context's
// engine (FP64 directions, 64-iteration blocks); same inputs and outputs.
int engine_solve(tem_ctx* ctx, const std::vector<double>& shifts_re, const std::vector<double>& shifts_im, double s0,
                 const tem_solve_opts& o, int njobs, double2* const* Ys, SolveState* states, double& seconds) {
  tem_engine* E = ctx->engine;
  const int J = (int)shifts_re.size();
  constexpr int B = kEngineBlock;
  const size_t n3 = ctx->n3;
  int rc;
  if ((rc = ensure_slots(ctx, njobs))) return rc;
  for (int i = 0; i < njobs; ++i) {
    SolveSlot& sl = ctx->slots[i];
    if ((rc = ensure(ctx, sl.R, (size_t)B * n3 * sizeof(double))) ||
        (rc = ensure(ctx, sl.pbuf, 2 * n3 * sizeof(double))) || (rc = ensure(ctx, sl.q, n3 * sizeof(double))) ||
        (rc = ensure(ctx, sl.P, (size_t)J * n3 * sizeof(double2))) ||
        (rc = ensure(ctx, sl.partials, 2 * (size_t)tem::kReduceSlots * sizeof(double))))
      return rc;
  }
  std::vector<std::unique_ptr<EngineJob>> jobs(njobs);
  auto cleanup = [&]() {
    for (auto& jb : jobs) {
      if (!jb) continue;
      if (jb->ready) (void)hipEventDestroy(jb->ready);
      if (jb->done) (void)hipEventDestroy(jb->done);
      if (jb->final_state) (void)hipHostFree(jb->final_state);
    }
  };
  for (int i = 0; i < njobs; ++i) {
    jobs[i].reset(new EngineJob());
    EngineJob& jb = *jobs[i];
    jb.ctx = ctx;
    jb.slot = i;
    jb.Y = Ys[i];
    jb.J = J;
    jb.s0 = s0;
    jb.max_iter = o.max_iter;
    jb.init.reset(new SolveState());
    SolveState& hs = *jb.init;
    std::memset(&hs, 0, sizeof(SolveState));
    hs.J = J;
    hs.B = B;
    hs.tol2 = o.rtol * o.rtol;
    for (int j = 0; j < J; ++j) {
      hs.sig_re[j] = shifts_re[j] - s0;
      hs.sig_im[j] = shifts_im[j];
      hs.z_re[j] = hs.zp_re[j] = 1.0;
      hs.active[j] = 1;
      for (int f = 0; f < tem::kPhases; ++f) {
        hs.apply[f][j] = 1;
        hs.cf[f][j][0][0] = 1.0;
      }
    }
    hipError_t e = hipEventCreateWithFlags(&jb.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&jb.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&jb.final_state, sizeof(SolveState), hipHostMallocDefault);
    // the right-hand side and the cleared buffers were written on the library stream
    if (e == hipSuccess) e = hipEventRecord(jb.ready, ctx->work);
    if (e != hipSuccess) {
      cleanup();
      return fail(ctx, TEM_EHIP, std::string("engine submit: ") + hipGetErrorString(e));
    }
  }
  const auto t0 = std::chrono::steady_clock::now();
  {
    std::unique_lock<std::mutex> lk(E->mu);
    for (auto& jb : jobs) E->pending.push_back(jb.get());
    E->cv.notify_all();
    E->done_cv.wait(lk, [&] {
      for (auto& jb : jobs)
        if (!jb->finished) return false;
      return true;
    });
  }
  hipError_t e = E->error;
  bool breakdown = false;
  for (int i = 0; i < njobs && e == hipSuccess; ++i) {
    e = hipEventSynchronize(jobs[i]->done);
    if (e != hipSuccess) break;
    states[i] = *jobs[i]->final_state;
    states[i].k = jobs[i]->k;
    states[i].breakdown = jobs[i]->breakdown ? 1 : 0;
    breakdown |= jobs[i]->breakdown;
    e = hipStreamWaitEvent(ctx->work, jobs[i]->done, 0);  // later work on the library stream reads Y
  }
  seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  cleanup();
  if (e != hipSuccess) return fail(ctx, TEM_EHIP, std::string("solve engine: ") + hipGetErrorString(e));
  if (breakdown) return fail(ctx, TEM_EBREAKDOWN, "Krylov breakdown in the shared recurrence");
  for (int i = 0; i < njobs; ++i)
    for (int j = 0; j < J; ++j)
      if (states[i].active[j]) return fail(ctx, TEM_ENOCONV, "max_iter reached before every shift converged");
  return TEM_OK;
}

// njobs independent multi-shift solves (all J shifts each), job i in slot i
// with its right-hand side g = M^{-1/2} f already in slots[i].gvec (written on
// the library stream).  Ys[i] receives the scaled solutions y_j = M^{1/2} x_j
// (node-padded, complex FP64); the per-shift search directions p_j are kept
// in PV (double2 for the FP64 path, float2 for precision 1); states[i] the
// final solver state.  Each job runs on its slot's stream; the host replays
// every active job's block graph before it waits for any of them, so their
// kernels overlap.
template <typename PV>
int multishift_solve(tem_ctx* ctx, const std::vector<double>& shifts_re, const std::vector<double>& shifts_im,
                     double s0, const tem_solve_opts& o, int njobs, double2* const* Ys, SolveState* states,
                     double& seconds) {
  if constexpr (std::is_same<PV, double2>::value) {
    if (uses_engine(ctx)) return engine_solve(ctx, shifts_re, shifts_im, s0, o, njobs, Ys, states, seconds);
  }
  const int J = (int)shifts_re.size();
  const int B = block_length(o.block);
  const GridArgs& g = ctx->g;
  const size_t n3 = ctx->n3;
  int rc;
  if ((rc = ensure_slots(ctx, njobs))) return rc;
  std::unique_ptr<SolveState> hs(new SolveState());
  std::memset(hs.get(), 0, sizeof(SolveState));
  hs->J = J;
  hs->B = B;
  hs->tol2 = o.rtol * o.rtol;
  for (int j = 0; j < J; ++j) {
    hs->sig_re[j] = shifts_re[j] - s0;
    hs->sig_im[j] = shifts_im[j];
    hs->z_re[j] = hs->zp_re[j] = 1.0;  // zeta_0 = zeta_{-1} = 1
    hs->active[j] = 1;
    for (int f = 0; f < tem::kPhases; ++f) {
      hs->apply[f][j] = 1;
      hs->cf[f][j][0][0] = 1.0;  // a = 1, c = 0: no update before the first block
    }
  }
  HIPCHK(ctx, hipEventRecord(ctx->work_ev, ctx->work));
  auto t0 = std::chrono::steady_clock::now();

  // One block of B seed iterations plus the deferred shift update is the same
  // launch sequence every time (slots depend on k mod B only), so it is
  // built once per job as a HIP graph and replayed; with opts.profile,
  // job 0 issues one block in kProfileEvery directly, each seed kernel's
  // dispatch recording its own start and stop events (sampling the kernel
  // times inside the timed solve).
  constexpr int kProfileEvery = 16;
  std::vector<hipEvent_t> ev;
  if (o.profile) {
    ev.resize(2 * (2 * B + 1));
    for (auto& e : ev) HIPCHK(ctx, hipEventCreate(&e));
  }
  // With overlap, block b runs its seed iterations on ring third f = b mod 3
  // and coefficient set f, and its deferred update runs on the slot's second
  // stream while block b+1's seed iterations proceed (the update is HBM-bound,
  // the seed latency-bound); block b+3, which reuses third f and set f, waits
  // for that update.  Without overlap the ring has B slots and the update ends
  // the block's own launch sequence.
  const bool overlap = overlap_updates();
  const bool one_kernel = ctx->seed_one_kernel;
  // unscaled seed vectors (the ring holds M^-1/2 r): the one-kernel form, and
  // the two-kernel form on the two tiles the library chooses
  const bool unscaled = one_kernel || tem::seed_stencil_unscaled_tile(ctx->g);
  const int RS = overlap ? tem::kPhases * B : B;  // ring slots
  // pbuf: p_{k-1}, p_k by parity (two-kernel form), or p_i, p_{i+1} and then
  // q_i, q_{i+1} by parity (one-kernel form)
  auto launch_block = [&](int i, bool timed, tem::Sink& st, int f) {
    SolveSlot& sl = ctx->slots[i];
    double* R = (double*)sl.R.p;
    double* pb = (double*)sl.pbuf.p;
    double* q = (double*)sl.q.p;
    const tem::Reduce red{(double*)sl.partials.p, ctx->d_counters};
    for (int l = 0; l < B; ++l) {
      double* r = R + (size_t)(f * B + l) * n3;
      double* rn = R + (size_t)((f * B + l + 1) % RS) * n3;
      double* pold = pb + (size_t)((l + 1) & 1) * n3;
      double* pnew = pb + (size_t)(l & 1) * n3;
      if (one_kernel) {
        tem::launch_seed_step(g, r, pb + (size_t)(l & 1) * n3, pb + (size_t)(2 + (l & 1)) * n3, rn,
                              pb + (size_t)((l + 1) & 1) * n3, pb + (size_t)(2 + ((l + 1) & 1)) * n3, ctx->d_dinv,
                              s0, red, sl.d_state, l, 0, st, timed ? ev[4 * l] : nullptr,
                              timed ? ev[4 * l + 1] : nullptr);
        continue;
      }
      tem::launch_seed_stencil(g, r, pold, pnew, q, ctx->d_dinv, s0, red, sl.d_state, l, unscaled, st,
                               timed ? ev[4 * l] : nullptr, timed ? ev[4 * l + 1] : nullptr);
      tem::launch_seed_update(g, r, q, rn, red, sl.d_state, l, unscaled ? ctx->d_dinv : nullptr, st,
                              timed ? ev[4 * l + 2] : nullptr,
                              timed ? ev[4 * l + 3] : nullptr);
    }
    if (!overlap && timed) (void)hipEventRecord(ev[4 * B], st.stream);
    if (one_kernel) tem::launch_shift_block_step(g, J, red, sl.d_state, st, f);
    else tem::launch_shift_block(g, J, red, sl.d_state, st, f);
    if (!overlap) {
      tem::launch_block_update(g, R, R, Ys[i], (PV*)sl.P.p, J, B, sl.d_state, st, 0, 4096,
                               unscaled ? ctx->d_sqrtm : nullptr);
      if (timed) (void)hipEventRecord(ev[4 * B + 1], st.stream);
    }
  };
  // the deferred update of block b (phase f) on the second stream, after its shift recurrences
  auto launch_update = [&](int i, bool timed, int f) -> hipError_t {
    SolveSlot& sl = ctx->slots[i];
    double* R = (double*)sl.R.p;
    hipError_t e = hipEventRecord(sl.sb_ev[f], sl.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(sl.stream2, sl.sb_ev[f], 0);
    if (e != hipSuccess) return e;
    if (timed) (void)hipEventRecord(ev[4 * B], sl.stream2);
    tem::Sink d;
    d.stream = sl.stream2;
    tem::launch_block_update(g, R + (size_t)f * B * n3, R + (size_t)((f + 1) % tem::kPhases) * B * n3, Ys[i],
                             (PV*)sl.P.p, J, B, sl.d_state, d, f, overlap_blocks(), unscaled ? ctx->d_sqrtm : nullptr);
    if (timed) (void)hipEventRecord(ev[4 * B + 1], sl.stream2);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(sl.bu_ev[f], sl.stream2);
    return e;
  };
  struct Run {
    hipGraph_t graph[tem::kPhases] = {};
    hipGraphExec_t exec[tem::kPhases] = {};
    int k = 0;             // seed iterations of the blocks whose head the host has read
    int launched = 0;      // blocks issued
    int checked = 0;       // blocks whose head the host has read
    int sampled = -1;      // block issued with timing events
    bool done = false;
    bool breakdown = false;
  };
  std::vector<Run> run(njobs);
  auto cleanup = [&]() {
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (Run& r : run)
      for (int f = 0; f < tem::kPhases; ++f) {
        if (r.exec[f]) (void)hipGraphExecDestroy(r.exec[f]);
        if (r.graph[f]) (void)hipGraphDestroy(r.graph[f]);
      }
  };
  for (int i = 0; i < njobs; ++i) {
    SolveSlot& sl = ctx->slots[i];
    hipStream_t st = sl.stream;
    if ((rc = ensure(ctx, sl.R, (size_t)RS * n3 * sizeof(double))) ||
        (rc = ensure(ctx, sl.pbuf, (one_kernel ? 4 : 2) * n3 * sizeof(double))) ||
        (rc = ensure(ctx, sl.q, n3 * sizeof(double))) ||
        (rc = ensure(ctx, sl.P, (size_t)J * n3 * sizeof(double2))) ||
        (rc = ensure(ctx, sl.partials, 8 * (size_t)tem::kReduceSlots * sizeof(double)))) {
      cleanup();
      return rc;
    }
    // buffers allocated above are cleared on the library stream; the slot's
    // work starts after that and after its right-hand side
    hipError_t se = hipEventRecord(ctx->work_ev, ctx->work);
    if (se == hipSuccess) se = hipStreamWaitEvent(st, ctx->work_ev, 0);
    if (se == hipSuccess)
      se = hipMemcpyAsync(sl.d_state, hs.get(), sizeof(SolveState), hipMemcpyHostToDevice, st);
    if (se == hipSuccess) {
      const tem::Reduce red{(double*)sl.partials.p, ctx->d_counters};
      tem::launch_seed_init(g, (const double*)sl.gvec.p, (double*)sl.R.p, (double*)sl.pbuf.p + n3, Ys[i],
                            (PV*)sl.P.p, J, red, sl.d_state, st, unscaled ? ctx->d_dinv : nullptr);
      if (one_kernel) {  // p_0 = r_0, q_0 = A0 r_0 into slot 0 and the partials of step 0
        tem::Sink pro;
        pro.stream = st;
        const double* r0 = (const double*)sl.R.p;
        tem::launch_seed_step(g, r0, r0, r0, nullptr, (double*)sl.pbuf.p, (double*)sl.pbuf.p + 2 * n3,
                              ctx->d_dinv, s0, red, sl.d_state, 0, 1, pro);
      }
      se = hipGetLastError();
    }
    if (se != hipSuccess) {
      for (int m = 0; m <= i; ++m) (void)hipStreamSynchronize(ctx->slots[m].stream);
      cleanup();
      return fail(ctx, TEM_EHIP, std::string("solver set-up: ") + hipGetErrorString(se));
    }
    // the block's kernels become the nodes of a graph built explicitly (no
    // stream capture: a capture could be invalidated by a device-wide call such
    // as hipFree from another request's thread); on failure the blocks are
    // launched directly
    hipError_t ge = hipSuccess;
    for (int f = 0; f < (overlap ? tem::kPhases : 1) && ge == hipSuccess; ++f) {
      tem::Sink gk;
      ge = hipGraphCreate(&run[i].graph[f], 0);
      if (ge == hipSuccess) {
        gk.graph = run[i].graph[f];
        launch_block(i, false, gk, f);
        ge = gk.err;
      }
      if (ge == hipSuccess) ge = hipGraphInstantiate(&run[i].exec[f], run[i].graph[f], nullptr, nullptr, 0);
    }
    if (ge != hipSuccess) {
      (void)hipGetLastError();
      for (int f = 0; f < tem::kPhases; ++f) {
        if (run[i].exec[f]) (void)hipGraphExecDestroy(run[i].exec[f]);
        if (run[i].graph[f]) (void)hipGraphDestroy(run[i].graph[f]);
        run[i].graph[f] = nullptr;
        run[i].exec[f] = nullptr;
      }
      if (verbose()) fprintf(stderr, "[tem] solver block graph not built (%s): direct launches\n", hipGetErrorString(ge));
    }
  }
  hipError_t lerr = hipSuccess;
  bool breakdown = false;
  double next_report = 10.0;
  // Issue block `launched` of job i: the graph (or direct launches when timed),
  // then the copy of the head into pinned slot (launched mod 2) and its event.
  auto issue = [&](int i) -> hipError_t {
    SolveSlot& sl = ctx->slots[i];
    Run& r = run[i];
    const bool timed = o.profile && i == 0 && r.launched % kProfileEvery == 0;
    const int f = overlap ? r.launched % tem::kPhases : 0;
    hipError_t e = hipSuccess;
    // block b reuses ring third and coefficient set f after block b-3's update
    if (overlap && r.launched >= tem::kPhases) e = hipStreamWaitEvent(sl.stream, sl.bu_ev[f], 0);
    if (e == hipSuccess && r.exec[f] && !timed) {
      e = hipGraphLaunch(r.exec[f], sl.stream);
    } else if (e == hipSuccess) {
      tem::Sink direct;
      direct.stream = sl.stream;
      launch_block(i, timed, direct, f);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && overlap) e = launch_update(i, timed, f);
    const int h = r.launched & 1;
    if (e == hipSuccess)
      e = hipMemcpyAsync((char*)sl.head + h * kHeadStride, sl.d_state, sizeof(tem::SolveHead),
                         hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.head_ev[h], sl.stream);
    if (timed) r.sampled = r.launched;
    ++r.launched;
    return e;
  };
  // Two blocks per job stay in flight: the host reads block b's head while
  // block b+1 already runs, so the device never waits for the host between
  // blocks.  A job that turns out converged at block b has issued block b+1
  // as well; with every shift inactive that block changes no y_j (its shift
  // update applies nothing), and its seed steps are not counted.
  for (;;) {
    bool any = false;
    for (int i = 0; i < njobs && lerr == hipSuccess; ++i) {
      Run& r = run[i];
      if (r.done) continue;
      any = true;
      while (lerr == hipSuccess && r.launched - r.checked < 2 && (long long)r.launched * B < o.max_iter)
        lerr = issue(i);
    }
    if (!any || lerr != hipSuccess) break;
    int n_active_all = 0;
    for (int i = 0; i < njobs && lerr == hipSuccess; ++i) {
      Run& r = run[i];
      if (r.done) continue;
      SolveSlot& sl = ctx->slots[i];
      const int h = r.checked & 1;
      lerr = hipEventSynchronize(sl.head_ev[h]);
      if (lerr != hipSuccess) break;
      const tem::SolveHead head = *(const tem::SolveHead*)((const char*)sl.head + h * kHeadStride);
      ++r.checked;
      r.k = r.checked * B;
      int n_active = 0;
      for (int j = 0; j < J; ++j) n_active += head.active[j];
      n_active_all += n_active;
      if (head.breakdown) r.breakdown = breakdown = true;
      if (head.breakdown || n_active == 0 || r.k >= o.max_iter) r.done = true;
      if (r.sampled == r.checked - 1) {
        for (int l = 0; l < B; ++l) {
          float a = 0.f, b = 0.f;
          (void)hipEventElapsedTime(&a, ev[4 * l], ev[4 * l + 1]);
          if (!one_kernel) (void)hipEventElapsedTime(&b, ev[4 * l + 2], ev[4 * l + 3]);
          ctx->prof_ms[TEM_K_STENCIL] += a;
          if (!one_kernel) ctx->prof_ms[TEM_K_UPDATE] += b;
        }
        float c = 0.f;
        (void)hipEventSynchronize(ev[4 * B + 1]);  // with overlap the update ends on the second stream
        (void)hipEventElapsedTime(&c, ev[4 * B], ev[4 * B + 1]);
        ctx->prof_ms[TEM_K_BLOCK] += c;
        ctx->prof_n[TEM_K_STENCIL] += B;
        if (!one_kernel) ctx->prof_n[TEM_K_UPDATE] += B;
        ctx->prof_n[TEM_K_BLOCK] += 1;
      }
    }
    if (verbose()) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el >= next_report) {
        fprintf(stderr, "[tem] multi-shift: %d solves, %d iterations, %d shifts active, %.1f s\n", njobs, run[0].k,
                n_active_all, el);
        next_report = el + 10.0;
      }
    }
  }
  if (lerr != hipSuccess) {
    // blocks still in flight finish before their graphs and events are destroyed
    for (int i = 0; i < njobs; ++i) {
      (void)hipStreamSynchronize(ctx->slots[i].stream);
      (void)hipStreamSynchronize(ctx->slots[i].stream2);
    }
    cleanup();
    return fail(ctx, TEM_EHIP, std::string("solver loop: ") + hipGetErrorString(lerr));
  }
  seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  hipError_t fe = hipSuccess;
  for (int i = 0; i < njobs; ++i) {
    SolveSlot& sl = ctx->slots[i];
    // the last block's update (second stream) precedes everything that reads Y
    if (overlap && run[i].launched > 0)
      fe = hipStreamWaitEvent(sl.stream, sl.bu_ev[(run[i].launched - 1) % tem::kPhases], 0);
    if (fe == hipSuccess)
      fe = hipMemcpyAsync(&states[i], sl.d_state, sizeof(SolveState), hipMemcpyDeviceToHost, sl.stream);
    // also waits for a block issued after the last one the host read
    const hipError_t se = hipStreamSynchronize(sl.stream);
    if (fe == hipSuccess) fe = se;
    // the solve ended at the block the host last read; a block issued after it
    // only advanced the seed
    states[i].k = run[i].k;
    states[i].breakdown = run[i].breakdown ? 1 : 0;
    // later work on the library stream reads Ys[i]
    if (fe == hipSuccess) fe = hipEventRecord(sl.ev, sl.stream);
    if (fe == hipSuccess) fe = hipStreamWaitEvent(ctx->work, sl.ev, 0);
  }
  cleanup();
  if (fe != hipSuccess) return fail(ctx, TEM_EHIP, std::string("solver end: ") + hipGetErrorString(fe));
  for (int i = 0; i < njobs; ++i) breakdown |= states[i].breakdown != 0;
  if (breakdown) return fail(ctx, TEM_EBREAKDOWN, "Krylov breakdown in the shared recurrence");
  for (int i = 0; i < njobs; ++i)
    for (int j = 0; j < J; ++j)
      if (states[i].active[j]) return fail(ctx, TEM_ENOCONV, "max_iter reached before every shift converged");
  return TEM_OK;
}

// Batched COCG on (A + s_j) mu_j = h_j for the J shifts in ctx->sh, vectors
// of V storage (Mu, Rr, P0, P1, Q: J node-padded vectors each); stops shift j
// when |r_j| <= rtol |h_j|.  Shifts with h_j = 0 stay inactive (mu_j = 0).
// With stall > 0, shift j is also stopped once its recursive residual has not
// fallen by 10% over `stall` iterations (checked every 32 iterations), so
// that a correction which stagnates cannot run to its cap.
template <typename V>
int cocg_solve(tem_ctx* ctx, int J, const double2* H, V* Mu, V* Rr, V* P0, V* P1, V* Q, double rtol, int max_iter,
               tem::CocgState& hs, int& iterations, const int* caps = nullptr, int stall = 0) {
  hipStream_t st = ctx->work;
  int rc;
  if ((rc = ensure(ctx, ctx->cst, tem::cocg_state_bytes())) ||
      (rc = ensure(ctx, ctx->cocg_part, (size_t)tem::cocg_partials(ctx->g, J) * sizeof(double))))
    return rc;
  const double* shd = (const double*)ctx->sh.p;
  std::memset(&hs, 0, sizeof(tem::CocgState));
  hs.J = J;
  hs.tol2 = rtol * rtol;
  for (int j = 0; j < J; ++j) hs.cap[j] = caps ? std::min(caps[j], max_iter) : max_iter;
  HIPCHK(ctx, hipMemcpyAsync(ctx->cst.p, &hs, sizeof(tem::CocgState), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemsetAsync(ctx->d_counters + 4, 0, 4 * sizeof(unsigned int), st));
  double* partials = (double*)ctx->cocg_part.p;
  tem::launch_cocg_init(ctx->g, J, H, Mu, Rr, P0, partials, ctx->d_counters + 4, ctx->cst.p, st);
  int it = 0;
  const int chunk = 32;
  hipError_t e = hipSuccess;
  iterations = 0;
  const auto t0 = std::chrono::steady_clock::now();
  double next_report = 10.0;
  std::vector<double> best(J, -1.0);  // smallest |r_j|^2 that was a 10% reduction, and when
  std::vector<int> best_it(J, 0), cap_now(hs.cap, hs.cap + J);
  while (it < max_iter) {
    for (int i = 0; i < chunk; ++i, ++it) {
      V* Pold = (it & 1) ? P1 : P0;
      V* Pnew = (it & 1) ? P0 : P1;
      tem::launch_cocg_stencil(ctx->g, J, Rr, Pold, Pnew, Q, ctx->d_dinv, shd, shd + TEM_MAX_SHIFTS, partials,
                               ctx->d_counters + 5, ctx->cst.p, st);
      tem::launch_cocg_update(ctx->g, J, Mu, Rr, Pnew, Q, partials, ctx->d_counters + 6, ctx->cst.p, st);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hs, ctx->cst.p, sizeof(tem::CocgState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ctx, TEM_EHIP, std::string("COCG: ") + hipGetErrorString(e));
    iterations = it;
    if (hs.breakdown) return fail(ctx, TEM_EBREAKDOWN, "COCG breakdown");
    if (hs.n_active == 0) break;
    if (stall > 0) {
      bool changed = false;
      for (int j = 0; j < J; ++j) {
        if (!hs.active[j]) continue;
        if (best[j] < 0.0 || hs.rn2[j] <= 0.81 * best[j]) {
          best[j] = hs.rn2[j];
          best_it[j] = hs.iters[j];
        } else if (hs.iters[j] - best_it[j] >= stall && cap_now[j] > hs.iters[j] + 1) {
          cap_now[j] = hs.iters[j] + 1;  // the next update stops it
          changed = true;
        }
      }
      if (changed) {
        tem::CocgState* dst = (tem::CocgState*)ctx->cst.p;
        e = hipMemcpyAsync(dst->cap, cap_now.data(), J * sizeof(int), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // cap_now is host memory read by the copy
        if (e != hipSuccess) return fail(ctx, TEM_EHIP, std::string("COCG: ") + hipGetErrorString(e));
      }
    }
    if (verbose()) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el >= next_report) {
        fprintf(stderr, "[tem] COCG: %d iterations, %d of %d systems active, %.1f s\n", it, hs.n_active, J, el);
        next_report = el + 10.0;
      }
    }
  }
  // a shift stopped by its iteration cap has not converged
  bool capped = hs.n_active > 0;
  for (int j = 0; j < J; ++j) capped |= hs.iters[j] >= hs.cap[j] && hs.rn2[j] > hs.tol2 * hs.hn2[j];
  return capped ? fail(ctx, TEM_ENOCONV, "COCG did not reach rtol within its iteration cap") : TEM_OK;
}

// Two-pass form (opts.method 1) for the source whose right-hand side is in
// slot i: pass 1 runs the seed recurrence with the shift-block convergence
// test and records alpha_k, beta_k, (r_{k+1}, r_{k+1}) and q_r . (M^-1/2 r_k);
// the host replays each shift's recurrence (the k_shift_block formulas) to
// get y_j = sum_k gamma_jk r_k, gamma_jk = zeta_jk S_jk with
// S_jk = alpha^s_jk + beta^s_jk S_j,k+1, and w_kt = Re sum_j c_jt gamma_jk;
// data[t][r] = sum_k (q_r . M^-1/2 r_k) w_kt.  With fields, pass 2 reruns the
// seed (the same kernels and state, so the same residuals bit for bit) and
// accumulates U = sum_k r_k w_k^T block by block on MFMA.
int lanczos_source(tem_ctx* ctx, int i, const std::vector<double>& shifts_re, const std::vector<double>& shifts_im,
                   double s0, const tem_solve_opts& o, int T, const double* c, int n_rx, double* data, double* fields,
                   SolveState& fin, double& secs) {
  const int J = (int)shifts_re.size();
  const int B = block_length(o.block);
  const GridArgs& g = ctx->g;
  const size_t n3 = ctx->n3;
  hipStream_t st = ctx->work;
  int rc;
  SolveSlot& sl = ctx->slots[i];
  const bool one_kernel = ctx->seed_one_kernel;
  // unscaled seed vectors (the ring holds M^-1/2 r): the one-kernel form, and
  // the two-kernel form on the two tiles the library chooses
  const bool unscaled = one_kernel || tem::seed_stencil_unscaled_tile(ctx->g);
  if ((rc = ensure(ctx, sl.R, (size_t)B * n3 * sizeof(double))) ||
      (rc = ensure(ctx, sl.pbuf, (one_kernel ? 4 : 2) * n3 * sizeof(double))) ||
      (rc = ensure(ctx, sl.q, n3 * sizeof(double))) ||
      (rc = ensure(ctx, sl.partials, 8 * (size_t)tem::kReduceSlots * sizeof(double))))
    return rc;
  const int nrx = std::max(n_rx, 1);
  DevBuf hqd, Wd, Ud;
  double* hq_pin = nullptr;  // pinned: the receiver values of the two blocks in flight
  auto cleanup = [&]() {
    release(hqd);
    release(Wd);
    release(Ud);
    if (hq_pin) (void)hipHostFree(hq_pin);
  };
  if ((rc = ensure(ctx, hqd, (size_t)B * nrx * sizeof(double)))) return rc;
  if (hipHostMalloc((void**)&hq_pin, 2 * (size_t)B * nrx * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    cleanup();
    return fail(ctx, TEM_ENOMEM, "pinned receiver buffer");
  }
  std::unique_ptr<SolveState> hs(new SolveState());
  std::memset(hs.get(), 0, sizeof(SolveState));
  hs->J = J;
  hs->B = B;
  hs->tol2 = o.rtol * o.rtol;
  for (int j = 0; j < J; ++j) {
    hs->sig_re[j] = shifts_re[j] - s0;
    hs->sig_im[j] = shifts_im[j];
    hs->z_re[j] = hs->zp_re[j] = 1.0;
    hs->active[j] = 1;
    for (int f = 0; f < tem::kPhases; ++f) {
      hs->apply[f][j] = 1;
      hs->cf[f][j][0][0] = 1.0;
    }
  }
  // the leading part of the state up to and including this block's history
  const size_t hist_bytes = offsetof(SolveState, carry_alpha);
  static_assert(offsetof(SolveState, carry_alpha) <= kHeadStride, "history head fits the pinned buffer");
  const tem::Reduce red{(double*)sl.partials.p, ctx->d_counters};
  double* R = (double*)sl.R.p;
  double* pb = (double*)sl.pbuf.p;
  double* q = (double*)sl.q.p;
  const int* rxp = (const int*)ctx->rx.p;
  auto init = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(sl.d_state, hs.get(), sizeof(SolveState), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    tem::launch_seed_init(g, (const double*)sl.gvec.p, R, pb + n3, (double2*)nullptr, (double2*)nullptr, 0, red,
                          sl.d_state, st, unscaled ? ctx->d_dinv : nullptr);
    if (one_kernel) {
      tem::Sink pro;
      pro.stream = st;
      tem::launch_seed_step(g, R, R, R, nullptr, pb, pb + 2 * n3, ctx->d_dinv, s0, red, sl.d_state, 0, 1, pro);
    }
    return hipGetLastError();
  };
  // the seed kernels of one block plus the shift recurrences (convergence and
  // the iteration count); `extra` appends the pass's own kernel
  auto build = [&](hipGraph_t* gr, hipGraphExec_t* ex, const std::function<void(tem::Sink&)>& extra) -> hipError_t {
    hipError_t e = hipGraphCreate(gr, 0);
    if (e != hipSuccess) return e;
    tem::Sink k;
    k.graph = *gr;
    for (int l = 0; l < B; ++l) {
      double* r = R + (size_t)l * n3;
      double* rn = R + (size_t)((l + 1) % B) * n3;
      if (one_kernel) {
        tem::launch_seed_step(g, r, pb + (size_t)(l & 1) * n3, pb + (size_t)(2 + (l & 1)) * n3, rn,
                              pb + (size_t)((l + 1) & 1) * n3, pb + (size_t)(2 + ((l + 1) & 1)) * n3, ctx->d_dinv, s0,
                              red, sl.d_state, l, 0, k);
        continue;
      }
      tem::launch_seed_stencil(g, r, pb + (size_t)((l + 1) & 1) * n3, pb + (size_t)(l & 1) * n3, q, ctx->d_dinv, s0,
                               red, sl.d_state, l, unscaled, k);
      tem::launch_seed_update(g, r, q, rn, red, sl.d_state, l, unscaled ? ctx->d_dinv : nullptr, k);
    }
    if (one_kernel) tem::launch_shift_block_step(g, J, red, sl.d_state, k);
    else tem::launch_shift_block(g, J, red, sl.d_state, k);
    extra(k);
    if (k.err != hipSuccess) return k.err;
    return hipGraphInstantiate(ex, *gr, nullptr, nullptr, 0);
  };
  hipGraph_t g1 = nullptr, g2 = nullptr;
  hipGraphExec_t x1 = nullptr, x2 = nullptr;
  auto drop = [&]() {
    for (hipGraphExec_t x : {x1, x2})
      if (x) (void)hipGraphExecDestroy(x);
    for (hipGraph_t gg : {g1, g2})
      if (gg) (void)hipGraphDestroy(gg);
  };
  const auto t0 = std::chrono::steady_clock::now();
  // ---- pass 1
  std::vector<double> ha, hb, hr, hq;  // alpha_k, beta_k, (r_{k+1}, r_{k+1}); q_r . M^-1/2 r_k
  hipError_t e = init();
  if (e == hipSuccess && n_rx > 0) {
    tem::Sink d;
    d.stream = st;
    tem::launch_ring_receivers(g, R, B, unscaled ? nullptr : ctx->d_dinv, rxp, n_rx, ctx->ks, (double*)hqd.p, 1, d);
    hq.resize(n_rx);
    e = hipMemcpyAsync(hq.data(), hqd.p, n_rx * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e == hipSuccess)
    e = build(&g1, &x1, [&](tem::Sink& k) {
      if (n_rx > 0)
        tem::launch_ring_receivers(g, R, B, unscaled ? nullptr : ctx->d_dinv, rxp, n_rx, ctx->ks, (double*)hqd.p, 0, k);
    });
  int launched = 0, checked = 0;
  bool done = false, breakdown = false;
  while (e == hipSuccess && !done) {
    while (e == hipSuccess && launched - checked < 2 && (long long)launched * B < o.max_iter) {
      const int h = launched & 1;
      e = hipGraphLaunch(x1, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync((char*)sl.head + h * kHeadStride, sl.d_state, hist_bytes, hipMemcpyDeviceToHost, st);
      // the block's receiver values, copied before the next block overwrites them
      if (e == hipSuccess && n_rx > 0)
        e = hipMemcpyAsync(hq_pin + (size_t)h * B * n_rx, hqd.p, (size_t)B * n_rx * sizeof(double),
                           hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipEventRecord(sl.head_ev[h], st);
      ++launched;
    }
    if (e != hipSuccess || launched == checked) break;
    const int h = checked & 1;
    e = hipEventSynchronize(sl.head_ev[h]);
    if (e != hipSuccess) break;
    const SolveState* hd = (const SolveState*)((const char*)sl.head + h * kHeadStride);
    ha.insert(ha.end(), hd->alpha_h, hd->alpha_h + B);
    hb.insert(hb.end(), hd->beta_h, hd->beta_h + B);
    hr.insert(hr.end(), hd->rr_h, hd->rr_h + B);
    if (n_rx > 0) hq.insert(hq.end(), hq_pin + (size_t)h * B * n_rx, hq_pin + (size_t)(h + 1) * B * n_rx);
    ++checked;
    int n_active = 0;
    for (int j = 0; j < J; ++j) n_active += hd->active[j];
    if (hd->breakdown) breakdown = true;
    if (hd->breakdown || n_active == 0 || (long long)checked * B >= o.max_iter) done = true;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&fin, sl.d_state, sizeof(SolveState), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    drop();
    cleanup();
    return fail(ctx, TEM_EHIP, std::string("two-pass solve: ") + hipGetErrorString(e));
  }
  fin.k = checked * B;
  fin.breakdown = breakdown ? 1 : 0;
  // ---- host: the shifted recurrences and the channel weights w_kt
  int kmax = 0;
  for (int j = 0; j < J; ++j) kmax = std::max(kmax, fin.iters[j]);
  const int nblk = (kmax + B - 1) / B;
  const size_t rows = (size_t)nblk * B + 1;
  std::vector<double> W(rows * T, 0.0);
  using cd = std::complex<double>;
  for (int j = 0; j < J; ++j) {
    const int K = fin.iters[j];
    const cd sig(hs->sig_re[j], hs->sig_im[j]);
    std::vector<cd> zeta(K + 1), as(K), bs(K);
    cd z(1.0, 0.0), zp(1.0, 0.0);
    for (int k = 0; k < K; ++k) {
      const double a_k = ha[k], b_k = hb[k];
      const double a_km1 = k ? ha[k - 1] : 1.0, b_km1 = k ? hb[k - 1] : 0.0;
      const cd num = a_km1 * z * zp;
      const cd den = (a_k * b_km1) * (zp - z) + a_km1 * zp * (1.0 + sig * a_k);
      const cd zn = num / den;
      const cd ratio = a_km1 * zp / den;
      zeta[k] = z;
      as[k] = a_k * ratio;
      bs[k] = b_k * ratio * ratio;
      zp = z;
      z = zn;
    }
    cd S(0.0, 0.0);
    for (int k = K - 1; k >= 0; --k) {
      S = as[k] + bs[k] * S;
      const cd gamma = zeta[k] * S;
      for (int t = 0; t < T; ++t) {
        const cd cjt(c[2 * ((size_t)j * T + t)], c[2 * ((size_t)j * T + t) + 1]);
        W[(size_t)k * T + t] += (cjt * gamma).real();
      }
    }
  }
  // receivers: data[t][r] = sum_k hq[k][r] w_kt
  if (n_rx > 0) {
    std::fill(data, data + (size_t)T * n_rx, 0.0);
    const size_t kk = std::min((size_t)kmax, hq.size() / n_rx);
    for (size_t k = 0; k < kk; ++k)
      for (int r = 0; r < n_rx; ++r) {
        const double v = hq[k * n_rx + r];
        for (int t = 0; t < T; ++t) data[(size_t)t * n_rx + r] += v * W[k * T + t];
      }
  }
  // ---- pass 2: the fields
  if (fields) {
    if ((rc = ensure(ctx, Wd, rows * T * sizeof(double))) || (rc = ensure(ctx, Ud, (size_t)T * n3 * sizeof(double)))) {
      drop();
      cleanup();
      return rc;
    }
    e = hipMemcpyAsync(Wd.p, W.data(), rows * T * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = init();
    if (e == hipSuccess) {
      tem::launch_ring_contract_init(g, R, (const double*)Wd.p, T, (double*)Ud.p, st);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = build(&g2, &x2, [&](tem::Sink& k) {
        tem::launch_ring_contract(g, R, B, (const double*)Wd.p, T, (double*)Ud.p, sl.d_state, k);
      });
    for (int b = 0; b < nblk && e == hipSuccess; ++b) e = hipGraphLaunch(x2, st);
    if (e == hipSuccess) {
      tem::launch_ring_fields(g, (const double*)Ud.p, T, unscaled ? nullptr : ctx->d_dinv, fields, rxp, 0, ctx->ks,
                              nullptr, st);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  drop();
  cleanup();
  secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) return fail(ctx, TEM_EHIP, std::string("two-pass solve: ") + hipGetErrorString(e));
  if (breakdown) return fail(ctx, TEM_EBREAKDOWN, "Krylov breakdown in the shared recurrence");
  for (int j = 0; j < J; ++j)
    if (fin.active[j]) return fail(ctx, TEM_ENOCONV, "max_iter reached before every shift converged");
  return TEM_OK;
}

}  // namespace

extern "C" {

int tem_setup_grid(tem_ctx** out, int nx, int ny, int nz, const double* hx, const double* hy, const double* hz,
                   int k_surface, int device, void* hip_stream) {
  if (out == nullptr) return fail(nullptr, TEM_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  if (nx < 2 || ny < 2 || nz < 2 || nx > 4096 || ny > 4096 || nz > 4096)
    return fail(nullptr, TEM_EINVAL, "grid dimensions must be in [2, 4096]");
  if (!hx || !hy || !hz || !finite_pos(hx, nx) || !finite_pos(hy, ny) || !finite_pos(hz, nz))
    return fail(nullptr, TEM_EINVAL, "cell widths must be finite and positive");
  if (!(0 < k_surface && k_surface < nz)) return fail(nullptr, TEM_EINVAL, "k_surface must satisfy 0 < k_surface < nz");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, TEM_EHIP, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, TEM_EHIP, "hipSetDevice failed");
  std::unique_ptr<tem_ctx> c(new tem_ctx());
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->ks = k_surface;
  c->hx.assign(hx, hx + nx);
  c->hy.assign(hy, hy + ny);
  c->hz.assign(hz, hz + nz);
  GridArgs& g = c->g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.px = nx + 1;
  g.py = ny + 1;
  g.pz = nz + 1;
  g.nn = (long long)g.px * g.py * g.pz;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) n_cu = 0;
  g.seed_tile = tem::choose_seed_tile(g, n_cu);
  {  // TEM_SEED_TILE=17 (the one-plane stencil tile) also gives the one-kernel step one plane per tile
    const char* e = getenv("TEM_SEED_TILE");
    g.step_kz = (e && atoi(e) == 17) ? 1 : 2;
  }
  c->seed_one_kernel = seed_one_kernel_for(g, n_cu);
  c->engine_batches = n_cu > 0 && tem::seed_step_blocks(g) < n_cu;
  if (tem::seed_step_blocks(g) > tem::kReduceSlots) return fail(nullptr, TEM_EINVAL, "grid too large: more seed tiles than partial-sum slots");
  // the seed kernels address a 3 nn real field by 32-bit byte offsets
  if (3.0 * (double)g.nn * sizeof(double) >= 4294967296.0)
    return fail(nullptr, TEM_EINVAL, "grid too large: a real field must stay below 4 GiB");
  c->n3 = 3 * g.nn;
  c->nstore = tem::storage_edges(g);
  if (tem::seed_stencil_blocks(g) > tem::kReduceSlots) return fail(nullptr, TEM_EINVAL, "grid too large: more stencil tiles than partial-sum slots");
  c->nunk = (long long)nx * (ny - 1) * (nz - 1) + (long long)(nx - 1) * ny * (nz - 1) + (long long)(nx - 1) * (ny - 1) * nz;
  // axis arrays: h, 1/h, dual/mu0 per axis, each padded to n+1
  const int L = std::max(nx, std::max(ny, nz)) + 1;
  std::vector<double> ax(9 * (size_t)L, 0.0);
  const std::vector<double>* hs[3] = {&c->hx, &c->hy, &c->hz};
  for (int a = 0; a < 3; ++a) {
    const std::vector<double>& h = *hs[a];
    const int n = (int)h.size();
    double* H = &ax[(3 * a + 0) * (size_t)L];
    double* IH = &ax[(3 * a + 1) * (size_t)L];
    double* DW = &ax[(3 * a + 2) * (size_t)L];
    for (int i = 0; i < n; ++i) {
      H[i] = h[i];
      IH[i] = 1.0 / h[i];
    }
    for (int i = 0; i <= n; ++i) {
      const double lo = i > 0 ? h[i - 1] : 0.0, hi = i < n ? h[i] : 0.0;
      DW[i] = 0.5 * (lo + hi) / tem::kMu0;  // node-centred dual width over mu0
    }
  }
  tem_ctx* ctx = c.get();
  HIPCHK(ctx, hipMalloc(&c->d_axis, ax.size() * sizeof(double)));
  HIPCHK(ctx, hipMemcpy(c->d_axis, ax.data(), ax.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int a = 0; a < 3; ++a) {
    g.h[a] = c->d_axis + (3 * a + 0) * (size_t)L;
    g.ih[a] = c->d_axis + (3 * a + 1) * (size_t)L;
    g.dw[a] = c->d_axis + (3 * a + 2) * (size_t)L;
  }
  const long long ncell = (long long)nx * ny * nz;
  HIPCHK(ctx, hipMalloc(&c->d_sigma, ncell * sizeof(double)));
  HIPCHK(ctx, hipMalloc(&c->d_mass, c->n3 * sizeof(double)));
  HIPCHK(ctx, hipMalloc(&c->d_dinv, c->n3 * sizeof(double)));
  HIPCHK(ctx, hipMalloc(&c->d_sqrtm, c->n3 * sizeof(double)));
  HIPCHK(ctx, hipMalloc(&c->d_counters, 16 * sizeof(unsigned int)));
  HIPCHK(ctx, hipMemset(c->d_counters, 0, 16 * sizeof(unsigned int)));
  HIPCHK(ctx, hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking));
  HIPCHK(ctx, hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming));
  HIPCHK(ctx, hipEventCreateWithFlags(&c->work_ev, hipEventDisableTiming));
  HIPCHK(ctx, hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming));
  // the device is current (hipSetDevice above): look up its copy of the array
  HIPCHK(ctx, scratch_address(device, &c->scratch));
  *out = c.release();
  return TEM_OK;
}

int tem_set_conductivity(tem_ctx* ctx, const double* sigma, int flags) {
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (!sigma) return fail(ctx, TEM_EINVAL, "sigma is NULL");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const long long ncell = (long long)ctx->nx * ctx->ny * ctx->nz;
  std::vector<double> h(ncell);
  if (flags & TEM_DEVICE_PTR) {
    HIPCHK(ctx, hipMemcpy(h.data(), sigma, ncell * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(h.data(), sigma, ncell * sizeof(double));
  }
  for (long long i = 0; i < ncell; ++i) {
    if (flags & TEM_SIGMA_LOG) {
      if (!std::isfinite(h[i])) return fail(ctx, TEM_EINVAL, "ln sigma must be finite");
      h[i] = std::exp(h[i]);
    }
    if (!(std::isfinite(h[i]) && h[i] > 0.0)) return fail(ctx, TEM_EINVAL, "sigma must be finite and positive");
  }
  if (int rc = order_after_caller(ctx)) return rc;
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_sigma, h.data(), ncell * sizeof(double), hipMemcpyHostToDevice, ctx->work));
  tem::launch_mass(ctx->g, ctx->d_sigma, ctx->d_mass, ctx->d_dinv, ctx->d_sqrtm, ctx->work);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipStreamSynchronize(ctx->work));
  ctx->has_sigma = true;
  ctx->fwd_valid = false;
  ctx->fwd_meta = false;
  return TEM_OK;
}

int tem_forward(tem_ctx* ctx, const tem_loop* src, int n_src, const tem_receiver* rx, int n_rx, int T, int J,
                const double* xi, const double* c, const tem_solve_opts* opts, double* data, double* fields,
                tem_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  ctx->fwd_valid = ctx->fwd_meta = false;  // a new forward replaces the stored one, also when it fails
  if (!ctx->has_sigma) return fail(ctx, TEM_ESTATE, "conductivity not set");
  int rc;
  if ((rc = check_loops(ctx, src, n_src))) return rc;
  if (n_rx < 0 || (n_rx > 0 && (!rx || !data))) return fail(ctx, TEM_EINVAL, "bad receiver arguments");
  for (int r = 0; r < n_rx; ++r)
    if (rx[r].i < 0 || rx[r].i >= ctx->nx || rx[r].j < 0 || rx[r].j >= ctx->ny)
      return fail(ctx, TEM_EINVAL, "receiver " + std::to_string(r) + " outside the surface");
  if (T < 1 || T > 64) return fail(ctx, TEM_EINVAL, "T must be in [1, 64]");
  if (J < 1 || J > TEM_MAX_SHIFTS || !xi || !c) return fail(ctx, TEM_EINVAL, "J must be in [1, 64] with xi and c");
  std::vector<double> sre(J), sim(J);
  for (int j = 0; j < J; ++j) {
    if (!std::isfinite(xi[2 * j]) || !std::isfinite(xi[2 * j + 1])) return fail(ctx, TEM_EINVAL, "non-finite pole");
    sre[j] = -xi[2 * j];  // shifts s_j = -xi_j of (K + s_j M) x_j = f
    sim[j] = -xi[2 * j + 1];
    if (sre[j] <= 0.0 && sim[j] == 0.0) return fail(ctx, TEM_EINVAL, "a real pole on x >= 0 makes K - xi M singular");
  }
  for (long long i = 0; i < 2LL * J * T; ++i)
    if (!std::isfinite(c[i])) return fail(ctx, TEM_EINVAL, "non-finite residue");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const tem_solve_opts o = resolve_opts(opts);
  if (o.precision != 0 && o.precision != 1)
    return fail(ctx, TEM_EINVAL, "precision must be 0 (FP64) or 1 (FP32 sweeps + FP64 refinement)");
  double s0 = o.seed_shift;
  if (!(s0 > 0.0)) {
    double minre = 1e300, minabs = 1e300;
    for (int j = 0; j < J; ++j) {
      minre = std::min(minre, sre[j]);
      minabs = std::min(minabs, std::hypot(sre[j], sim[j]));
    }
    s0 = std::max(minre, 1e-3 * minabs);
  }
  if ((rc = order_after_caller(ctx))) return rc;
  hipStream_t st = ctx->work;
  if (o.method == 1) {
    if (o.precision != 0 || o.keep_solutions)
      return fail(ctx, TEM_EINVAL, "the two-pass form (method 1) is FP64 only and keeps no solutions");
    // memory-lean two-pass form: no per-shift vectors; sources one at a time
    if ((rc = ensure_slots(ctx, 1)) || (rc = ensure(ctx, ctx->slots[0].gvec, ctx->n3 * sizeof(double))) ||
        (rc = ensure(ctx, ctx->f, ctx->n3 * sizeof(double))) ||
        (rc = ensure(ctx, ctx->rx, 2 * (size_t)std::max(n_rx, 1) * sizeof(int))))
      return rc;
    std::vector<int> rxi(2 * std::max(n_rx, 1), 0);
    for (int r = 0; r < n_rx; ++r) {
      rxi[2 * r] = rx[r].i;
      rxi[2 * r + 1] = rx[r].j;
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->rx.p, rxi.data(), rxi.size() * sizeof(int), hipMemcpyHostToDevice, st));
    // the shifts on the device, for an adjoint after this forward
    if ((rc = ensure(ctx, ctx->sh, 4 * (size_t)TEM_MAX_SHIFTS * sizeof(double)))) return rc;
    HIPCHK(ctx, hipMemcpyAsync(ctx->sh.p, sre.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync((double*)ctx->sh.p + TEM_MAX_SHIFTS, sim.data(), J * sizeof(double),
                               hipMemcpyHostToDevice, st));
    tem_stats S{};
    S.n_shifts = J;
    S.converged = 1;
    int status = TEM_OK;
    std::vector<double> fs(ctx->n3);
    std::unique_ptr<SolveState> fin(new SolveState());
    for (int s = 0; s < n_src; ++s) {
      loop_source(ctx, src[s], fs);
      HIPCHK(ctx, hipMemcpyAsync(ctx->f.p, fs.data(), ctx->n3 * sizeof(double), hipMemcpyHostToDevice, st));
      tem::launch_scale(ctx->n3, ctx->d_dinv, (const double*)ctx->f.p, (double*)ctx->slots[0].gvec.p, st);
      HIPCHK(ctx, hipGetLastError());
      double secs = 0.0;
      const int r = lanczos_source(ctx, 0, sre, sim, s0, o, T, c, n_rx, n_rx > 0 ? data + (size_t)s * T * n_rx : nullptr,
                                   fields ? fields + (size_t)s * T * ctx->nstore : nullptr, *fin, secs);
      if (r == TEM_ENOCONV) {
        S.converged = 0;
        status = r;
      } else if (r != TEM_OK) {
        return r;
      }
      S.iterations = fin->k;
      for (int j = 0; j < J; ++j) {
        S.iters_per_shift[j] = fin->iters[j];
        S.est_res[j] = fin->est[j] / std::sqrt(fin->rr0);
        S.true_res[j] = -1.0;
        S.unknown_updates += (double)ctx->nunk * fin->iters[j];
      }
    }
    ctx->fwd_valid = false;
    ctx->fwd_meta = true;
    ctx->fwd_J = J;
    ctx->fwd_T = T;
    ctx->fwd_nsrc = n_src;
    ctx->fwd_nrx = n_rx;
    ctx->fwd_xi.assign(xi, xi + 2 * J);
    ctx->fwd_c.assign(c, c + 2 * (size_t)J * T);
    ctx->fwd_rx.assign(rx, rx + n_rx);
    ctx->fwd_src.assign(src, src + n_src);
    ctx->fwd_opts = o;
    ctx->fwd_opts.method = 0;  // an adjoint after this forward recomputes the solutions (FP64, method 0)
    ctx->fwd_s0 = s0;
    S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = S;
    return status;
  }
  const size_t ysz = (size_t)J * ctx->n3 * sizeof(double2);
  const int nconc = std::min(n_src, kMaxConcurrentSolves);  // sources solved at once
  const int nY = o.keep_solutions ? n_src : nconc;
  if ((int)ctx->Y.size() < nY) ctx->Y.resize(nY);
  for (int s = 0; s < nY; ++s)
    if ((rc = ensure(ctx, ctx->Y[s], ysz))) return rc;
  if ((rc = ensure_slots(ctx, nconc))) return rc;
  for (int i = 0; i < nconc; ++i) {
    if ((rc = ensure(ctx, ctx->slots[i].gvec, ctx->n3 * sizeof(double)))) return rc;
  }
  if ((rc = ensure(ctx, ctx->P, (size_t)J * ctx->n3 * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx, ctx->gc, ctx->n3 * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx, ctx->f, ctx->n3 * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->C, 2 * (size_t)J * T * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->rx, 2 * (size_t)std::max(n_rx, 1) * sizeof(int)))) return rc;
  if ((rc = ensure(ctx, ctx->data, (size_t)T * std::max(n_rx, 1) * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->sh, 4 * (size_t)TEM_MAX_SHIFTS * sizeof(double)))) return rc;
  const int cpb = tem::cstencil_partials(ctx->g);
  if ((rc = ensure(ctx, ctx->cpart, (size_t)J * cpb * sizeof(double)))) return rc;
  HIPCHK(ctx, hipMemcpyAsync(ctx->C.p, c, 2 * (size_t)J * T * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<int> rxi(2 * std::max(n_rx, 1), 0);
  for (int r = 0; r < n_rx; ++r) {
    rxi[2 * r] = rx[r].i;
    rxi[2 * r + 1] = rx[r].j;
  }
  HIPCHK(ctx, hipMemcpyAsync(ctx->rx.p, rxi.data(), rxi.size() * sizeof(int), hipMemcpyHostToDevice, st));
  double* shd = (double*)ctx->sh.p;
  HIPCHK(ctx, hipMemcpyAsync(shd, sre.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(shd + TEM_MAX_SHIFTS, sim.data(), J * sizeof(double), hipMemcpyHostToDevice, st));

  tem_stats S{};
  S.n_shifts = J;
  for (int i = 0; i < 4; ++i) {
    ctx->prof_ms[i] = 0.0;
    ctx->prof_n[i] = 0;
  }
  S.converged = 1;
  std::vector<std::vector<double>> fs(nconc, std::vector<double>(ctx->n3));
  std::vector<double> true2(J);
  std::vector<SolveState> states(nconc);
  int status = TEM_OK;
  for (int s_first = 0; s_first < n_src; s_first += nconc) {
    const int nb = std::min(nconc, n_src - s_first);
    // right-hand sides g = M^-1/2 f of this group, one per solve slot
    for (int i = 0; i < nb; ++i) {
      loop_source(ctx, src[s_first + i], fs[i]);
      HIPCHK(ctx, hipMemcpyAsync(ctx->f.p, fs[i].data(), ctx->n3 * sizeof(double), hipMemcpyHostToDevice, st));
      tem::launch_scale(ctx->n3, ctx->d_dinv, (const double*)ctx->f.p, (double*)ctx->slots[i].gvec.p, st);
      HIPCHK(ctx, hipGetLastError());
    }
    double secs = 0.0;
    int r;
    std::vector<double2*> ys(nb);
    for (int i = 0; i < nb; ++i) ys[i] = (double2*)ctx->Y[o.keep_solutions ? s_first + i : i].p;
    if (o.precision == 1) {
      // the sweep accumulates y_j in FP64 and keeps only the search directions
      // p_j in complex FP32; it stops at the recursive tolerance kSweepTolFP32
      // and the FP64 residual refinement below takes over
      tem_solve_opts o32 = o;
      o32.rtol = kSweepTolFP32;
      r = multishift_solve<float2>(ctx, sre, sim, s0, o32, nb, ys.data(), states.data(), secs);
    } else {
      r = multishift_solve<double2>(ctx, sre, sim, s0, o, nb, ys.data(), states.data(), secs);
    }
    if (r == TEM_ENOCONV) {
      S.converged = 0;
      status = r;
    } else if (r != TEM_OK) {
      return r;
    }
    for (int i = 0; i < nb; ++i) {
      const int s = s_first + i;
      double2* Y = (double2*)ctx->Y[o.keep_solutions ? s : i].p;
      const SolveState& hs = states[i];
      S.iterations = hs.k;
      for (int j = 0; j < J; ++j) {
        S.iters_per_shift[j] = hs.iters[j];
        S.est_res[j] = hs.est[j] / std::sqrt(hs.rr0);
        S.unknown_updates += (double)ctx->nunk * hs.iters[j];
      }
      // FP64 true residuals rho_j = g - (A + s_j) y_j into the P buffer (free
      // after the sweep) and ||rho_j||^2 into true2
      tem::launch_to_complex(ctx->n3, (const double*)ctx->slots[i].gvec.p, (double2*)ctx->gc.p, st);
      auto true_residuals = [&]() -> int {
        tem::launch_cstencil(ctx->g, Y, ctx->n3, ctx->d_dinv, shd, shd + TEM_MAX_SHIFTS, J, (const double2*)ctx->gc.p,
                             (double2*)ctx->P.p, ctx->n3, (double*)ctx->cpart.p, st);
        tem::launch_reduce_rows((const double*)ctx->cpart.p, J, cpb, shd + 2 * TEM_MAX_SHIFTS, st);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipMemcpyAsync(true2.data(), shd + 2 * TEM_MAX_SHIFTS, J * sizeof(double), hipMemcpyDeviceToHost,
                                   st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        return TEM_OK;
      };
      if ((rc = true_residuals())) return rc;
      if (verbose()) {
        double w = 0.0;
        for (int j = 0; j < J; ++j) w = std::max(w, std::sqrt(true2[j] / hs.rr0));
        fprintf(stderr, "[tem] source %d: %d seed iterations in %.2f s, max scaled FP64 residual %.2e\n", s, hs.k, secs,
                w);
      }
      if (o.precision == 1) {
        // FP64 residual refinement: (A + s_j) d_j = rho_j by batched COCG with
        // complex FP32 vectors to kRefinePassTol, then the minimal-residual step
        // y_j += omega_j d_j, omega_j = (w_j, rho_j) / (w_j, w_j), w_j = (A + s_j) d_j
        // in FP64, so no pass raises a shift's FP64 residual.  Every pass is
        // bounded: at most kRefinePassCap COCG iterations per shift (later passes
        // at most 16x what the previous one took, and at least 2048), and a shift
        // whose correction residual has not fallen by 10% over kRefineStall
        // iterations stops early.  A shift whose FP64 residual falls by less than
        // 10% in a pass has reached what FP32 corrections can do and is not
        // refined further.
        auto rel = [&](int j) { return std::sqrt(true2[j] / hs.rr0); };
        auto worst = [&]() {
          double w = 0.0;
          for (int j = 0; j < J; ++j) w = std::max(w, rel(j));
          return w;
        };
        std::vector<char> stalled(J, 0);
        std::vector<int> caps(J, std::min(o.max_iter, kRefinePassCap));
        const int nbd = tem::dot_shifts_blocks(ctx->g);
        int passes = 0;
        while (passes < o.refine_max) {
          unsigned long long todo = 0;
          for (int j = 0; j < J; ++j)
            if (!stalled[j] && rel(j) > o.rtol) todo |= 1ull << j;
          if (!todo) break;
          const size_t vn = (size_t)J * ctx->n3;
          if ((rc = ensure(ctx, ctx->refine, 5 * vn * sizeof(float2))) ||
              (rc = ensure(ctx, ctx->refine64, 2 * vn * sizeof(double2))) ||
              (rc = ensure(ctx, ctx->refdot, (size_t)(3 * nbd + 8) * TEM_MAX_SHIFTS * sizeof(double))))
            return rc;
          for (int j = 0; j < J; ++j)  // a zero right-hand side leaves shift j inactive (d_j = 0)
            if (!((todo >> j) & 1ull))
              HIPCHK(ctx, hipMemsetAsync((double2*)ctx->P.p + (size_t)j * ctx->n3, 0, ctx->n3 * sizeof(double2), st));
          float2* v = (float2*)ctx->refine.p;
          tem::CocgState cs;
          int its = 0;
          const int cap = *std::max_element(caps.begin(), caps.end());
          int r2 = cocg_solve(ctx, J, (const double2*)ctx->P.p, v, v + vn, v + 2 * vn, v + 3 * vn, v + 4 * vn,
                              kRefinePassTol, cap, cs, its, caps.data(), kRefineStall);
          if (r2 != TEM_OK && r2 != TEM_ENOCONV) return r2;
          for (int j = 0; j < J; ++j) S.unknown_updates += (double)ctx->nunk * cs.iters[j];
          // a later pass of shift j may take up to 16x the iterations of this
          // one (at least 2048): an FP32 correction that stagnates on a stiff
          // grid would otherwise run to twice the sweep's length every pass
          for (int j = 0; j < J; ++j)
            if ((todo >> j) & 1ull) caps[j] = std::min(caps[j], std::max(2048, 16 * cs.iters[j]));
          // d_j in FP64, w_j = (A + s_j) d_j, dots against rho_j (the P buffer)
          double2* D = (double2*)ctx->refine64.p;
          double2* Wv = D + vn;
          double* dp = (double*)ctx->refdot.p;            // partials, 3 J rows of nbd
          double* dsum = dp + (size_t)3 * nbd * TEM_MAX_SHIFTS;  // 3 J sums
          double* om = dsum + 3 * TEM_MAX_SHIFTS;        // 2 J step lengths
          tem::launch_accumulate(ctx->g, J, v, D, 0, 0, st);
          tem::launch_cstencil(ctx->g, D, ctx->n3, ctx->d_dinv, shd, shd + TEM_MAX_SHIFTS, J, nullptr, Wv, ctx->n3,
                               nullptr, st);
          tem::launch_dot_shifts(ctx->g, J, Wv, (const double2*)ctx->P.p, dp, st);
          tem::launch_reduce_rows(dp, 3 * J, nbd, dsum, st);
          HIPCHK(ctx, hipGetLastError());
          std::vector<double> dots(3 * J), omega(2 * J, 0.0);
          HIPCHK(ctx, hipMemcpyAsync(dots.data(), dsum, 3 * J * sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(ctx, hipStreamSynchronize(st));
          for (int j = 0; j < J; ++j) {
            const double ww = dots[3 * j + 2];
            if (((todo >> j) & 1ull) && ww > 0.0 && std::isfinite(ww)) {
              omega[2 * j] = dots[3 * j] / ww;
              omega[2 * j + 1] = dots[3 * j + 1] / ww;
            }
          }
          HIPCHK(ctx, hipMemcpyAsync(om, omega.data(), 2 * J * sizeof(double), hipMemcpyHostToDevice, st));
          tem::launch_caxpy_shifts(ctx->g, J, om, D, Y, st);
          const std::vector<double> before = true2;
          ++passes;
          if ((rc = true_residuals())) return rc;
          int slow = 0;
          for (int j = 0; j < J; ++j)
            if (((todo >> j) & 1ull) && !(true2[j] < 0.81 * before[j])) {
              ++slow;
              stalled[j] = 1;
            }
          if (verbose())
            fprintf(stderr, "[tem] refinement pass %d: %d COCG iterations, %d shifts reduced by < 10%%, max scaled "
                    "FP64 residual %.2e\n", passes, its, slow, worst());
        }
        S.refine_passes = std::max(S.refine_passes, passes);
        if (worst() > o.rtol) {
          S.converged = 0;
          status = fail(ctx, TEM_ENOCONV, "FP64 residual refinement did not reach rtol within refine_max passes");
        }
      }
      // receivers and (optionally) full fields
      if (n_rx > 0) {
        tem::launch_receivers(ctx->g, Y, J, ctx->d_dinv, (const double*)ctx->C.p, T, (const int*)ctx->rx.p, n_rx,
                              ctx->ks, (double*)ctx->data.p, st);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipMemcpyAsync(data + (size_t)s * T * n_rx, ctx->data.p, (size_t)T * n_rx * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
      }
      if (fields) {
        tem::launch_contract(ctx->g, Y, J, ctx->d_dinv, (const double*)ctx->C.p, T,
                             fields + (size_t)s * T * ctx->nstore, st);
        HIPCHK(ctx, hipGetLastError());
      }
      HIPCHK(ctx, hipStreamSynchronize(st));
      for (int j = 0; j < J; ++j) S.true_res[j] = std::sqrt(true2[j] / hs.rr0);
    }
  }
  ctx->fwd_valid = o.keep_solutions != 0;
  ctx->fwd_meta = true;
  ctx->fwd_J = J;
  ctx->fwd_T = T;
  ctx->fwd_nsrc = n_src;
  ctx->fwd_nrx = n_rx;
  ctx->fwd_xi.assign(xi, xi + 2 * J);
  ctx->fwd_c.assign(c, c + 2 * (size_t)J * T);
  ctx->fwd_rx.assign(rx, rx + n_rx);
  ctx->fwd_src.assign(src, src + n_src);
  ctx->fwd_opts = o;
  ctx->fwd_s0 = s0;
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  for (int i = 0; i < 4; ++i) {
    S.kernel_ms[i] = ctx->prof_ms[i];
    S.kernel_launches[i] = ctx->prof_n[i];
  }
  if (stats) *stats = S;
  return status;
}

int tem_forward_single(tem_ctx* ctx, const tem_loop* src, int n_src, const tem_receiver* rx, int n_rx, int T,
                       const double* t, int J, const double* xi, const double* a, double a0,
                       const tem_solve_opts* opts, double* data, double* fields, tem_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  ctx->fwd_valid = ctx->fwd_meta = false;  // no adjoint follows a single-time forward
  if (!ctx->has_sigma) return fail(ctx, TEM_ESTATE, "conductivity not set");
  int rc;
  if ((rc = check_loops(ctx, src, n_src))) return rc;
  if (n_rx < 0 || (n_rx > 0 && (!rx || !data))) return fail(ctx, TEM_EINVAL, "bad receiver arguments");
  for (int r = 0; r < n_rx; ++r)
    if (rx[r].i < 0 || rx[r].i >= ctx->nx || rx[r].j < 0 || rx[r].j >= ctx->ny)
      return fail(ctx, TEM_EINVAL, "receiver " + std::to_string(r) + " outside the surface");
  if (T < 1 || T > 64 || !t) return fail(ctx, TEM_EINVAL, "T must be in [1, 64] with t");
  if (J < 1 || J > kMaxSinglePoles || !xi || !a) return fail(ctx, TEM_EINVAL, "J must be in [1, 32] with xi and a");
  if (!std::isfinite(a0)) return fail(ctx, TEM_EINVAL, "non-finite alpha0");
  for (int k = 0; k < T; ++k)
    if (!(std::isfinite(t[k]) && t[k] > 0.0)) return fail(ctx, TEM_EINVAL, "channel times must be positive");
  for (int j = 0; j < J; ++j) {
    if (!std::isfinite(xi[2 * j]) || !std::isfinite(xi[2 * j + 1]) || !std::isfinite(a[2 * j]) ||
        !std::isfinite(a[2 * j + 1]))
      return fail(ctx, TEM_EINVAL, "non-finite pole or residue");
    if (xi[2 * j] >= 0.0 && xi[2 * j + 1] == 0.0)
      return fail(ctx, TEM_EINVAL, "a real pole on x >= 0 makes t K - xi M singular");
  }
  const tem_solve_opts o = resolve_opts(opts);
  if (o.precision != 0 || o.method != 0 || o.keep_solutions)
    return fail(ctx, TEM_EINVAL, "the single-time forward is FP64 (precision 0, method 0) and keeps no solutions");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  // the J T systems (t_k K - xi_j M) x = f = t_k (K + s M) x with s = -xi_j / t_k,
  // all on one shared seed recurrence when they fit one solve (kMaxShifts),
  // else ordered by |s| and cut into equal sweeps, each taking shifts of one
  // scale (sweeps routed to a solve engine take at most 64)
  const int Jt = J * T;
  std::vector<int> order(Jt);
  std::vector<double> sre_all(Jt), sim_all(Jt);
  for (int j = 0; j < J; ++j)
    for (int k = 0; k < T; ++k) {
      sre_all[j * T + k] = -xi[2 * j] / t[k];
      sim_all[j * T + k] = -xi[2 * j + 1] / t[k];
    }
  for (int q = 0; q < Jt; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
    return std::hypot(sre_all[u], sim_all[u]) < std::hypot(sre_all[v], sim_all[v]);
  });
  const int cap = uses_engine(ctx) ? TEM_MAX_SHIFTS : tem::kMaxShifts;
  const int nch = (Jt + cap - 1) / cap;
  const int per = (Jt + nch - 1) / nch;
  // coefficients: column q (sorted position) of shift (j, k) feeds channel k
  // with a_j / t_k; column Jt holds g = M^-1/2 f, so alpha0 b = alpha0 M^-1/2 g
  // comes out of the same contraction
  std::vector<double> Ch(2 * (size_t)(Jt + 1) * T, 0.0);
  for (int q = 0; q < Jt; ++q) {
    const int j = order[q] / T, k = order[q] % T;
    Ch[2 * ((size_t)q * T + k)] = a[2 * j] / t[k];
    Ch[2 * ((size_t)q * T + k) + 1] = a[2 * j + 1] / t[k];
  }
  for (int k = 0; k < T; ++k) Ch[2 * ((size_t)Jt * T + k)] = a0;
  if ((rc = order_after_caller(ctx))) return rc;
  hipStream_t st = ctx->work;
  const size_t n3 = ctx->n3;
  const int nconc = std::min(n_src, kMaxConcurrentSolves);
  if ((int)ctx->Y.size() < nconc) ctx->Y.resize(nconc);
  for (int i = 0; i < nconc; ++i)
    if ((rc = ensure(ctx, ctx->Y[i], (size_t)(Jt + 1) * n3 * sizeof(double2)))) return rc;
  if ((rc = ensure_slots(ctx, nconc))) return rc;
  for (int i = 0; i < nconc; ++i)
    if ((rc = ensure(ctx, ctx->slots[i].gvec, n3 * sizeof(double)))) return rc;
  const int cpb = tem::cstencil_partials(ctx->g);
  if ((rc = ensure(ctx, ctx->P, (size_t)TEM_MAX_SHIFTS * n3 * sizeof(double2))) ||
      (rc = ensure(ctx, ctx->gc, n3 * sizeof(double2))) || (rc = ensure(ctx, ctx->f, n3 * sizeof(double))) ||
      (rc = ensure(ctx, ctx->C, Ch.size() * sizeof(double))) ||
      (rc = ensure(ctx, ctx->rx, 2 * (size_t)std::max(n_rx, 1) * sizeof(int))) ||
      (rc = ensure(ctx, ctx->data, (size_t)T * std::max(n_rx, 1) * sizeof(double))) ||
      (rc = ensure(ctx, ctx->sh, 4 * (size_t)TEM_MAX_SHIFTS * sizeof(double))) ||
      (rc = ensure(ctx, ctx->cpart, (size_t)TEM_MAX_SHIFTS * cpb * sizeof(double))))
    return rc;
  HIPCHK(ctx, hipMemcpyAsync(ctx->C.p, Ch.data(), Ch.size() * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<int> rxi(2 * std::max(n_rx, 1), 0);
  for (int r = 0; r < n_rx; ++r) {
    rxi[2 * r] = rx[r].i;
    rxi[2 * r + 1] = rx[r].j;
  }
  HIPCHK(ctx, hipMemcpyAsync(ctx->rx.p, rxi.data(), rxi.size() * sizeof(int), hipMemcpyHostToDevice, st));
  double* shd = (double*)ctx->sh.p;
  tem_stats S{};
  S.n_shifts = Jt;
  S.converged = 1;
  int status = TEM_OK;
  std::vector<std::vector<double>> fs(nconc, std::vector<double>(n3));
  std::vector<SolveState> states(nconc);
  std::vector<double> true2(TEM_MAX_SHIFTS);
  std::vector<double> worst_true(T, 0.0), worst_est(T, 0.0);  // per channel, over sources and poles
  std::vector<int> worst_iters(T, 0);
  for (int s_first = 0; s_first < n_src; s_first += nconc) {
    const int nb = std::min(nconc, n_src - s_first);
    for (int i = 0; i < nb; ++i) {
      loop_source(ctx, src[s_first + i], fs[i]);
      HIPCHK(ctx, hipMemcpyAsync(ctx->f.p, fs[i].data(), n3 * sizeof(double), hipMemcpyHostToDevice, st));
      tem::launch_scale(n3, ctx->d_dinv, (const double*)ctx->f.p, (double*)ctx->slots[i].gvec.p, st);
      HIPCHK(ctx, hipGetLastError());
    }
    std::vector<int> its(nb, 0);
    for (int c0 = 0; c0 < Jt; c0 += per) {
      const int Jc = std::min(per, Jt - c0);
      std::vector<double> sre(Jc), sim(Jc);
      for (int q = 0; q < Jc; ++q) {
        sre[q] = sre_all[order[c0 + q]];
        sim[q] = sim_all[order[c0 + q]];
      }
      double s0 = o.seed_shift;
      if (!(s0 > 0.0)) {
        double minre = 1e300, minabs = 1e300;
        for (int q = 0; q < Jc; ++q) {
          minre = std::min(minre, sre[q]);
          minabs = std::min(minabs, std::hypot(sre[q], sim[q]));
        }
        s0 = std::max(minre, 1e-3 * minabs);
      }
      std::vector<double2*> ys(nb);
      for (int i = 0; i < nb; ++i) ys[i] = (double2*)ctx->Y[i].p + (size_t)c0 * n3;
      double secs = 0.0;
      const int r = multishift_solve<double2>(ctx, sre, sim, s0, o, nb, ys.data(), states.data(), secs);
      if (r == TEM_ENOCONV) {
        S.converged = 0;
        status = r;
      } else if (r != TEM_OK) {
        return r;
      }
      for (int i = 0; i < nb; ++i) {
        const SolveState& hs = states[i];
        its[i] += hs.k;
        tem::launch_to_complex(n3, (const double*)ctx->slots[i].gvec.p, (double2*)ctx->gc.p, st);
        // FP64 true residuals of this sweep's shifts, up to 64 at a time
        for (int q0 = 0; q0 < Jc; q0 += TEM_MAX_SHIFTS) {
          const int nq = std::min(TEM_MAX_SHIFTS, Jc - q0);
          HIPCHK(ctx, hipMemcpyAsync(shd, sre.data() + q0, nq * sizeof(double), hipMemcpyHostToDevice, st));
          HIPCHK(ctx, hipMemcpyAsync(shd + TEM_MAX_SHIFTS, sim.data() + q0, nq * sizeof(double),
                                     hipMemcpyHostToDevice, st));
          tem::launch_cstencil(ctx->g, ys[i] + (size_t)q0 * n3, n3, ctx->d_dinv, shd, shd + TEM_MAX_SHIFTS, nq,
                               (const double2*)ctx->gc.p, (double2*)ctx->P.p, n3, (double*)ctx->cpart.p, st);
          tem::launch_reduce_rows((const double*)ctx->cpart.p, nq, cpb, shd + 2 * TEM_MAX_SHIFTS, st);
          HIPCHK(ctx, hipGetLastError());
          HIPCHK(ctx, hipMemcpyAsync(true2.data(), shd + 2 * TEM_MAX_SHIFTS, nq * sizeof(double),
                                     hipMemcpyDeviceToHost, st));
          HIPCHK(ctx, hipStreamSynchronize(st));
          for (int q = q0; q < q0 + nq; ++q) {
            const int k = order[c0 + q] % T;
            worst_true[k] = std::max(worst_true[k], std::sqrt(true2[q - q0] / hs.rr0));
            worst_est[k] = std::max(worst_est[k], hs.est[q] / std::sqrt(hs.rr0));
            worst_iters[k] = std::max(worst_iters[k], hs.iters[q]);
            S.unknown_updates += (double)ctx->nunk * hs.iters[q];
          }
        }
      }
    }
    for (int i = 0; i < nb; ++i) {
      const int s = s_first + i;
      double2* Y = (double2*)ctx->Y[i].p;
      tem::launch_to_complex(n3, (const double*)ctx->slots[i].gvec.p, Y + (size_t)Jt * n3, st);
      if (n_rx > 0) {
        tem::launch_receivers(ctx->g, Y, Jt + 1, ctx->d_dinv, (const double*)ctx->C.p, T, (const int*)ctx->rx.p,
                              n_rx, ctx->ks, (double*)ctx->data.p, st);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipMemcpyAsync(data + (size_t)s * T * n_rx, ctx->data.p, (size_t)T * n_rx * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
      }
      if (fields) {
        tem::launch_contract(ctx->g, Y, Jt + 1, ctx->d_dinv, (const double*)ctx->C.p, T,
                             fields + (size_t)s * T * ctx->nstore, st);
        HIPCHK(ctx, hipGetLastError());
      }
      HIPCHK(ctx, hipStreamSynchronize(st));
      S.iterations = its[i];
    }
    for (int k = 0; k < T; ++k) {
      S.true_res[k] = worst_true[k];
      S.est_res[k] = worst_est[k];
      S.iters_per_shift[k] = worst_iters[k];
    }
  }
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (stats) *stats = S;
  return status;
}

int tem_solutions(tem_ctx* ctx, int s, double* X) {
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (!ctx->fwd_valid) return fail(ctx, TEM_ESTATE, "no stored solutions (run tem_forward with keep_solutions)");
  if (s < 0 || s >= ctx->fwd_nsrc || !X) return fail(ctx, TEM_EINVAL, "bad source index or NULL output");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int J = ctx->fwd_J;
  DevBuf tmp;
  int rc;
  if ((rc = ensure(ctx, tmp, (size_t)J * ctx->nstore * sizeof(double2)))) return rc;
  tem::launch_gather_solutions(ctx->g, (const double2*)ctx->Y[s].p, J, ctx->d_dinv, (double2*)tmp.p, ctx->work);
  hipError_t e = hipMemcpyAsync(X, tmp.p, (size_t)J * ctx->nstore * sizeof(double2), hipMemcpyDeviceToHost, ctx->work);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->work);
  release(tmp);
  if (e != hipSuccess) return fail(ctx, TEM_EHIP, hipGetErrorString(e));
  return TEM_OK;
}

int tem_apply(tem_ctx* ctx, double shift_re, double shift_im, const double* x, double* y) {
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (!ctx->has_sigma) return fail(ctx, TEM_ESTATE, "conductivity not set");
  if (!x || !y || !std::isfinite(shift_re) || !std::isfinite(shift_im)) return fail(ctx, TEM_EINVAL, "bad arguments");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (int rc0 = order_after_caller(ctx)) return rc0;
  hipStream_t st = ctx->work;
  DevBuf xp, xpad, ypad, shv, part;
  int rc;
  const size_t sb = ctx->nstore * sizeof(double2), pb = ctx->n3 * sizeof(double2);
  if ((rc = ensure(ctx, xp, sb)) || (rc = ensure(ctx, xpad, pb)) || (rc = ensure(ctx, ypad, pb)) ||
      (rc = ensure(ctx, shv, 2 * sizeof(double)))) {
    release(xp); release(xpad); release(ypad); release(shv);
    return rc;
  }
  const double shh[2] = {shift_re, shift_im};
  hipError_t e = hipMemcpyAsync(xp.p, x, sb, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(shv.p, shh, sizeof(shh), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    // y = M^1/2 (A + s) M^1/2 x = K x + s M x on interior edges
    tem::launch_scatter_storage(ctx->g, (const double2*)xp.p, ctx->d_sqrtm, (double2*)xpad.p, st);
    tem::launch_cstencil(ctx->g, (const double2*)xpad.p, 0, ctx->d_dinv, (const double*)shv.p,
                         (const double*)shv.p + 1, 1, nullptr, (double2*)ypad.p, 0, nullptr, st);
    tem::launch_gather_storage(ctx->g, (const double2*)ypad.p, ctx->d_sqrtm, (double2*)xp.p, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(y, xp.p, sb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  release(xp); release(xpad); release(ypad); release(shv); release(part);
  if (e != hipSuccess) return fail(ctx, TEM_EHIP, hipGetErrorString(e));
  return TEM_OK;
}

int tem_apply_noalloc(tem_ctx* ctx, double shift_re, double shift_im, const double* x, double* y) {
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (!ctx->has_sigma) return fail(ctx, TEM_ESTATE, "conductivity not set");
  if (!x || !y || !std::isfinite(shift_re) || !std::isfinite(shift_im)) return fail(ctx, TEM_EINVAL, "bad arguments");
  if (x == y) return fail(ctx, TEM_EINVAL, "x and y must not alias");
  // layout of the array: the shift (re, im) in the first 256 bytes, then the
  // node-padded input and output, 3 nn complex values each
  const size_t pad = (size_t)ctx->n3 * sizeof(double2);
  const size_t need = 256 + 2 * pad;
  if (need > kNoAllocScratchBytes)
    return fail(ctx, TEM_EINVAL, "grid too large for tem_apply_noalloc: needs " + std::to_string(need) +
                                     " bytes of its fixed " + std::to_string(kNoAllocScratchBytes) +
                                     "-byte device array (2 * 3 (nx+1)(ny+1)(nz+1) * 16 + 256)");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (int rc = order_after_caller(ctx)) return rc;
  hipStream_t st = ctx->work;
  double* shv = (double*)ctx->scratch;
  double2* xpad = (double2*)((char*)ctx->scratch + 256);
  double2* ypad = xpad + ctx->n3;
  // the array keeps the previous call's contents (any grid): padding entries
  // are cleared before use, the shift is written by the stream itself
  tem::launch_zero2(2 * ctx->n3, xpad, st);
  tem::launch_store2(shv, shift_re, shift_im, st);
  // y = M^1/2 (A + s) M^1/2 x = K x + s M x on interior edges (as tem_apply)
  tem::launch_scatter_storage(ctx->g, (const double2*)x, ctx->d_sqrtm, xpad, st);
  tem::launch_cstencil(ctx->g, xpad, 0, ctx->d_dinv, shv, shv + 1, 1, nullptr, ypad, 0, nullptr, st);
  tem::launch_gather_storage(ctx->g, ypad, ctx->d_sqrtm, (double2*)y, st);
  HIPCHK(ctx, hipGetLastError());
  // later work on the caller's stream sees y
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, st));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->done_ev, 0));
  return TEM_OK;
}

int tem_adjoint(tem_ctx* ctx, const double* w, double* grad, tem_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (!ctx->fwd_meta) return fail(ctx, TEM_ESTATE, "tem_adjoint needs a preceding tem_forward");
  if (!w || !grad) return fail(ctx, TEM_EINVAL, "w and grad must not be NULL");
  const int J = ctx->fwd_J, T = ctx->fwd_T, n_rx = ctx->fwd_nrx, n_src = ctx->fwd_nsrc;
  if (n_rx < 1) return fail(ctx, TEM_EINVAL, "the forward had no receivers");
  for (long long i = 0; i < (long long)n_src * T * n_rx; ++i)
    if (!std::isfinite(w[i])) return fail(ctx, TEM_EINVAL, "non-finite w");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int rc;
  if ((rc = order_after_caller(ctx))) return rc;
  hipStream_t st = ctx->work;
  // the adjoint solves are FP64, to the FP64 default after a precision-1 forward
  tem_solve_opts o = ctx->fwd_opts;
  if (o.precision == 1) {
    o.precision = 0;
    o.rtol = 1e-12;
  }
  const size_t vb = (size_t)J * ctx->n3 * sizeof(double2);
  DevBuf H, Mu, Rr, Pb, Q, z, gd, gam, cst;
  auto cleanup = [&]() {
    for (DevBuf* b : {&H, &Mu, &Rr, &Pb, &Q, &z, &gd, &gam, &cst}) release(*b);
  };
  const long long ncell = (long long)ctx->nx * ctx->ny * ctx->nz;
  // receiver-row multi-shift solves (up to kAdjointMultishiftMaxRx receivers)
  // or one batched COCG; TEM_ADJOINT=cocg / multishift forces either.  With a
  // solve engine attached, up to kMaxBatchJobs rows share its batched launches.
  bool use_rows = n_rx <= kAdjointMultishiftMaxRx;
  if (const char* m = getenv("TEM_ADJOINT")) {
    if (!strcmp(m, "cocg")) use_rows = false;
    if (!strcmp(m, "multishift")) use_rows = true;
  }
  const int row_conc = std::min(n_rx, uses_engine(ctx) ? tem::kMaxBatchJobs : kMaxConcurrentSolves);
  const int nH = use_rows ? row_conc : 1;
  if ((rc = ensure(ctx, H, nH * vb)) || (rc = ensure(ctx, Mu, vb)) || (rc = ensure(ctx, Rr, vb)) ||
      (rc = ensure(ctx, Pb, 2 * vb)) || (rc = ensure(ctx, Q, vb)) || (rc = ensure(ctx, z, ctx->n3 * sizeof(double))) ||
      (rc = ensure(ctx, gd, ncell * sizeof(double))) || (rc = ensure(ctx, gam, 2 * (size_t)J * n_rx * sizeof(double))) ||
      (rc = ensure(ctx, cst, (size_t)(2 * TEM_MAX_SHIFTS * tem::kMaxBatchJobs * sizeof(double))))) {
    cleanup();
    return rc;
  }
  // shifts s_j = -xi_j on the device (sh buffer of the forward holds them)
  double* shd = (double*)ctx->sh.p;
  std::unique_ptr<tem::CocgState> hs(new tem::CocgState());
  tem_stats S{};
  S.n_shifts = J;
  S.converged = 1;
  std::vector<double> gamma(2 * (size_t)J * n_rx);
  const double* C = ctx->fwd_c.data();
  hipError_t e = hipSuccess;
  for (int s = 0; s < n_src && e == hipSuccess; ++s) {
    // gamma_jr = sum_k c_jk w[s][k][r]  (the adjoint source g_j = sum_r gamma_jr q_r)
    for (int j = 0; j < J; ++j)
      for (int r = 0; r < n_rx; ++r) {
        double gr = 0.0, gi = 0.0;
        for (int k = 0; k < T; ++k) {
          const double wk = w[((size_t)s * T + k) * n_rx + r];
          gr += C[2 * ((size_t)j * T + k)] * wk;
          gi += C[2 * ((size_t)j * T + k) + 1] * wk;
        }
        gamma[2 * ((size_t)j * n_rx + r)] = gr;
        gamma[2 * ((size_t)j * n_rx + r) + 1] = gi;
      }
    e = hipMemcpyAsync(gam.p, gamma.data(), gamma.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    // forward solutions x_j of source s: stored, or recomputed now (one more
    // FP64 multi-shift solve; only one source's solutions are held at a time)
    if (!ctx->fwd_valid) {
      // room for one source's solutions (a two-pass forward holds none)
      if (ctx->Y.empty()) ctx->Y.resize(1);
      if ((rc = ensure(ctx, ctx->Y[0], (size_t)J * ctx->n3 * sizeof(double2)))) {
        cleanup();
        return rc;
      }
    }
    double2* Ys = (double2*)ctx->Y[ctx->fwd_valid ? s : 0].p;
    if (!ctx->fwd_valid) {
      std::vector<double> fsrc(ctx->n3), sre(J), sim(J);
      for (int j = 0; j < J; ++j) {
        sre[j] = -ctx->fwd_xi[2 * j];
        sim[j] = -ctx->fwd_xi[2 * j + 1];
      }
      if ((rc = ensure_slots(ctx, 1)) || (rc = ensure(ctx, ctx->slots[0].gvec, ctx->n3 * sizeof(double)))) {
        cleanup();
        return rc;
      }
      loop_source(ctx, ctx->fwd_src[s], fsrc);
      e = hipMemcpyAsync(ctx->f.p, fsrc.data(), ctx->n3 * sizeof(double), hipMemcpyHostToDevice, st);
      if (e != hipSuccess) break;
      tem::launch_scale(ctx->n3, ctx->d_dinv, (const double*)ctx->f.p, (double*)ctx->slots[0].gvec.p, st);
      const tem_solve_opts& of = o;  // an FP64 solve (o is FP64 here)
      std::unique_ptr<SolveState> fst(new SolveState());
      double secs = 0.0;
      const int r1 = multishift_solve<double2>(ctx, sre, sim, ctx->fwd_s0, of, 1, &Ys, fst.get(), secs);
      if (r1 == TEM_ENOCONV) S.converged = 0;
      else if (r1 != TEM_OK) {
        cleanup();
        return r1;
      }
      for (int j = 0; j < J; ++j) S.unknown_updates += (double)ctx->nunk * fst->iters[j];
    }
    if (use_rows) {
      // lambda_j = sum_r gamma_jr (K + s_j M)^-1 q_r: one multi-shift solve per
      // receiver row (all shifts share its Krylov recurrence), up to
      // kMaxConcurrentSolves rows at once, combined on the device
      e = hipMemsetAsync(Mu.p, 0, vb, st);
      std::vector<double> sre(J), sim(J);
      for (int j = 0; j < J; ++j) {
        sre[j] = -ctx->fwd_xi[2 * j];
        sim[j] = -ctx->fwd_xi[2 * j + 1];
      }
      const int nconc = row_conc;
      if ((rc = ensure_slots(ctx, nconc))) {
        cleanup();
        return rc;
      }
      for (int i = 0; i < nconc; ++i)
        if ((rc = ensure(ctx, ctx->slots[i].gvec, ctx->n3 * sizeof(double)))) {
          cleanup();
          return rc;
        }
      std::vector<std::vector<double>> qrows(nconc, std::vector<double>(ctx->n3));
      std::vector<SolveState> states(nconc);
      std::vector<double> gcol(2 * (size_t)J * nconc);
      for (int r_first = 0; r_first < n_rx && e == hipSuccess; r_first += nconc) {
        const int nb = std::min(nconc, n_rx - r_first);
        for (int i = 0; i < nb && e == hipSuccess; ++i) {
          receiver_row(ctx, ctx->fwd_rx[r_first + i], qrows[i]);
          e = hipMemcpyAsync(ctx->f.p, qrows[i].data(), ctx->n3 * sizeof(double), hipMemcpyHostToDevice, st);
          if (e == hipSuccess)
            tem::launch_scale(ctx->n3, ctx->d_dinv, (const double*)ctx->f.p, (double*)ctx->slots[i].gvec.p, st);
        }
        if (e != hipSuccess) break;
        std::vector<double2*> ys(nb);
        for (int i = 0; i < nb; ++i) ys[i] = (double2*)H.p + (size_t)i * J * ctx->n3;
        double secs = 0.0;
        int r2 = multishift_solve<double2>(ctx, sre, sim, ctx->fwd_s0, o, nb, ys.data(), states.data(), secs);
        if (r2 == TEM_ENOCONV) S.converged = 0;
        else if (r2 != TEM_OK) {
          cleanup();
          return r2;
        }
        for (int i = 0; i < nb; ++i) {
          const SolveState& shs = states[i];
          S.iterations += shs.k;
          for (int j = 0; j < J; ++j) {
            S.iters_per_shift[j] += shs.iters[j];
            S.est_res[j] = std::max(S.est_res[j], shs.est[j] / std::sqrt(shs.rr0));
            S.unknown_updates += (double)ctx->nunk * shs.iters[j];
            gcol[2 * ((size_t)i * J + j)] = gamma[2 * ((size_t)j * n_rx + r_first + i)];
            gcol[2 * ((size_t)i * J + j) + 1] = gamma[2 * ((size_t)j * n_rx + r_first + i) + 1];
          }
        }
        e = hipMemcpyAsync(cst.p, gcol.data(), 2 * (size_t)J * nb * sizeof(double), hipMemcpyHostToDevice, st);
        for (int i = 0; i < nb && e == hipSuccess; ++i) {
          tem::launch_caxpy_shifts(ctx->g, J, (const double*)cst.p + 2 * (size_t)i * J, ys[i], (double2*)Mu.p, st);
          e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // gcol and the rows are reused by the next group
      }
      if (e != hipSuccess) break;
      tem::launch_grad_edges(ctx->g, J, (const double2*)Mu.p, Ys, ctx->d_dinv, shd, shd + TEM_MAX_SHIFTS,
                             (double*)z.p, st);
      continue;
    }
    if (e == hipSuccess) e = hipMemsetAsync(H.p, 0, vb, st);
    if (e != hipSuccess) break;
    tem::launch_adj_rhs(ctx->g, J, n_rx, (const int*)ctx->rx.p, ctx->ks, (const double*)gam.p, ctx->d_dinv,
                        (double2*)H.p, st);
    double2* P0 = (double2*)Pb.p;
    double2* P1 = P0 + (size_t)J * ctx->n3;
    int its = 0;
    const int r3 = cocg_solve(ctx, J, (const double2*)H.p, (double2*)Mu.p, (double2*)Rr.p, P0, P1, (double2*)Q.p,
                              o.rtol, o.max_iter, *hs, its);
    if (r3 == TEM_ENOCONV) {
      S.converged = 0;
    } else if (r3 != TEM_OK) {
      cleanup();
      return r3;
    }
    S.iterations = its;
    for (int j = 0; j < J; ++j) {
      S.iters_per_shift[j] = hs->iters[j];
      S.est_res[j] = hs->hn2[j] > 0 ? std::sqrt(hs->rn2[j] / hs->hn2[j]) : 0.0;
      S.unknown_updates += (double)ctx->nunk * hs->iters[j];
    }
    tem::launch_grad_edges(ctx->g, J, (const double2*)Mu.p, Ys, ctx->d_dinv, shd, shd + TEM_MAX_SHIFTS,
                           (double*)z.p, st);
  }
  if (e == hipSuccess) {
    tem::launch_grad_cells(ctx->g, ctx->d_sigma, (const double*)z.p, (double*)gd.p, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(grad, gd.p, ncell * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return fail(ctx, TEM_EHIP, std::string("adjoint: ") + hipGetErrorString(e));
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (stats) *stats = S;
  return S.converged ? TEM_OK : fail(ctx, TEM_ENOCONV, "adjoint COCG did not reach rtol within max_iter");
}

int tem_jacobian_apply(tem_ctx* ctx, const double* dm, double* ddata, tem_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (!ctx->fwd_valid)
    return fail(ctx, TEM_ESTATE, "tem_jacobian_apply needs a preceding tem_forward with keep_solutions");
  if (!dm || !ddata) return fail(ctx, TEM_EINVAL, "dm and ddata must not be NULL");
  const int J = ctx->fwd_J, T = ctx->fwd_T, n_rx = ctx->fwd_nrx, n_src = ctx->fwd_nsrc;
  if (n_rx < 1) return fail(ctx, TEM_EINVAL, "the forward had no receivers");
  const long long ncell = (long long)ctx->nx * ctx->ny * ctx->nz;
  for (long long i = 0; i < ncell; ++i)
    if (!std::isfinite(dm[i])) return fail(ctx, TEM_EINVAL, "non-finite dm");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int rc;
  if ((rc = order_after_caller(ctx))) return rc;
  hipStream_t st = ctx->work;
  // the sensitivity systems are FP64, to the FP64 default after a precision-1 forward
  tem_solve_opts o = ctx->fwd_opts;
  if (o.precision == 1) o.rtol = 1e-12;
  const size_t vb = (size_t)J * ctx->n3 * sizeof(double2);
  DevBuf H, Mu, Rr, Pb, Q, ddm;
  auto cleanup = [&]() {
    for (DevBuf* b : {&H, &Mu, &Rr, &Pb, &Q, &ddm}) release(*b);
  };
  if ((rc = ensure(ctx, H, vb)) || (rc = ensure(ctx, Mu, vb)) || (rc = ensure(ctx, Rr, vb)) ||
      (rc = ensure(ctx, Pb, 2 * vb)) || (rc = ensure(ctx, Q, vb)) || (rc = ensure(ctx, ddm, ncell * sizeof(double)))) {
    cleanup();
    return rc;
  }
  const double* shd = (const double*)ctx->sh.p;
  std::unique_ptr<tem::CocgState> hs(new tem::CocgState());
  tem_stats S{};
  S.n_shifts = J;
  S.converged = 1;
  hipError_t e = hipMemcpyAsync(ddm.p, dm, ncell * sizeof(double), hipMemcpyHostToDevice, st);
  for (int s = 0; s < n_src && e == hipSuccess; ++s) {
    // h_j = -s_j (dM/M) y_j, then (A + s_j) dy_j = h_j by batched COCG (a
    // different right-hand side per shift), then the receivers of
    // Re sum_j c_jk dx_j, as in the forward
    tem::launch_jvp_rhs(ctx->g, J, ctx->d_sigma, (const double*)ddm.p, ctx->d_mass, shd, shd + TEM_MAX_SHIFTS,
                        (const double2*)ctx->Y[s].p, (double2*)H.p, st);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    double2* P0 = (double2*)Pb.p;
    double2* P1 = P0 + (size_t)J * ctx->n3;
    int its = 0;
    const int r3 = cocg_solve(ctx, J, (const double2*)H.p, (double2*)Mu.p, (double2*)Rr.p, P0, P1, (double2*)Q.p,
                              o.rtol, o.max_iter, *hs, its);
    if (r3 == TEM_ENOCONV) {
      S.converged = 0;
    } else if (r3 != TEM_OK) {
      cleanup();
      return r3;
    }
    S.iterations = its;
    for (int j = 0; j < J; ++j) {
      S.iters_per_shift[j] = hs->iters[j];
      S.est_res[j] = hs->hn2[j] > 0 ? std::sqrt(hs->rn2[j] / hs->hn2[j]) : 0.0;
      S.unknown_updates += (double)ctx->nunk * hs->iters[j];
    }
    tem::launch_receivers(ctx->g, (const double2*)Mu.p, J, ctx->d_dinv, (const double*)ctx->C.p, T,
                          (const int*)ctx->rx.p, n_rx, ctx->ks, (double*)ctx->data.p, st);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(ddata + (size_t)s * T * n_rx, ctx->data.p, (size_t)T * n_rx * sizeof(double),
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  cleanup();
  if (e != hipSuccess) return fail(ctx, TEM_EHIP, std::string("jacobian: ") + hipGetErrorString(e));
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (stats) *stats = S;
  return S.converged ? TEM_OK : fail(ctx, TEM_ENOCONV, "sensitivity COCG did not reach rtol within max_iter");
}

int tem_engine_create(tem_engine** out, int device, int max_jobs) {
  if (!out) return fail(nullptr, TEM_EINVAL, "engine pointer is NULL");
  *out = nullptr;
  if (max_jobs <= 0) max_jobs = tem::kMaxBatchJobs;
  if (max_jobs > tem::kMaxBatchJobs) return fail(nullptr, TEM_EINVAL, "max_jobs must be at most 16");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, TEM_EHIP, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, TEM_EHIP, "hipSetDevice failed");
  std::unique_ptr<tem_engine> E(new tem_engine());
  E->device = device;
  E->max_jobs = max_jobs;
  auto chk = [&](hipError_t e, const char* what) -> int {
    if (e == hipSuccess) return TEM_OK;
    return fail(nullptr, TEM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  const size_t tab = (size_t)tem_engine::kGens * tem::kMaxBatchJobs * sizeof(tem::BatchJob);
  int rc;
  if ((rc = chk(hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking), "engine stream")) ||
      (rc = chk(hipMalloc(&E->d_tables, tab), "engine tables")) ||
      (rc = chk(hipHostMalloc((void**)&E->h_tables, tab, hipHostMallocDefault), "engine tables")) ||
      (rc = chk(hipMalloc(&E->d_heads, tem::kMaxBatchJobs * sizeof(tem::SolveHead)), "engine heads")) ||
      (rc = chk(hipHostMalloc((void**)&E->h_heads, 2 * tem::kMaxBatchJobs * sizeof(tem::SolveHead),
                              hipHostMallocDefault), "engine heads")) ||
      (rc = chk(hipEventCreateWithFlags(&E->head_ev[0], hipEventDisableTiming), "engine events")) ||
      (rc = chk(hipEventCreateWithFlags(&E->head_ev[1], hipEventDisableTiming), "engine events"))) {
    tem_engine_destroy(E.release());
    return rc;
  }
  E->worker = std::thread(engine_worker, E.get());
  *out = E.release();
  return TEM_OK;
}

int tem_attach_engine(tem_ctx* ctx, tem_engine* eng) {
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (eng) {
    if (eng->device != ctx->device) return fail(ctx, TEM_EINVAL, "engine and context are on different devices");
    int ntx = 0, nty = 0;
    if (tem::batch_tiles(ctx->g, &ntx, &nty) > tem::kReduceSlots)
      return fail(ctx, TEM_EINVAL, "grid too large for batched launches: more tiles than partial-sum slots");
  }
  ctx->engine = eng;
  return TEM_OK;
}

int tem_engine_stats(tem_engine* eng, long long* blocks, long long* job_blocks, int* max_jobs, int* max_contexts) {
  if (!eng) return fail(nullptr, TEM_EINVAL, "engine is NULL");
  std::lock_guard<std::mutex> lk(eng->mu);
  if (blocks) *blocks = eng->blocks;
  if (job_blocks) *job_blocks = eng->job_blocks;
  if (max_jobs) *max_jobs = eng->max_jobs_seen;
  if (max_contexts) *max_contexts = eng->max_ctx_seen;
  return TEM_OK;
}

void tem_engine_destroy(tem_engine* eng) {
  if (!eng) return;
  (void)hipSetDevice(eng->device);
  if (eng->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(eng->mu);
      eng->stop = true;
    }
    eng->cv.notify_all();
    eng->worker.join();
  }
  if (eng->stream) (void)hipStreamSynchronize(eng->stream);
  for (hipEvent_t e : eng->head_ev)
    if (e) (void)hipEventDestroy(e);
  if (eng->d_tables) (void)hipFree(eng->d_tables);
  if (eng->h_tables) (void)hipHostFree(eng->h_tables);
  if (eng->d_heads) (void)hipFree(eng->d_heads);
  if (eng->h_heads) (void)hipHostFree(eng->h_heads);
  if (eng->stream) (void)hipStreamDestroy(eng->stream);
  delete eng;
}

int tem_sizes(const tem_ctx* ctx, long long* n_storage, long long* n_unknowns) {
  if (!ctx) return fail(nullptr, TEM_EINVAL, "ctx is NULL");
  if (n_storage) *n_storage = ctx->nstore;
  if (n_unknowns) *n_unknowns = ctx->nunk;
  return TEM_OK;
}

void tem_destroy(tem_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  if (ctx->work) hipStreamSynchronize(ctx->work);
  for (SolveSlot& sl : ctx->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    if (sl.stream2) hipStreamSynchronize(sl.stream2);
  }
  for (double* p : {ctx->d_axis, ctx->d_sigma, ctx->d_mass, ctx->d_dinv, ctx->d_sqrtm})
    if (p) hipFree(p);
  if (ctx->d_counters) hipFree(ctx->d_counters);
  for (DevBuf* b : {&ctx->gc, &ctx->f, &ctx->P, &ctx->C, &ctx->rx, &ctx->data, &ctx->res, &ctx->cpart, &ctx->sh,
                    &ctx->refine, &ctx->cst, &ctx->cocg_part, &ctx->refine64, &ctx->refdot})
    release(*b);
  for (DevBuf& b : ctx->Y) release(b);
  for (SolveSlot& sl : ctx->slots) release_slot(sl);
  if (ctx->order_ev) hipEventDestroy(ctx->order_ev);
  if (ctx->work_ev) hipEventDestroy(ctx->work_ev);
  if (ctx->done_ev) hipEventDestroy(ctx->done_ev);
  if (ctx->work) hipStreamDestroy(ctx->work);
  delete ctx;
}

const char* tem_last_error(const tem_ctx* ctx) { return ctx ? ctx->err.c_str() : g_global_error.c_str(); }

int tem_poles(int T, const double* t, const double* w, int degree, double tol, int J_max, int* J, double* xi,
              double* c, double* err) {
  if (T < 1 || T > 64 || !t || !J || !xi || !c) return fail(nullptr, TEM_EINVAL, "bad arguments to tem_poles");
  std::vector<double> tv(t, t + T), wv(T, 1.0);
  for (int k = 0; k < T; ++k)
    if (!(std::isfinite(tv[k]) && tv[k] > 0.0)) return fail(nullptr, TEM_EINVAL, "channel times must be positive");
  if (w) {
    for (int k = 0; k < T; ++k) {
      if (!(std::isfinite(w[k]) && w[k] > 0.0)) return fail(nullptr, TEM_EINVAL, "weights must be positive");
      wv[k] = w[k];
    }
  }
  if (degree == 0) {
    const double ratio = *std::max_element(tv.begin(), tv.end()) / *std::min_element(tv.begin(), tv.end());
    if (!(tol > 0.0)) return fail(nullptr, TEM_EINVAL, "degree 0 needs a positive tol");
    degree = tem::table1_degree(ratio, tol);
    if (degree <= 0) return fail(nullptr, TEM_EINVAL, "no Table 1 degree for this ratio and tolerance");
  }
  if (degree < 2 || degree > 2 * TEM_MAX_SHIFTS) return fail(nullptr, TEM_EINVAL, "degree must be in [2, 128]");
  tem::RkfitResult res;
  std::string msg;
  int rc = tem::rkfit(tv, wv, degree, res, msg);
  if (rc != TEM_OK) return fail(nullptr, rc, msg);
  const int nJ = (int)res.xi.size();
  if (nJ > J_max) return fail(nullptr, TEM_EINVAL, "J_max too small for the fitted poles");
  *J = nJ;
  for (int j = 0; j < nJ; ++j) {
    xi[2 * j] = res.xi[j].real();
    xi[2 * j + 1] = res.xi[j].imag();
    for (int k = 0; k < T; ++k) {
      c[2 * ((size_t)j * T + k)] = res.c[(size_t)j * T + k].real();
      c[2 * ((size_t)j * T + k) + 1] = res.c[(size_t)j * T + k].imag();
    }
  }
  if (err)
    for (int k = 0; k < T; ++k) err[k] = res.err[k];
  return TEM_OK;
}

int tem_poles_single(int m, int* J, double* xi, double* a, double* alpha0, double* err) {
  if (m < 1 || m > kMaxSinglePoles || !J || !xi || !a || !alpha0)
    return fail(nullptr, TEM_EINVAL, "bad arguments to tem_poles_single (m must be in [1, 32])");
  tem::SingleResult res;
  std::string msg;
  const int rc = tem::best_rational(m, res, msg);
  if (rc != TEM_OK) return fail(nullptr, rc, msg);
  const int nJ = (int)res.xi.size();
  *J = nJ;
  for (int j = 0; j < nJ; ++j) {
    xi[2 * j] = res.xi[j].real();
    xi[2 * j + 1] = res.xi[j].imag();
    a[2 * j] = res.a[j].real();
    a[2 * j + 1] = res.a[j].imag();
  }
  *alpha0 = res.a0;
  if (err) *err = res.err;
  return TEM_OK;
}

}  // extern "C"
