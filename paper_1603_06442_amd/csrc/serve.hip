// Continuous-batching server for Fourier evolutions of particle states.
//
// Requests (dimension, lattice, mass, state, time, precision) are queued by
// qw_server_submit. A worker thread admits them in arrival order while the
// device memory they need fits the byte budget, groups admitted requests of
// the same shape and precision into batches of up to max_batch, and runs
// each batch on one of several streams: state preparation (Sec. 5.1,
// Definition 1 and the Sec. 5.2 superposition), the Fourier evolution to each
// request's own time with its own mass (Sec. 4), and the position / norm
// reductions of Sec. 5.2 about the request's centre. Completion is signalled
// from the stream itself (a host function after the result copy); memory is
// returned to a pool and waiting requests are admitted at once, so requests
// that arrive while others are on the device join as capacity frees up.
// Every kernel treats the instances of a batch independently and the
// reduction order depends only on the shape, so a request's result is the
// same whether it ran alone or in a mix.
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "plan.h"

using namespace qw;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Key {
  int dim;
  int64_t N[3];
  int dtype;
  bool operator<(const Key& o) const {
    return std::tie(dim, N[0], N[1], N[2], dtype) < std::tie(o.dim, o.N[0], o.N[1], o.N[2], o.dtype);
  }
};

struct Pending {
  int64_t ticket;
  qw_request req;
  double t_submit;
  size_t footprint;
  Key key;
};

// Pool of device / pinned blocks by power-of-two size class.
struct Pool {
  std::map<size_t, std::vector<void*>> dev_free, host_free;
  std::vector<void*> dev_all, host_all;
  static size_t cls(size_t b) {
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
  }
  hipError_t get_dev(size_t b, void** out) {
    const size_t c = cls(b);
    auto& v = dev_free[c];
    if (!v.empty()) {
      *out = v.back();
      v.pop_back();
      return hipSuccess;
    }
    hipError_t e = hipMalloc(out, c);
    if (e == hipSuccess) dev_all.push_back(*out);
    return e;
  }
  hipError_t get_host(size_t b, void** out) {
    const size_t c = cls(b);
    auto& v = host_free[c];
    if (!v.empty()) {
      *out = v.back();
      v.pop_back();
      return hipSuccess;
    }
    hipError_t e = hipHostMalloc(out, c, hipHostMallocDefault);
    if (e == hipSuccess) host_all.push_back(*out);
    return e;
  }
  void put_dev(size_t b, void* p) { dev_free[cls(b)].push_back(p); }
  void put_host(size_t b, void* p) { host_free[cls(b)].push_back(p); }
  void release() {
    for (void* p : dev_all) (void)hipFree(p);
    for (void* p : host_all) (void)hipHostFree(p);
    dev_all.clear();
    host_all.clear();
    dev_free.clear();
    host_free.clear();
  }
};

struct Batch;

// A captured batch chain: the device and pinned-host buffers of one batch of
// B requests of one shape, and an instantiated HIP graph of everything that
// batch enqueues (parameter upload, state preparation, evolution with the
// fused reductions, result copies), recorded against those buffers. A batch
// of the same shape and size that finds an idle slot writes its parameters
// into the slot's pinned buffer and replays the graph: one launch instead of
// the chain's copies and kernels.
struct GraphSlot {
  int dim;
  int64_t N[3];
  int dtype;
  int B;
  void* dmem = nullptr;
  void* hmem = nullptr;
  size_t dbytes = 0, hbytes = 0;
  hipGraphExec_t exec = nullptr;  // null until captured (or if the capture failed)
  bool busy = false;
  uint64_t last_use = 0;
  qw_plan_t plan = nullptr;       // for the deferred capture
  bool capture_failed = false;    // not tried again; the chain runs directly
};

}  // namespace

struct qw_server_s {
  size_t budget = 0, used = 0, peak_used = 0;
  int64_t cancelled = 0;
  size_t laid_out = 0, peak_laid_out = 0;  // device bytes of the in-flight batches' layouts
  int max_batch = 1;
  int device = 0;
  std::vector<hipStream_t> streams;
  hipStream_t plan_stream = nullptr;  // plan set-up only
  int next_stream = 0;
  std::mutex mu;
  std::condition_variable cv;       // worker wake-up
  std::condition_variable cv_done;  // result waiters
  std::deque<Pending> queue;
  std::vector<Batch*> inflight;
  std::vector<Batch*> finished;     // signalled by the stream, not yet retired
  std::unordered_map<int64_t, qw_result> results;  // completed, not yet collected
  std::unordered_set<int64_t> live;                // submitted, not yet collected
  std::map<Key, qw_plan_t> plans;
  Pool pool;
  std::thread worker;
  bool stop = false;
  bool hold = false;      // admit nothing while set
  int max_inflight = 2;   // batches on the device at once (per server)
  int64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, batches = 0, peak_inflight = 0;
  std::string worker_error;
  // Graph replay of batches (see GraphSlot): slots are touched by the
  // worker thread only.
  bool use_graphs = true;
  bool autotune = true;
  int max_slots = 256;
  // Direct runs so far of each (shape, precision, batch size): a chain is
  // captured on its second direct run, so batch sizes seen once cost no
  // capture.
  std::map<std::tuple<int, int64_t, int64_t, int64_t, int, int>, int> chain_runs;
  std::vector<GraphSlot*> slots;
  size_t slot_bytes = 0;  // device bytes held by the slots
  uint64_t slot_clock = 0;
  int64_t graphs_captured = 0, graph_launches = 0;
  int64_t launch_host_ns = 0;  // host time spent enqueuing batches (worker thread)
  // Slots whose chain is still to be captured: the worker records the
  // captures when it has no batch to form, so that a capture never delays
  // the requests waiting in the queue.
  std::vector<GraphSlot*> to_capture;
};

namespace {

// Device and pinned-host layout of one batch of B requests of one shape:
// the fields (and the four-step transpose buffer), the per-instance state,
// apply and origin parameters, the partial sums of the state preparation and
// the reductions, the sector norms and the results, each 256-byte aligned.
// Every part is B times a per-instance size that does not depend on B, so a
// batch's layout never exceeds the sum of its requests' own layouts (which is
// what admission charges against the budget).
struct Layout {
  size_t off_field, off_scratch, off_sinst, off_inst, off_orig, off_part, off_norm, off_res;
  size_t dbytes;
  size_t h_sinst, h_inst, h_orig, h_res, h_norm;
  size_t hbytes;
  int64_t nbo, nbf;  // reduction blocks per instance: separate pass, fused pass (0: none)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout batch_layout(const Key& k, int B) {
  Layout L;
  const bool dbl = k.dtype == QW_C128;
  const int s = k.dim == 1 ? 2 : 4;
  int64_t V = 1;
  StateGeom sg;
  memset(&sg, 0, sizeof sg);
  ObsGeom og;
  memset(&og, 0, sizeof og);
  sg.dim = og.dim = k.dim;
  sg.s = og.s = s;
  for (int i = 0; i < 3; ++i) sg.N[i] = og.N[i] = i < k.dim ? k.N[i] : 1;
  for (int i = 0; i < k.dim; ++i) V *= k.N[i];
  sg.V = og.V = V;
  const size_t fb = (size_t)V * s * (dbl ? 16 : 8);
  const bool fourstep = k.dim == 1 && k.N[0] > kFourStepL;
  L.nbo = observables_blocks(og, B);
  L.nbf = (int64_t)s * fused_obs_blocks_of(k.dim, k.N, dbl);
  size_t o = 0;
  L.off_field = o;
  o = align256(o + fb * B);
  L.off_scratch = o;
  if (fourstep) o = align256(o + fb * B);
  L.off_sinst = o;
  o = align256(o + sizeof(StateInst) * B);
  L.off_inst = o;
  o = align256(o + sizeof(InstParam) * B);
  L.off_orig = o;
  o = align256(o + sizeof(double) * 3 * B);
  L.off_part = o;
  o = align256(o + sizeof(double) * std::max<int64_t>(
                       state_scratch_doubles(sg, B),
                       (int64_t)B * (std::max<int64_t>(L.nbo, L.nbf) * kObsFields + 64 * kObsFields)));
  L.off_norm = o;
  o = align256(o + sizeof(double) * 2 * B);
  L.off_res = o;
  o = align256(o + sizeof(double) * kObsFields * B);
  L.dbytes = o;
  size_t h = 0;
  L.h_sinst = h;
  h = align256(h + sizeof(StateInst) * B);
  L.h_inst = h;
  h = align256(h + sizeof(InstParam) * B);
  L.h_orig = h;
  h = align256(h + sizeof(double) * 3 * B);
  L.h_res = h;
  h = align256(h + sizeof(double) * kObsFields * B);
  L.h_norm = h;
  h = align256(h + sizeof(double) * 2 * B);
  L.hbytes = h;
  return L;
}

struct Batch {
  qw_server_s* srv;
  Key key;
  qw_plan_t plan;
  std::vector<Pending> reqs;
  Layout lay;
  void* dmem = nullptr;
  void* hmem = nullptr;
  size_t footprint = 0;
  hipStream_t st = nullptr;
  GraphSlot* slot = nullptr;  // buffers of a graph slot (else of the pool)
  bool replayed = false;
  double t_launch = 0.0, t_done = 0.0;
  qw_status status = QW_OK;
};

Key key_of(const qw_request& r) {
  Key k;
  k.dim = r.dim;
  for (int i = 0; i < 3; ++i) k.N[i] = i < r.dim ? r.N[i] : 1;
  k.dtype = (int)r.dtype;
  return k;
}

// Device bytes a request is charged at admission: its own one-request layout.
size_t request_footprint(const qw_request& r) { return batch_layout(key_of(r), 1).dbytes; }

qw_status validate(const qw_request* r) {
  if (!r) return fail(QW_ERR_INVALID, "request is NULL");
  if (r->dim < 1 || r->dim > 3) return fail(QW_ERR_INVALID, "dim must be 1, 2 or 3");
  if (r->dtype != QW_C64 && r->dtype != QW_C128) return fail(QW_ERR_INVALID, "unknown dtype");
  const int64_t maxN = r->dim == 1 ? 65536 : (r->dim == 2 ? 1024 : 512);
  for (int i = 0; i < r->dim; ++i) {
    const int64_t n = r->N[i];
    if (n < 2 || n > maxN || (n & (n - 1)))
      return fail(QW_ERR_UNSUPPORTED, "N[%d] = %lld unsupported", i, (long long)n);
    if (!isfinite(r->k0[i]) || !isfinite(r->center[i]))
      return fail(QW_ERR_INVALID, "k0 / center not finite");
  }
  if (!(r->m >= 0.0 && r->m <= 1.0)) return fail(QW_ERR_INVALID, "m must lie in [0, 1]");
  if (!(r->sigma > 0.0) || !isfinite(r->sigma)) return fail(QW_ERR_INVALID, "sigma must be > 0");
  if (!isfinite(r->c_plus) || !isfinite(r->c_minus) || (r->c_plus == 0.0 && r->c_minus == 0.0))
    return fail(QW_ERR_INVALID, "c_plus, c_minus must be finite and not both zero");
  if (r->t > (int64_t(1) << 53) || r->t < -(int64_t(1) << 53))
    return fail(QW_ERR_UNSUPPORTED, "|t| must be at most 2^53");
  return QW_OK;
}

void on_stream_done(void* arg) {
  Batch* b = (Batch*)arg;
  qw_server_s* s = b->srv;
  b->t_done = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  s->finished.push_back(b);
  s->cv.notify_all();
}

// Per-instance parameters of a batch into its pinned buffer H.
void fill_params(Batch* b, char* H) {
  const int B = (int)b->reqs.size();
  qw_plan_t p = b->plan;
  const Layout& Ly = b->lay;
  StateInst* hs = (StateInst*)(H + Ly.h_sinst);
  InstParam* hi = (InstParam*)(H + Ly.h_inst);
  double* ho = (double*)(H + Ly.h_orig);
  for (int k = 0; k < B; ++k) {
    const qw_request& r = b->reqs[k].req;
    hs[k] = make_state_inst(p, r.m, r.k0, r.sigma, r.center, r.c_plus, r.c_minus);
    hi[k].m = r.m;
    hi[k].n = sqrt(1.0 - r.m * r.m);
    hi[k].t = (double)r.t;
    for (int i = 0; i < 3; ++i) ho[3 * k + i] = i < r.dim ? r.center[i] : 0.0;
  }
}

// Everything one batch enqueues on st, against device buffer D and pinned
// buffer H (already holding the parameters): one upload of the parameters,
// the state preparation, the evolution with the reductions, the result
// copies. Only copies and kernels: the same chain can be captured.
qw_status enqueue_chain(qw_plan_t p, int B, const Layout& Ly, char* D, char* H, hipStream_t st) {
  const StateGeom sg = state_geom(p);
  const ObsGeom og = obs_geom(p);
  const int64_t nbf = Ly.nbf;  // 0: separate reduction pass
  // one upload of the three parameter arrays (contiguous in both layouts)
  HIP_TRY(hipMemcpyAsync(D + Ly.off_sinst, H + Ly.h_sinst, Ly.h_res - Ly.h_sinst,
                         hipMemcpyHostToDevice, st));
  void* field = D + Ly.off_field;
  void* scratch = p->fourstep ? (void*)(D + Ly.off_scratch) : nullptr;
  double* part = (double*)(D + Ly.off_part);
  HIP_TRY(launch_state_prepare(p->dbl, sg, B, (const StateInst*)(D + Ly.off_sinst), part,
                               (double*)(D + Ly.off_norm), field, st));
  // The state is prepared as its spectrum: apply D_q^t there and invert once.
  // The 1D four-step keeps its transposed spectrum internal, so it goes to
  // position space and through the full evolution. Where the schedule ends
  // with a strided pass, the reductions are fused into it and psi(t) is
  // never written.
  const InstParam* dinst = (const InstParam*)(D + Ly.off_inst);
  const double* origins = (const double*)(D + Ly.off_orig);
  double* res = (double*)(D + Ly.off_res);
  const ObsFuse fuse = make_fuse(p, nullptr, origins, part, false);
  const ObsFuse* fz = nbf > 0 ? &fuse : nullptr;
  qw_status r;
  if (!p->fourstep) {
    r = evolve_spectrum_impl(p, B, field, dinst, st, fz);
  } else {
    r = transform_impl(p, B, field, field, -1, scratch, st);
    if (r == QW_OK) {
      InstParam unused;
      unused.m = 0.0;
      unused.n = 1.0;
      unused.t = 0;
      r = evolve_impl(p, B, field, field, dinst, unused, st, fz);
    }
  }
  if (r != QW_OK) return r;
  if (fz)
    HIP_TRY(launch_reduce_partials(B, nbf, part, part + (size_t)B * nbf * kObsFields, res, st));
  else
    HIP_TRY(launch_observables(p->dbl, og, B, field, nullptr, origins, part, res, st));
  HIP_TRY(hipMemcpyAsync(H + Ly.h_res, D + Ly.off_res, sizeof(double) * kObsFields * B,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(H + Ly.h_norm, D + Ly.off_norm, sizeof(double) * 2 * B,
                         hipMemcpyDeviceToHost, st));
  return QW_OK;
}

bool slot_matches(const GraphSlot* g, const Batch* b) {
  return g->dim == b->key.dim && g->N[0] == b->key.N[0] && g->N[1] == b->key.N[1] &&
         g->N[2] == b->key.N[2] && g->dtype == b->key.dtype && g->B == (int)b->reqs.size();
}

void drop_slot(qw_server_s* s, GraphSlot* g) {  // worker thread, slot idle
  auto pc = std::find(s->to_capture.begin(), s->to_capture.end(), g);
  if (pc != s->to_capture.end()) s->to_capture.erase(pc);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  s->pool.put_dev(g->dbytes, g->dmem);
  s->pool.put_host(g->hbytes, g->hmem);
  s->slot_bytes -= g->dbytes;
  s->slots.erase(std::find(s->slots.begin(), s->slots.end(), g));
  delete g;
}

// A new slot for batch b (its buffers from the pool), after evicting the
// least recently used idle slots while there are max_slots slots or the
// slots hold more than the budget. Null if none can be made.
GraphSlot* new_slot(qw_server_s* s, Batch* b) {
  for (;;) {
    const bool full = (int)s->slots.size() >= s->max_slots ||
                      s->slot_bytes + b->lay.dbytes > s->budget;
    if (!full) break;
    GraphSlot* lru = nullptr;
    for (GraphSlot* g : s->slots)
      if (!g->busy && (!lru || g->last_use < lru->last_use)) lru = g;
    if (!lru) return nullptr;
    drop_slot(s, lru);
  }
  GraphSlot* g = new GraphSlot();
  g->dim = b->key.dim;
  for (int i = 0; i < 3; ++i) g->N[i] = b->key.N[i];
  g->dtype = b->key.dtype;
  g->B = (int)b->reqs.size();
  g->plan = b->plan;
  g->dbytes = b->lay.dbytes;
  g->hbytes = b->lay.hbytes;
  if (s->pool.get_dev(g->dbytes, &g->dmem) != hipSuccess) {
    delete g;
    return nullptr;
  }
  if (s->pool.get_host(g->hbytes, &g->hmem) != hipSuccess) {
    s->pool.put_dev(g->dbytes, g->dmem);
    delete g;
    return nullptr;
  }
  s->slots.push_back(g);
  s->slot_bytes += g->dbytes;
  return g;
}

// Runs with the lock NOT held, on the worker thread. With graphs, a batch
// replays the graph of an idle slot of its shape and size; otherwise it
// takes a new slot, runs the chain eagerly on its buffers and captures the
// chain into the slot's graph (recorded on the set-up stream, not run) for
// the batches after it. Without graphs (or without a slot) the buffers come
// from the pool and the chain runs eagerly.
qw_status launch_batch(qw_server_s* s, Batch* b) {
  hipStream_t st = b->st;
  GraphSlot* g = nullptr;
  if (s->use_graphs) {
    GraphSlot* uncaptured = nullptr;  // an idle slot whose capture is pending
    for (GraphSlot* c : s->slots)
      if (!c->busy && slot_matches(c, b)) {
        if (c->exec) {
          g = c;
          break;
        }
        uncaptured = c;
      }
    if (g) {
      g->busy = true;
      g->last_use = ++s->slot_clock;
      b->slot = g;
      b->replayed = true;
      fill_params(b, (char*)g->hmem);
      HIP_TRY(hipGraphLaunch(g->exec, st));
      ++s->graph_launches;
      HIP_TRY(hipLaunchHostFunc(st, on_stream_done, b));
      return QW_OK;
    }
    const auto ck = std::make_tuple(b->key.dim, b->key.N[0], b->key.N[1], b->key.N[2],
                                    b->key.dtype, (int)b->reqs.size());
    if (++s->chain_runs[ck] >= 2) g = uncaptured ? uncaptured : new_slot(s, b);
  }
  char* D;
  char* H;
  if (g) {
    g->busy = true;
    g->last_use = ++s->slot_clock;
    b->slot = g;
    D = (char*)g->dmem;
    H = (char*)g->hmem;
  } else {
    HIP_TRY(s->pool.get_dev(b->lay.dbytes, &b->dmem));
    HIP_TRY(s->pool.get_host(b->lay.hbytes, &b->hmem));
    D = (char*)b->dmem;
    H = (char*)b->hmem;
  }
  fill_params(b, H);
  qw_status r = enqueue_chain(b->plan, (int)b->reqs.size(), b->lay, D, H, st);
  if (r != QW_OK) return r;
  HIP_TRY(hipLaunchHostFunc(st, on_stream_done, b));
  // captured when the worker is idle (once per slot)
  if (g && !g->capture_failed &&
      std::find(s->to_capture.begin(), s->to_capture.end(), g) == s->to_capture.end())
    s->to_capture.push_back(g);
  return QW_OK;
}

// Records the chain of slot g against its buffers (on the set-up stream,
// which runs nothing while capturing) and instantiates it. Worker thread,
// lock not held.
void capture_slot(qw_server_s* s, GraphSlot* g) {
  const Key k{g->dim, {g->N[0], g->N[1], g->N[2]}, g->dtype};
  const Layout Ly = batch_layout(k, g->B);
  hipStream_t cs = s->plan_stream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    const qw_status rc = enqueue_chain(g->plan, g->B, Ly, (char*)g->dmem, (char*)g->hmem, cs);
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc == QW_OK && e == hipSuccess && graph &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
      g->exec = exec;
      ++s->graphs_captured;
    }
    if (graph) (void)hipGraphDestroy(graph);
  }
  if (!g->exec) g->capture_failed = true;
  (void)hipGetLastError();
}

void retire(qw_server_s* s, Batch* b) {  // lock held
  const int B = (int)b->reqs.size();
  const char* H = (const char*)(b->slot ? b->slot->hmem : b->hmem);
  const double* R = (const double*)(H + b->lay.h_res);
  const double* NR = (const double*)(H + b->lay.h_norm);
  for (int k = 0; k < B; ++k) {
    const Pending& pd = b->reqs[k];
    qw_result res;
    memset(&res, 0, sizeof res);
    res.ticket = pd.ticket;
    res.status = b->status;
    res.batch_size = B;
    res.queue_s = b->t_launch - pd.t_submit;
    res.latency_s = b->t_done - pd.t_submit;
    if (b->status == QW_OK) {
      finish_obs(b->plan, R + (size_t)k * kObsFields, pd.req.center, &res.obs);
      res.obs.overlap_re = res.obs.overlap_im = res.obs.ref_norm2 = 0.0;
      res.sector_norm2[0] = NR[2 * k];
      res.sector_norm2[1] = NR[2 * k + 1];
      if ((pd.req.c_plus != 0.0 && !(NR[2 * k] > 0.0)) || (pd.req.c_minus != 0.0 && !(NR[2 * k + 1] > 0.0)))
        res.status = QW_ERR_INVALID;
    }
    s->results[pd.ticket] = res;
    ++s->completed;
  }
  if (b->slot) b->slot->busy = false;
  if (b->dmem) s->pool.put_dev(b->lay.dbytes, b->dmem);
  if (b->hmem) s->pool.put_host(b->lay.hbytes, b->hmem);
  s->used -= b->footprint;
  s->laid_out -= b->lay.dbytes;
  s->inflight.erase(std::find(s->inflight.begin(), s->inflight.end(), b));
  delete b;
  s->cv_done.notify_all();
}

// Worker thread only, server lock NOT held: plan creation synchronises its
// own stream, and a completion host function queued on a serving stream
// takes the server lock, so no HIP call may be made while holding it.
// With autotuning, the schedule (workgroup size and pencil groups of the
// pass along the contiguous axis) is timed once per shape on a second plan of
// that shape, whose scratch field is released with it, and copied over.
qw_plan_t make_plan(qw_server_s* s, const Key& k) {
  qw_plan_t p = nullptr;
  if (qw_plan(&p, k.dim, k.N, 0.0, (qw_dtype)k.dtype, s->plan_stream) != QW_OK) return nullptr;
  if (s->autotune) {
    qw_plan_t tp = nullptr;
    if (qw_plan(&tp, k.dim, k.N, 0.0, (qw_dtype)k.dtype, s->plan_stream) == QW_OK) {
      int sl, ce, cb, gw;
      if (qw_autotune(tp, s->plan_stream, nullptr) == QW_OK &&
          qw_get_schedule(tp, &sl, &ce, &cb, &gw) == QW_OK)
        (void)qw_set_schedule(p, sl, ce, cb, gw);
      (void)hipStreamSynchronize(s->plan_stream);
      delete tp;  // its work is done; qw_destroy would wait for the whole device
    }
  }
  return p;
}

void worker_main(qw_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // retire batches whose stream has signalled
    while (!s->finished.empty()) {
      Batch* b = s->finished.back();
      s->finished.pop_back();
      retire(s, b);
    }
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    // Batches are formed while fewer than max_inflight are on the device, so
    // requests that arrive while it is busy gather into the next batches. The
    // oldest queued request always opens the next batch (no starvation); the
    // batch then takes the later queued requests of the same shape, in
    // arrival order, while they fit the budget.
    std::vector<Batch*> ready;
    while (!s->hold && !s->queue.empty() &&
           (int)(s->inflight.size() + ready.size()) < s->max_inflight) {
      Pending& head = s->queue.front();
      if (s->used + head.footprint > s->budget) break;  // wait for memory
      const Key key = head.key;
      qw_plan_t p = nullptr;
      auto pit = s->plans.find(key);
      if (pit != s->plans.end()) {
        p = pit->second;
      } else {
        // Only this thread removes from the queue, so head stays in front.
        lk.unlock();
        p = make_plan(s, key);
        lk.lock();
        if (p) s->plans[key] = p;
      }
      if (!p) {
        Pending& pd = s->queue.front();
        qw_result res;
        memset(&res, 0, sizeof res);
        res.ticket = pd.ticket;
        res.status = QW_ERR_DEVICE;
        s->results[pd.ticket] = res;
        ++s->completed;
        s->queue.pop_front();
        s->cv_done.notify_all();
        continue;
      }
      Batch* b = new Batch();
      b->srv = s;
      b->key = key;
      b->plan = p;
      b->st = s->streams[s->next_stream];
      s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
      for (auto it = s->queue.begin();
           it != s->queue.end() && (int)b->reqs.size() < s->max_batch;) {
        if (it->key.dim == key.dim && it->key.N[0] == key.N[0] && it->key.N[1] == key.N[1] &&
            it->key.N[2] == key.N[2] && it->key.dtype == key.dtype &&
            s->used + it->footprint <= s->budget) {
          s->used += it->footprint;
          b->footprint += it->footprint;
          b->reqs.push_back(*it);
          it = s->queue.erase(it);
        } else {
          ++it;
        }
      }
      s->peak_used = std::max(s->peak_used, s->used);
      b->lay = batch_layout(key, (int)b->reqs.size());
      s->laid_out += b->lay.dbytes;
      s->peak_laid_out = std::max(s->peak_laid_out, s->laid_out);
      ready.push_back(b);
    }
    if (!ready.empty()) {
      for (Batch* b : ready) s->inflight.push_back(b);
      s->batches += (int64_t)ready.size();
      s->peak_inflight = std::max<int64_t>(s->peak_inflight, (int64_t)s->inflight.size());
      lk.unlock();
      for (Batch* b : ready) {
        b->t_launch = now_s();
        b->status = launch_batch(s, b);
        s->launch_host_ns += (int64_t)((now_s() - b->t_launch) * 1e9);
        if (b->status != QW_OK) {
          // the stream still runs whatever was enqueued; mark and signal when it drains
          (void)hipStreamSynchronize(b->st);
          on_stream_done(b);
        }
      }
      lk.lock();
      continue;
    }
    if (!s->to_capture.empty() && s->finished.empty()) {
      // nothing to form now: record one deferred capture
      GraphSlot* g = s->to_capture.back();
      s->to_capture.pop_back();
      lk.unlock();
      capture_slot(s, g);
      lk.lock();
      continue;
    }
    s->cv.wait(lk);
  }
}

}  // namespace

extern "C" {

// QW_HBM_BUDGET: bytes, with an optional K, M or G suffix (powers of 1024).
static size_t env_budget() {
  const char* v = getenv("QW_HBM_BUDGET");
  if (!v || !*v) return 0;
  char* end = nullptr;
  const double x = strtod(v, &end);
  if (!(x > 0.0)) return 0;
  double mul = 1.0;
  if (end && (*end == 'K' || *end == 'k')) mul = 1024.0;
  if (end && (*end == 'M' || *end == 'm')) mul = 1024.0 * 1024.0;
  if (end && (*end == 'G' || *end == 'g')) mul = 1024.0 * 1024.0 * 1024.0;
  return (size_t)(x * mul);
}

qw_status qw_server_create(qw_server_t* out, size_t budget_bytes, int max_batch, int nstreams) {
  if (!out) return fail(QW_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (budget_bytes == 0) {
    budget_bytes = env_budget();
    if (budget_bytes == 0) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
        return fail(QW_ERR_DEVICE, "hipMemGetInfo failed (pass a budget)");
      budget_bytes = free_b / 2;
    }
  }
  if (budget_bytes < (1u << 20)) return fail(QW_ERR_INVALID, "budget must be at least 1 MiB");
  if (max_batch < 1 || max_batch > 4096) return fail(QW_ERR_INVALID, "max_batch must lie in [1, 4096]");
  if (nstreams < 1 || nstreams > 16) return fail(QW_ERR_INVALID, "nstreams must lie in [1, 16]");
  qw_server_s* s = new (std::nothrow) qw_server_s();
  if (!s) return fail(QW_ERR_NOMEM, "host allocation failed");
  s->budget = budget_bytes;
  s->max_batch = max_batch;
  s->max_inflight = 2 * nstreams;
  (void)hipGetDevice(&s->device);
  for (int i = 0; i <= nstreams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      if (s->plan_stream) (void)hipStreamDestroy(s->plan_stream);
      delete s;
      return fail(QW_ERR_DEVICE, "stream creation failed");
    }
    if (i == nstreams)
      s->plan_stream = st;
    else
      s->streams.push_back(st);
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return QW_OK;
}

qw_status qw_server_configure(qw_server_t s, int use_graphs, int autotune, int max_graphs) {
  if (!s) return fail(QW_ERR_INVALID, "server is NULL");
  if (max_graphs < 1 || max_graphs > 4096) return fail(QW_ERR_INVALID, "max_graphs must lie in [1, 4096]");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->submitted > 0) return fail(QW_ERR_INVALID, "configure before the first submit");
  s->use_graphs = use_graphs != 0;
  s->autotune = autotune != 0;
  s->max_slots = max_graphs;
  return QW_OK;
}

qw_status qw_server_submit(qw_server_t s, const qw_request* req, int64_t* ticket) {
  if (!s || !ticket) return fail(QW_ERR_INVALID, "NULL argument");
  qw_status r = validate(req);
  if (r != QW_OK) return r;
  Pending pd;
  pd.req = *req;
  for (int i = req->dim; i < 3; ++i) {
    pd.req.N[i] = 1;
    pd.req.k0[i] = 0.0;
    pd.req.center[i] = 0.0;
  }
  pd.footprint = request_footprint(pd.req);
  if (pd.footprint > s->budget)
    return fail(QW_ERR_NOMEM, "request needs %zu bytes, budget is %zu", pd.footprint, s->budget);
  pd.key = key_of(pd.req);
  pd.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(QW_ERR_INVALID, "server is shutting down");
    pd.ticket = s->next_ticket++;
    s->live.insert(pd.ticket);
    ++s->submitted;
    s->queue.push_back(pd);
  }
  s->cv.notify_all();
  *ticket = pd.ticket;
  return QW_OK;
}

qw_status qw_server_poll(qw_server_t s, int64_t ticket, qw_result* out, int* done) {
  if (!s || !out || !done) return fail(QW_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->live.count(ticket)) return fail(QW_ERR_INVALID, "unknown or already collected ticket");
  auto it = s->results.find(ticket);
  if (it == s->results.end()) {
    *done = 0;
    return QW_OK;
  }
  *out = it->second;
  *done = 1;
  s->results.erase(it);
  s->live.erase(ticket);
  s->cv_done.notify_all();
  return QW_OK;
}

qw_status qw_server_wait(qw_server_t s, int64_t ticket, qw_result* out) {
  if (!s || !out) return fail(QW_ERR_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->live.count(ticket)) return fail(QW_ERR_INVALID, "unknown or already collected ticket");
  s->cv_done.wait(lk, [&] { return s->results.count(ticket) > 0 || !s->live.count(ticket); });
  if (!s->results.count(ticket)) return fail(QW_ERR_INVALID, "result collected by another caller");
  *out = s->results[ticket];
  s->results.erase(ticket);
  s->live.erase(ticket);
  s->cv_done.notify_all();
  return QW_OK;
}

qw_status qw_server_cancel(qw_server_t s, int64_t ticket, int* cancelled) {
  if (!s || !cancelled) return fail(QW_ERR_INVALID, "NULL argument");
  *cancelled = 0;
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->live.count(ticket)) return fail(QW_ERR_INVALID, "unknown or already collected ticket");
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    if (it->ticket != ticket) continue;
    qw_result res;
    memset(&res, 0, sizeof res);
    res.ticket = ticket;
    res.status = QW_ERR_CANCELLED;
    res.queue_s = res.latency_s = now_s() - it->t_submit;
    s->results[ticket] = res;
    ++s->completed;
    ++s->cancelled;
    s->queue.erase(it);
    *cancelled = 1;
    s->cv_done.notify_all();
    s->cv.notify_all();
    break;
  }
  return QW_OK;
}

qw_status qw_server_wait_for(qw_server_t s, int64_t ticket, double timeout_s, qw_result* out,
                             int* done) {
  if (!s || !out || !done) return fail(QW_ERR_INVALID, "NULL argument");
  if (!(timeout_s >= 0.0)) return fail(QW_ERR_INVALID, "timeout must be >= 0");
  *done = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->live.count(ticket)) return fail(QW_ERR_INVALID, "unknown or already collected ticket");
  auto finished = [&] { return s->results.count(ticket) > 0 || !s->live.count(ticket); };
  bool ready;
  if (timeout_s >= 1e9) {  // beyond what a clock duration can hold: no limit
    s->cv_done.wait(lk, finished);
    ready = true;
  } else {
    ready = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished);
  }
  if (!ready) return QW_OK;  // timed out: the request stays live
  if (!s->results.count(ticket)) return fail(QW_ERR_INVALID, "result collected by another caller");
  *out = s->results[ticket];
  s->results.erase(ticket);
  s->live.erase(ticket);
  *done = 1;
  s->cv_done.notify_all();
  return QW_OK;
}

qw_status qw_server_hold(qw_server_t s, int hold) {
  if (!s) return fail(QW_ERR_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->hold = hold != 0;
  }
  s->cv.notify_all();
  return QW_OK;
}

qw_status qw_server_stats(qw_server_t s, qw_server_info* out) {
  if (!s || !out) return fail(QW_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->batches = s->batches;
  out->queued = (int64_t)s->queue.size();
  out->inflight_batches = (int64_t)s->inflight.size();
  out->max_inflight_batches = s->peak_inflight;
  out->used_bytes = (int64_t)s->used;
  out->peak_used_bytes = (int64_t)s->peak_used;
  out->laid_out_bytes = (int64_t)s->laid_out;
  out->peak_laid_out_bytes = (int64_t)s->peak_laid_out;
  out->graphs_captured = s->graphs_captured;
  out->graph_launches = s->graph_launches;
  out->slot_bytes = (int64_t)s->slot_bytes;
  out->launch_host_ns = s->launch_host_ns;
  out->budget_bytes = (int64_t)s->budget;
  out->cancelled = s->cancelled;
  return QW_OK;
}

qw_status qw_server_destroy(qw_server_t s) {
  if (!s) return QW_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->hold = false;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (GraphSlot* g : s->slots) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    delete g;  // buffers belong to the pool, released below
  }
  s->slots.clear();
  for (auto& kv : s->plans) qw_destroy(kv.second);
  s->pool.release();
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  (void)hipStreamDestroy(s->plan_stream);
  delete s;
  return QW_OK;
}

}  // extern "C"
