// Serving engine: continuous batching of cross-section requests over resident
// processes (declarations in include/heget.h).
//
// A request asks for heget_integrate(process, n, sqrt_s, seed), optionally with
// its per-event |M|^2 copied to a host buffer.  One scheduler thread
//   * admits queued requests in arrival order while their device footprint
//     (per-block partials, and the |M|^2 buffer if asked for) fits the arena,
//     a single allocation made at creation;
//   * for every process, fuses the admitted requests' pending blocks into one
//     launch of the process's persistent batch kernel (at most max_chunk_blocks
//     of one request per launch, max_batch_blocks in all), replaying a HIP graph
//     captured at creation: table upload -> persistent kernel -> reduction of
//     the requests that finish in this launch -> result download;
//   * runs slots_per_process such launches per process on their own streams,
//     so launches of different processes, and of one process, overlap;
//   * polls the launches' events, finishes requests and frees their memory.
// Every request's blocks keep the Philox counters, partial-sum slots and
// reduction order of a heget_integrate of that request alone, so its result
// is bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "heget_internal.hpp"
#include "reduce.hpp"

using heget::BatchTable;
using heget::KernelArgs;
using heget::detail::fail;

namespace {

// Final reductions of the requests whose last blocks ran in this launch:
// block j reduces job j exactly as heget_integrate's reduction does.
__global__ __launch_bounds__(256) void reduce_jobs(BatchTable* bt) {
  const int j = blockIdx.x;
  if (j >= bt->n_jobs) return;  // uniform over the block
  heget::reduce_triples(bt->job[j].partials, bt->job[j].nblocks, bt->result[j]);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation, 256-byte granules.
class Arena {
 public:
  static constexpr size_t npos = ~size_t(0);
  hipError_t init(size_t bytes) {
    cap_ = bytes;
    free_.clear();
    free_[0] = bytes;
    return hipMalloc(&base_, bytes);
  }
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  size_t alloc(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used_ += bytes;
      high_ = std::max(high_, used_);
      return off;
    }
    return npos;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* base() const { return base_; }
  size_t capacity() const { return cap_; }
  size_t high_water() const { return high_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0, high_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  int proc = 0;
  int64_t n = 0, nblocks = 0;
  uint64_t seed = 0;
  double sqrt_s = 0, weight_factor = 0;
  double* me2_host = nullptr;
  size_t bytes = 0, off = Arena::npos;
  double* d_part = nullptr;
  double* d_me2 = nullptr;
  int64_t next_block = 0;  // first block not yet dispatched
  bool in_flight = false;
  bool done = false;
  heget_status status = HEGET_OK;
  std::string error;
  double t_submit = 0, t_done = 0;
  heget_result result{};
};

struct Slot {
  int proc = 0;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  BatchTable* d_table = nullptr;
  BatchTable* h_table = nullptr;  // pinned; read by the graph's upload node
  hipGraphExec_t exec = nullptr;
  void* d_work = nullptr;         // persistent kernels: this slot's own workspace
  bool busy = false;
  std::vector<Request*> seg_req;  // request of each segment
  std::vector<Request*> job_req;  // request of each reduction job
};

}  // namespace

struct heget_server {
  std::vector<heget_process_t> procs;
  heget_server_config cfg{};
  int device = 0;
  Arena arena;
  std::vector<std::unique_ptr<Slot>> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> inbox;                       // submitted, not yet seen by the scheduler
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  heget_server_stats stats{};

  // scheduler-thread state
  std::deque<Request*> queue;                       // waiting for admission, arrival order
  std::vector<std::vector<Request*>> admitted;      // per process, admission order
  std::thread thread;

  void run();
  bool dispatch(Slot& s);
  void complete(Slot& s);
  void finish(Request* r, heget_status st, const std::string& err);
  void abort_batch(Slot& s, const std::string& err);
};

// A launch failed: its requests end with an error and are never dispatched again.
void heget_server::abort_batch(Slot& s, const std::string& err) {
  s.busy = false;
  for (Request* r : s.seg_req) {
    r->in_flight = false;
    r->next_block = r->nblocks;
    if (r->done) continue;
    auto& lst = admitted[r->proc];
    auto it = std::find(lst.begin(), lst.end(), r);
    if (it != lst.end()) lst.erase(it);
    finish(r, HEGET_E_HIP, err);
  }
}

void heget_server::finish(Request* r, heget_status st, const std::string& err) {
  if (r->off != Arena::npos) arena.release(r->off, r->bytes);
  r->off = Arena::npos;
  std::lock_guard<std::mutex> lk(mu);
  r->status = st;
  r->error = err;
  r->t_done = now_s();
  r->done = true;
  ++stats.requests_done;
  cv_done.notify_all();
}

bool heget_server::dispatch(Slot& s) {
  BatchTable& t = *s.h_table;
  t.n_seg = 0;
  t.n_jobs = 0;
  int64_t total = 0, events = 0;
  s.seg_req.clear();
  s.job_req.clear();
  for (Request* r : admitted[s.proc]) {
    if (r->in_flight || r->next_block >= r->nblocks) continue;
    if (t.n_seg == heget::kMaxSegments || total >= cfg.max_batch_blocks) break;
    const int64_t take = std::min<int64_t>({r->nblocks - r->next_block, int64_t(cfg.max_chunk_blocks),
                                             int64_t(cfg.max_batch_blocks) - total});
    const bool last = r->next_block + take == r->nblocks;
    if (last && t.n_jobs == heget::kMaxJobs) break;
    heget::Segment& g = t.seg[t.n_seg++];
    g.block_begin = total;
    g.block_offset = r->next_block;
    g.n = r->n;
    g.seed = r->seed;
    g.sqrt_s = r->sqrt_s;
    g.weight_factor = r->weight_factor;
    g.me2_out = r->d_me2;
    g.partials = r->d_part;
    s.seg_req.push_back(r);
    if (last) {
      t.job[t.n_jobs].partials = r->d_part;
      t.job[t.n_jobs].nblocks = r->nblocks;
      ++t.n_jobs;
      s.job_req.push_back(r);
    }
    events += std::min<int64_t>(take * 256, r->n - r->next_block * 256);
    r->next_block += take;
    r->in_flight = true;
    total += take;
  }
  if (t.n_seg == 0) return false;
  t.total_blocks = total;
  hipError_t e = hipGraphLaunch(s.exec, s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
  if (e != hipSuccess) {
    abort_batch(s, std::string("batch launch: ") + hipGetErrorString(e));
    return true;
  }
  s.busy = true;
  int busy = 0;
  for (auto& x : slots) busy += x->busy;
  std::lock_guard<std::mutex> lk(mu);
  ++stats.launches;
  stats.segments += t.n_seg;
  stats.events += events;
  stats.max_busy_slots = std::max<int32_t>(stats.max_busy_slots, busy);
  return true;
}

void heget_server::complete(Slot& s) {
  s.busy = false;
  for (Request* r : s.seg_req) r->in_flight = false;
  for (size_t j = 0; j < s.job_req.size(); ++j) {
    Request* r = s.job_req[j];
    heget::detail::fill_result(s.h_table->result[j], r->n, &r->result);
    heget_status st = HEGET_OK;
    std::string err;
    if (r->me2_host) {
      hipError_t e = hipMemcpyAsync(r->me2_host, r->d_me2, size_t(r->n) * sizeof(double), hipMemcpyDeviceToHost,
                                    s.stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
      if (e != hipSuccess) {
        st = HEGET_E_HIP;
        err = std::string("|M|^2 download: ") + hipGetErrorString(e);
      }
    }
    auto& lst = admitted[r->proc];
    lst.erase(std::find(lst.begin(), lst.end(), r));
    finish(r, st, err);
  }
}

void heget_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    bool progressed = false;
    {
      std::lock_guard<std::mutex> lk(mu);
      while (!inbox.empty()) {
        queue.push_back(inbox.front());
        inbox.pop_front();
      }
    }
    // admission in arrival order while the footprint fits
    while (!queue.empty()) {
      Request* r = queue.front();
      const size_t off = arena.alloc(r->bytes);
      if (off == Arena::npos) break;
      r->off = off;
      char* base = arena.base() + off;
      r->d_part = reinterpret_cast<double*>(base);
      r->d_me2 = r->me2_host ? reinterpret_cast<double*>(base + Arena::round(size_t(r->nblocks) * 24)) : nullptr;
      admitted[r->proc].push_back(r);
      queue.pop_front();
      progressed = true;
    }
    for (auto& s : slots) {
      if (!s->busy) continue;
      const hipError_t q = hipEventQuery(s->done);
      if (q == hipSuccess) {
        complete(*s);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        abort_batch(*s, std::string("batch: ") + hipGetErrorString(q));
        progressed = true;
      }
    }
    for (auto& s : slots)
      if (!s->busy && dispatch(*s)) progressed = true;
    if (progressed) continue;
    std::unique_lock<std::mutex> lk(mu);
    bool idle = queue.empty();
    for (auto& s : slots) idle = idle && !s->busy;
    if (stop && inbox.empty() && idle) break;
    // woken by a submission; otherwise poll the in-flight launches again soon
    cv_work.wait_for(lk, std::chrono::microseconds(idle ? 2000 : 50));
  }
}

namespace {

void destroy_server(heget_server* s) {
  for (auto& sl : s->slots) {
    if (sl->exec) (void)hipGraphExecDestroy(sl->exec);
    if (sl->done) (void)hipEventDestroy(sl->done);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    if (sl->d_table) (void)hipFree(sl->d_table);
    if (sl->h_table) (void)hipHostFree(sl->h_table);
    if (sl->d_work) (void)hipFree(sl->d_work);
  }
  delete s;
}

// Capture the fixed launch sequence of one slot into a graph.
heget_status capture_slot(heget_server* s, Slot& sl) {
  heget_process_t p = s->procs[sl.proc];
  const void* fn = p->prec == HEGET_FP64 ? p->entry->batch_fp64 : p->entry->batch_mixed;
  const int grid = heget::detail::resident_blocks(fn);
  KernelArgs a = heget::detail::base_args(p);
  a.batch = sl.d_table;
  if (p->entry->persistent) {
    // the slot's own workspace: launches of one process on several slots run concurrently
    const size_t wb = size_t(grid) * size_t(p->work_stride) * heget::detail::complex_bytes(p);
    if (hipMalloc(&sl.d_work, wb) != hipSuccess) return fail(HEGET_E_OOM, "slot workspace allocation failed");
    a.work = sl.d_work;
  }
  void* args[] = {&a};
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t c = hipMemcpyAsync(sl.d_table, sl.h_table, sizeof(BatchTable), hipMemcpyHostToDevice, sl.stream);
    if (c == hipSuccess) c = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(256), args, 0, sl.stream);
    if (c == hipSuccess) {
      hipLaunchKernelGGL(reduce_jobs, dim3(heget::kMaxJobs), dim3(256), 0, sl.stream, sl.d_table);
      c = hipGetLastError();
    }
    if (c == hipSuccess)
      c = hipMemcpyAsync(sl.h_table->result, sl.d_table->result, sizeof(sl.h_table->result), hipMemcpyDeviceToHost,
                         sl.stream);
    e = hipStreamEndCapture(sl.stream, &graph);
    if (c != hipSuccess) e = c;
  }
  if (e == hipSuccess) e = hipGraphInstantiateWithFlags(&sl.exec, graph, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  return HEGET_OK;
}

}  // namespace

extern "C" {

heget_status heget_server_create(const heget_server_config* cfg, heget_server_t* out) {
  if (!cfg || !out) return fail(HEGET_E_INVALID, "null argument");
  *out = nullptr;
  if (cfg->n_processes < 1 || !cfg->processes) return fail(HEGET_E_INVALID, "no processes");
  if (cfg->arena_bytes < (1 << 20) || cfg->slots_per_process < 1 || cfg->slots_per_process > 8 ||
      cfg->max_batch_blocks < 1 || cfg->max_chunk_blocks < 1)
    return fail(HEGET_E_INVALID, "bad server configuration");
  for (int k = 0; k < cfg->n_processes; ++k)
    if (!cfg->processes[k]) return fail(HEGET_E_INVALID, "null process handle");
  auto* s = new heget_server();
  s->cfg = *cfg;
  s->procs.assign(cfg->processes, cfg->processes + cfg->n_processes);
  s->admitted.resize(cfg->n_processes);
  if (hipGetDevice(&s->device) != hipSuccess || s->arena.init(size_t(cfg->arena_bytes)) != hipSuccess) {
    destroy_server(s);
    return fail(HEGET_E_OOM, "arena allocation failed");
  }
  for (int k = 0; k < cfg->n_processes; ++k)
    for (int j = 0; j < cfg->slots_per_process; ++j) {
      auto sl = std::make_unique<Slot>();
      sl->proc = k;
      Slot& r = *sl;
      s->slots.push_back(std::move(sl));
      if (hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess ||
          hipMalloc(&r.d_table, sizeof(BatchTable)) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&r.h_table), sizeof(BatchTable), hipHostMallocDefault) != hipSuccess) {
        destroy_server(s);
        return fail(HEGET_E_OOM, "slot allocation failed");
      }
      std::memset(r.h_table, 0, sizeof(BatchTable));
      if (heget_status st = capture_slot(s, r)) {
        destroy_server(s);
        return st;
      }
    }
  s->thread = std::thread([s] { s->run(); });
  *out = s;
  return HEGET_OK;
}

heget_status heget_server_submit(heget_server_t s, int32_t process, int64_t n, uint64_t seed, double sqrt_s,
                                 double* me2_host, uint64_t* ticket) {
  if (!s || !ticket) return fail(HEGET_E_INVALID, "null argument");
  if (process < 0 || process >= int(s->procs.size())) return fail(HEGET_E_INVALID, "process index out of range");
  if (n < 2) return fail(HEGET_E_INVALID, "need n >= 2 events");
  if (!(sqrt_s > 0)) return fail(HEGET_E_INVALID, "sqrt_s must be > 0");
  auto r = std::make_unique<Request>();
  r->proc = process;
  r->n = n;
  r->nblocks = (n + 255) / 256;
  r->seed = seed;
  r->sqrt_s = sqrt_s;
  r->weight_factor = heget::detail::weight_factor(s->procs[process], sqrt_s);
  r->me2_host = me2_host;
  r->bytes = Arena::round(size_t(r->nblocks) * 24) + (me2_host ? Arena::round(size_t(n) * sizeof(double)) : 0);
  if (r->bytes > s->arena.capacity()) return fail(HEGET_E_INVALID, "request footprint exceeds the arena");
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(HEGET_E_INVALID, "server is shutting down");
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->inbox.push_back(r.get());
  s->reqs.emplace(r->ticket, std::move(r));
  ++s->stats.requests_submitted;
  s->cv_work.notify_one();
  return HEGET_OK;
}

heget_status heget_server_poll(heget_server_t s, uint64_t ticket, int32_t wait, heget_result* out,
                               double* latency_s, int32_t* done) {
  if (!s || !out || !done) return fail(HEGET_E_INVALID, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(HEGET_E_INVALID, "unknown ticket");
  Request* r = it->second.get();
  if (wait) s->cv_done.wait(lk, [r] { return r->done; });
  *done = r->done ? 1 : 0;
  if (!r->done) return HEGET_OK;
  const heget_status st = r->status;
  const std::string err = r->error;
  *out = r->result;
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  s->reqs.erase(it);
  if (st != HEGET_OK) return fail(st, err);
  return HEGET_OK;
}

heget_status heget_server_stats_get(heget_server_t s, heget_server_stats* out) {
  if (!s || !out) return fail(HEGET_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->arena_high_water = int64_t(s->arena.high_water());
  return HEGET_OK;
}

heget_status heget_server_destroy(heget_server_t s) {
  if (!s) return fail(HEGET_E_INVALID, "null handle");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_one();
  }
  if (s->thread.joinable()) s->thread.join();
  for (auto& sl : s->slots)
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
  destroy_server(s);
  return HEGET_OK;
}

}  // extern "C"
