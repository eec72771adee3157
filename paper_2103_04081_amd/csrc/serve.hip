// C ABI of libcpdmi: the request server (cpd_server_*, cpd_submit, cpd_poll).
//
// Two host threads per server:
//   the round thread: launch round_steps steps of every running request (one
//     launch of the persistent step kernel per rank-tile class, the classes
//     concurrently on two streams) and one fit check of all of them on the
//     step stream; wait; hand out the requests
//     that stopped; install the requests admitted meanwhile; repeat;
//   the admission thread: take waiting requests in order as slots and arena
//     space free up and initialise them on the admission stream (staging,
//     layout, distributions, ||X||^2), concurrently with the rounds.
// Device memory comes from the caller's arena: a small header (descriptor
// views, fit block tables, the states of all slots) and, after it, the
// workspaces of admitted requests, handed out first-fit.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "cpd_runtime.hpp"

using namespace cpdmi;

namespace {

constexpr int kMaxSlots = 4096;
constexpr int kClasses = 4;  // rank-tile classes RT = 1..4

size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size).
class Arena {
 public:
  void init(size_t off, size_t len) {
    free_.clear();
    if (len) free_[off] = len;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Waiting {
  uint64_t ticket;
  cpd_request req;
  double t_submit;
};

struct Slot {
  bool used = false;
  uint64_t ticket = 0;
  cpd_request req{};
  size_t off = 0, bytes = 0;
  WsPlan plan{};
  ChainDesc desc{};  // state points into the server's state array
  double t_submit = 0, t_admit0 = 0, t_admit1 = 0;
};

// An admitted request waiting to be installed at the next round boundary.
struct Admitted {
  Waiting w;
  size_t off, bytes;
  WsPlan plan;
  ChainDesc desc;  // as written to its own workspace by the admission
  double t_admit0, t_admit1;
};

}  // namespace

struct cpd_server {
  cpd_server_config cfg{};
  int device = 0;
  double wall_hz = 1e8;
  char* arena = nullptr;
  size_t arena_bytes = 0, heap_off = 0;
  hipStream_t step = nullptr, admit = nullptr;
  hipStream_t side = nullptr;  // rank-tile classes after the first, concurrent with it
  hipEvent_t fork = nullptr, join = nullptr;
  // device header
  ChainDesc* d_class[kClasses] = {};  // per rank-tile class, one entry per slot
  ChainDesc* d_fit[2] = {};           // per storage type, one entry per slot
  int32_t* d_fitmap[2] = {};
  ChainState* d_states = nullptr;
  // host mirrors
  std::vector<ChainDesc> h_class[kClasses], h_fit[2];
  FitPlan fit[2]{};
  size_t class_lds[kClasses] = {};
  int class_count[kClasses] = {}, fit_count[2] = {};
  bool dirty = true;
  std::vector<Slot> slots;
  std::vector<ChainState> states;
  // shared between the threads (under mu)
  Arena heap;
  std::vector<Admitted> admitted;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Waiting> queue;
  std::unordered_map<uint64_t, cpd_result> results;
  std::unordered_set<uint64_t> live;
  uint64_t next_ticket = 1;
  int running = 0;     // admitted or being admitted, not yet finished
  int reserved = 0;    // slots in use or promised to an admission
  cpd_status fatal = CPD_OK;
  std::string fatal_msg;
  std::atomic<bool> stop{false};
  std::thread loop, admitter;
};

namespace {

struct HeaderLayout {
  size_t cls[kClasses], fit[2], fitmap[2], states, total;
};

HeaderLayout header_layout(int slots) {
  HeaderLayout h;
  size_t off = 0;
  for (int c = 0; c < kClasses; ++c) {
    h.cls[c] = off;
    off = align_up(off + sizeof(ChainDesc) * slots);
  }
  for (int d = 0; d < 2; ++d) {
    h.fit[d] = off;
    off = align_up(off + sizeof(ChainDesc) * slots);
    h.fitmap[d] = off;
    off = align_up(off + sizeof(int32_t) * fit_table_len(slots));
  }
  h.states = off;
  off = align_up(off + sizeof(ChainState) * slots);
  h.total = off;
  return h;
}

// Admission of one request into its arena region, on the admission stream:
// the same initialisation as cpd_init.  Returns the request's status.
cpd_status admit_one(cpd_server* s, const Waiting& w, size_t off, const WsPlan& plan,
                     ChainDesc* desc) {
  const cpd_problem* p = &w.req.problem;
  const cpd_options* o = &w.req.options;
  char* base = s->arena + off;
  fill_desc(p, o, plan, base, desc);
  ChainDesc* d_desc = (ChainDesc*)(base + plan.desc);
  cpd_status st = init_member(p, o, w.req.X, w.req.x_dtype, w.req.x_space, w.req.A0, plan, base,
                              s->admit, desc, d_desc);
  if (st != CPD_OK) return st;
  int32_t fitmap[6];
  const FitPlan fp = plan_fit(desc, 1, fitmap);
  int32_t* d_fm = (int32_t*)(base + plan.fitmap);
  hipError_t e = hipMemcpyAsync(d_fm, fitmap, sizeof fitmap, hipMemcpyHostToDevice, s->admit);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(fit table)");
  StepArgs a{};
  a.op = OP_REFRESH;
  e = launch_chain_kernel(d_desc, 1, desc->RT, plan.lds, a, s->admit);
  if (e != hipSuccess) return hip_fail(e, "refresh kernel");
  e = launch_fit(d_desc, d_fm, 1, fp, o->storage, false, s->admit);
  if (e != hipSuccess) return hip_fail(e, "norm kernels");
  ChainState stt;
  e = hipMemcpyAsync(&stt, base + plan.state, sizeof stt, hipMemcpyDeviceToHost, s->admit);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state)");
  e = hipStreamSynchronize(s->admit);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (stt.status != 0) describe_status(stt.status);
  return stt.status;
}

// The admission thread: waiting requests in order, each as soon as a slot
// and its arena space are free.
void admission_loop(cpd_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) return;
  while (!s->stop.load()) {
    Waiting w;
    WsPlan plan;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto ready = [&] {
        if (s->stop.load()) return true;
        if (s->queue.empty() || s->reserved >= s->cfg.max_slots) return false;
        std::string why;
        plan_workspace(&s->queue.front().req.problem, &s->queue.front().req.options, &plan, &why);
        return s->heap.alloc(plan.total, &off);
      };
      while (!ready()) s->cv.wait_for(lk, std::chrono::milliseconds(20));
      if (s->stop.load()) return;
      w = s->queue.front();
      s->queue.pop_front();
      s->reserved++;
      s->running++;
    }
    Admitted a;
    a.w = w;
    a.off = off;
    a.bytes = plan.total;
    a.plan = plan;
    a.t_admit0 = now_s();
    const cpd_status st = admit_one(s, w, off, plan, &a.desc);
    a.t_admit1 = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    if (st != CPD_OK) {
      (void)hipStreamSynchronize(s->admit);
      cpd_result r{};
      r.status = st;
      r.seconds_queued = a.t_admit0 - w.t_submit;
      r.seconds_admit = a.t_admit1 - a.t_admit0;
      r.seconds_total = a.t_admit1 - w.t_submit;
      s->heap.release(off, plan.total);
      s->reserved--;
      s->running--;
      s->results[w.ticket] = r;
      s->live.erase(w.ticket);
      continue;
    }
    s->admitted.push_back(a);
    s->cv.notify_all();
  }
}

// Rebuild the class and fit views from the slots.
void rebuild_views(cpd_server* s) {
  const int n = s->cfg.max_slots;
  for (int c = 0; c < kClasses; ++c) {
    std::fill(s->h_class[c].begin(), s->h_class[c].end(), ChainDesc{});
    s->class_lds[c] = 0;
    s->class_count[c] = 0;
  }
  for (int d = 0; d < 2; ++d) {
    std::fill(s->h_fit[d].begin(), s->h_fit[d].end(), ChainDesc{});
    s->fit_count[d] = 0;
  }
  for (int i = 0; i < n; ++i) {
    const Slot& sl = s->slots[i];
    if (!sl.used) continue;
    const int c = std::min(sl.desc.RT, kClasses) - 1;
    s->h_class[c][i] = sl.desc;
    s->class_lds[c] = std::max(s->class_lds[c], sl.plan.lds);
    s->class_count[c]++;
    const int d = sl.desc.dtype == CPD_BF16 ? 1 : 0;
    s->h_fit[d][i] = sl.desc;
    s->fit_count[d]++;
  }
}

hipError_t upload_views(cpd_server* s) {
  const int n = s->cfg.max_slots;
  hipError_t e = hipSuccess;
  for (int c = 0; c < kClasses && e == hipSuccess; ++c)
    e = hipMemcpyAsync(s->d_class[c], s->h_class[c].data(), sizeof(ChainDesc) * n,
                       hipMemcpyHostToDevice, s->step);
  for (int d = 0; d < 2 && e == hipSuccess; ++d) {
    e = hipMemcpyAsync(s->d_fit[d], s->h_fit[d].data(), sizeof(ChainDesc) * n,
                       hipMemcpyHostToDevice, s->step);
    if (e != hipSuccess) break;
    std::vector<int32_t> fm(fit_table_len(n));
    s->fit[d] = plan_fit(s->h_fit[d].data(), n, fm.data());
    e = hipMemcpyAsync(s->d_fitmap[d], fm.data(), sizeof(int32_t) * fm.size(),
                       hipMemcpyHostToDevice, s->step);
    if (e == hipSuccess) e = hipStreamSynchronize(s->step);  // fm is released below
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->step);
  return e;
}

hipError_t launch_round(cpd_server* s) {
  StepArgs a{};
  a.op = OP_STEP;
  a.nsteps = s->cfg.round_steps;
  // the first populated class steps on the step stream, the others one
  // after the other on the side stream, forked from and joined back into
  // the step stream (classes are independent of each other)
  int populated = 0;
  for (int c = 0; c < kClasses; ++c) populated += s->class_count[c] ? 1 : 0;
  hipError_t e = hipSuccess;
  if (populated > 1) {
    e = hipEventRecord(s->fork, s->step);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->side, s->fork, 0);
    if (e != hipSuccess) return e;
  }
  for (int c = 0, q = 0; c < kClasses; ++c) {
    if (!s->class_count[c]) continue;
    e = launch_chain_kernel(s->d_class[c], s->cfg.max_slots, c + 1, s->class_lds[c], a,
                            q++ == 0 ? s->step : s->side);
    if (e != hipSuccess) return e;
  }
  if (populated > 1) {
    e = hipEventRecord(s->join, s->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->step, s->join, 0);
    if (e != hipSuccess) return e;
  }
  for (int d = 0; d < 2; ++d) {
    if (!s->fit_count[d]) continue;
    hipError_t e = launch_fit(s->d_fit[d], s->d_fitmap[d], s->cfg.max_slots, s->fit[d],
                              d ? CPD_BF16 : CPD_F32, true, s->step);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// After a round: hand out the results of the requests that stopped.
hipError_t collect(cpd_server* s) {
  const int n = s->cfg.max_slots;
  hipError_t e = hipMemcpyAsync(s->states.data(), s->d_states, sizeof(ChainState) * n,
                                hipMemcpyDeviceToHost, s->step);
  if (e == hipSuccess) e = hipStreamSynchronize(s->step);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    Slot& sl = s->slots[i];
    if (!sl.used) continue;
    const ChainState& st = s->states[i];
    if (!st.done && st.status == 0) continue;
    cpd_result r{};
    r.status = st.status;
    r.fit = st.fit;
    r.steps = st.t;
    r.reached = sl.req.options.fit_target > 0 && st.fit >= sl.req.options.fit_target;
    r.seconds_queued = sl.t_admit0 - sl.t_submit;
    r.seconds_admit = sl.t_admit1 - sl.t_admit0;
    r.seconds_to_fit =
        st.clock_done >= st.clock_start ? (st.clock_done - st.clock_start) / s->wall_hz : 0.0;
    for (int k = 0; k < sl.desc.N && e == hipSuccess; ++k)
      if (sl.req.out[k])
        e = hipMemcpyAsync(sl.req.out[k], sl.desc.A[k],
                           sizeof(float) * (size_t)sl.desc.dims[k] * sl.desc.R,
                           hipMemcpyDeviceToHost, s->step);
    if (e == hipSuccess) e = hipStreamSynchronize(s->step);
    if (e != hipSuccess) return e;
    r.seconds_total = now_s() - sl.t_submit;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->heap.release(sl.off, sl.bytes);
      s->results[sl.ticket] = r;
      s->live.erase(sl.ticket);
      s->running--;
      s->reserved--;
      s->cv.notify_all();
    }
    sl = Slot{};
    s->dirty = true;
  }
  return hipSuccess;
}

// Put the admitted requests into free slots; their states move into the
// server's state array (the step and fit kernels of the running set read
// them there).
hipError_t install(cpd_server* s) {
  std::vector<Admitted> batch;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    batch.swap(s->admitted);
  }
  for (const Admitted& a : batch) {
    int i = 0;
    while (s->slots[i].used) ++i;  // a free slot exists (admission counted them)
    Slot& sl = s->slots[i];
    sl.used = true;
    sl.ticket = a.w.ticket;
    sl.req = a.w.req;
    sl.off = a.off;
    sl.bytes = a.bytes;
    sl.plan = a.plan;
    sl.desc = a.desc;
    sl.t_submit = a.w.t_submit;
    sl.t_admit0 = a.t_admit0;
    sl.t_admit1 = a.t_admit1;
    ChainState* own = (ChainState*)(s->arena + a.off + a.plan.state);
    hipError_t e = hipMemcpyAsync(s->d_states + i, own, sizeof(ChainState),
                                  hipMemcpyDeviceToDevice, s->step);
    if (e != hipSuccess) return e;
    sl.desc.state = s->d_states + i;
    sl.desc.autostop = 1;
    sl.desc.step_limit = a.w.req.options.max_steps > 0 ? a.w.req.options.max_steps : 0;
    sl.desc.fit_target = a.w.req.options.fit_target;
    s->dirty = true;
  }
  return hipSuccess;
}

void fail_all(cpd_server* s, hipError_t e, const char* what) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->fatal = CPD_E_HIP;
  s->fatal_msg = std::string(what) + ": " + hipGetErrorString(e);
  for (uint64_t t : s->live) {
    cpd_result r{};
    r.status = CPD_E_HIP;
    s->results[t] = r;
  }
  s->live.clear();
  s->queue.clear();
  s->cv.notify_all();
}

void server_loop(cpd_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) return;
  while (!s->stop.load()) {
    hipError_t e = install(s);
    if (e != hipSuccess) return fail_all(s, e, "install");
    if (s->dirty) {
      rebuild_views(s);
      e = upload_views(s);
      if (e != hipSuccess) return fail_all(s, e, "descriptor upload");
      s->dirty = false;
    }
    int nrun = 0;
    for (int c = 0; c < kClasses; ++c) nrun += s->class_count[c];
    if (!nrun) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::milliseconds(50),
                     [&] { return s->stop.load() || !s->admitted.empty(); });
      continue;
    }
    e = launch_round(s);
    if (e != hipSuccess) return fail_all(s, e, "round launch");
    e = collect(s);
    if (e != hipSuccess) return fail_all(s, e, "collect");
  }
}

}  // namespace

extern "C" {

cpd_status cpd_server_create(const cpd_server_config* cfg, void* arena, size_t arena_bytes,
                             cpd_server** out) {
  try {
    if (!cfg || !arena || !out) {
      set_error("null argument");
      return CPD_E_INVALID;
    }
    *out = nullptr;
    if (cfg->max_slots < 1 || cfg->max_slots > kMaxSlots || cfg->round_steps < 1 ||
        cfg->queue_capacity < 1) {
      set_error("max_slots must be in [1, 4096], round_steps and queue_capacity >= 1");
      return CPD_E_INVALID;
    }
    if (((uintptr_t)arena) % kAlign) {
      set_error("arena must be 256-byte aligned");
      return CPD_E_INVALID;
    }
    const HeaderLayout H = header_layout(cfg->max_slots);
    if (arena_bytes <= H.total) {
      set_error("arena too small for the server header (" + std::to_string(H.total) + " bytes)");
      return CPD_E_OOM;
    }
    cpd_server* s = new (std::nothrow) cpd_server();
    if (!s) {
      set_error("out of host memory");
      return CPD_E_OOM;
    }
    s->cfg = *cfg;
    s->arena = (char*)arena;
    s->arena_bytes = arena_bytes;
    s->heap_off = H.total;
    auto fail = [&](hipError_t e, const char* what) {
      cpd_status r = hip_fail(e, what);
      if (s->step) (void)hipStreamDestroy(s->step);
      if (s->admit) (void)hipStreamDestroy(s->admit);
      if (s->side) (void)hipStreamDestroy(s->side);
      if (s->fork) (void)hipEventDestroy(s->fork);
      if (s->join) (void)hipEventDestroy(s->join);
      delete s;
      return r;
    };
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) return fail(e, "hipGetDevice");
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) == hipSuccess &&
        khz > 0)
      s->wall_hz = 1e3 * khz;
    e = hipStreamCreateWithFlags(&s->step, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(e, "hipStreamCreate");
    e = hipStreamCreateWithFlags(&s->admit, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(e, "hipStreamCreate");
    e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(e, "hipStreamCreate");
    e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->join, hipEventDisableTiming);
    if (e != hipSuccess) return fail(e, "hipEventCreate");
    for (int c = 0; c < kClasses; ++c) {
      s->d_class[c] = (ChainDesc*)(s->arena + H.cls[c]);
      s->h_class[c].assign(cfg->max_slots, ChainDesc{});
    }
    for (int d = 0; d < 2; ++d) {
      s->d_fit[d] = (ChainDesc*)(s->arena + H.fit[d]);
      s->d_fitmap[d] = (int32_t*)(s->arena + H.fitmap[d]);
      s->h_fit[d].assign(cfg->max_slots, ChainDesc{});
    }
    s->d_states = (ChainState*)(s->arena + H.states);
    s->states.assign(cfg->max_slots, ChainState{});
    s->slots.assign(cfg->max_slots, Slot{});
    // offsets are relative to the arena start; the header comes first
    s->heap.init(H.total, (arena_bytes - H.total) / kAlign * kAlign);
    e = hipMemsetAsync(s->arena, 0, H.total, s->step);
    if (e == hipSuccess) e = hipStreamSynchronize(s->step);
    if (e != hipSuccess) return fail(e, "hipMemsetAsync(header)");
    s->loop = std::thread(server_loop, s);
    s->admitter = std::thread(admission_loop, s);
    *out = s;
    return CPD_OK;
  } catch (...) {
    set_error("unexpected exception in cpd_server_create");
    return CPD_E_INVALID;
  }
}

cpd_status cpd_submit(cpd_server* s, const cpd_request* r, uint64_t* ticket) {
  try {
    if (!s || !r || !ticket || !r->X) {
      set_error("null argument");
      return CPD_E_INVALID;
    }
    WsPlan plan;
    std::string why;
    cpd_status st = plan_workspace(&r->problem, &r->options, &plan, &why);
    if (st == CPD_OK && plan.grid) {
      why = "served requests use the persistent step (B <= " +
            std::to_string(CPD_MAX_PERSISTENT_BATCH) + ", LDS within 160 KiB)";
      st = CPD_E_INVALID;
    }
    if (st == CPD_OK && r->options.rescale_every != 0) {
      why = "rescale_every applies to single handles only (must be 0 for a served request)";
      st = CPD_E_INVALID;
    }
    if (st != CPD_OK) {
      set_error(why);
      return st;
    }
    st = check_input_kinds(r->x_dtype, r->x_space);
    if (st != CPD_OK) return st;
    if (r->options.max_steps < 1) {
      set_error("a served request needs options.max_steps >= 1");
      return CPD_E_INVALID;
    }
    for (int k = 0; k < r->problem.N; ++k)
      if (!r->A0[k]) {
        set_error("null initial factor");
        return CPD_E_INVALID;
      }
    if (align_up(plan.total) > s->arena_bytes - s->heap_off) {
      set_error("request needs " + std::to_string(plan.total) +
                " bytes of workspace, more than the arena holds");
      return CPD_E_OOM;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != CPD_OK) {
      set_error(s->fatal_msg);
      return s->fatal;
    }
    if ((int)s->queue.size() >= s->cfg.queue_capacity) {
      set_error("the request queue is full");
      return CPD_E_QUEUE_FULL;
    }
    const uint64_t t = s->next_ticket++;
    s->queue.push_back(Waiting{t, *r, now_s()});
    s->live.insert(t);
    *ticket = t;
    s->cv.notify_all();  // both server threads wait on this variable
    return CPD_OK;
  } catch (...) {
    set_error("unexpected exception in cpd_submit");
    return CPD_E_INVALID;
  }
}

cpd_status cpd_poll(cpd_server* s, uint64_t ticket, cpd_result* out) {
  if (!s || !out) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it != s->results.end()) {
    *out = it->second;
    s->results.erase(it);
    return CPD_OK;
  }
  if (s->live.count(ticket)) return CPD_PENDING;
  set_error("unknown ticket");
  return CPD_E_NOT_FOUND;
}

cpd_status cpd_server_stats(cpd_server* s, int32_t* waiting, int32_t* running, int32_t* finished) {
  if (!s) {
    set_error("null server");
    return CPD_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (waiting) *waiting = (int32_t)s->queue.size();
  if (running) *running = s->running;
  if (finished) *finished = (int32_t)s->results.size();
  return CPD_OK;
}

cpd_status cpd_server_destroy(cpd_server* s) {
  if (!s) return CPD_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop.store(true);
  }
  s->cv.notify_all();
  if (s->loop.joinable()) s->loop.join();
  if (s->admitter.joinable()) s->admitter.join();
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->step);
  (void)hipStreamSynchronize(s->side);
  (void)hipStreamSynchronize(s->admit);
  (void)hipStreamDestroy(s->step);
  (void)hipStreamDestroy(s->side);
  (void)hipStreamDestroy(s->admit);
  (void)hipEventDestroy(s->fork);
  (void)hipEventDestroy(s->join);
  delete s;
  return CPD_OK;
}

}  // extern "C"
