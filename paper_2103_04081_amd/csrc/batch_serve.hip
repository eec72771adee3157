// C ABI of libcpdmi: batched decompositions (cpd_batch_*).
//
// Members are ordered by rank-tile class (RT = ceil(R / 16)); each class is
// one launch of the persistent step kernel with one workgroup per member,
// and the classes run concurrently on two streams.  A round (fit_every
// steps of every member of a class, then the fit check of that class, on
// the class's stream) is captured once in a HIP graph and replayed: the
// fit of a class that finishes its steps early streams its tensors while
// the other class still steps.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "cpd_runtime.hpp"

using namespace cpdmi;

namespace {

size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

// Tuned K-split per (mode size, rank, B, storage), shared by every batch of
// the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tuned;

struct Group {
  int rt, first, count;
  size_t lds;
  FitPlan fit{{0, 0}, {0, 0}, 1};  // the class's own fit launches
  int32_t* d_fitmap = nullptr;     // their block tables (descriptors first .. first+count)
};

}  // namespace

struct cpd_batch {
  int count = 0;
  int device = 0;
  hipStream_t stream = nullptr;  // caller's
  hipStream_t side = nullptr;    // rank-tile classes after the first
  hipStream_t cap = nullptr;     // graph capture (the caller's may be the null stream)
  hipEvent_t fork = nullptr, join = nullptr;
  char* ws = nullptr;
  std::vector<cpd_problem> ps;
  std::vector<cpd_options> os;
  std::vector<WsPlan> plans;
  std::vector<size_t> base;  // member workspace offset, by member index
  std::vector<int> pos;      // member index -> descriptor position
  std::vector<ChainDesc> descs;  // host mirror, by position
  ChainDesc* d_descs = nullptr;
  ChainState* d_states = nullptr;
  int32_t* d_fitmap = nullptr;  // fit block tables, by position
  FitPlan fit{{0, 0}, {0, 0}};
  std::vector<Group> groups;
  int dtype = CPD_F32, fit_every = 25;
  double wall_hz = 1e8;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<ChainState> states;  // host copy, by position
};

namespace {

struct BatchLayout {
  size_t descs, states, fitmap, total;
  std::vector<size_t> base;
};

cpd_status plan_batch(const cpd_problem* ps, const cpd_options* os, int count,
                      std::vector<WsPlan>* plans, BatchLayout* L) {
  if (!ps || !os || count < 1) {
    set_error("need at least one member");
    return CPD_E_INVALID;
  }
  plans->resize(count);
  size_t off = 0;
  L->descs = off;
  off = align_up(off + sizeof(ChainDesc) * count);
  L->states = off;
  off = align_up(off + sizeof(ChainState) * count);
  L->fitmap = off;
  // all members' tables, then one set per rank-tile class (at most
  // kMaxRankTiles classes, each at most count members)
  off = align_up(off + sizeof(int32_t) * (fit_table_len(count) + fit_table_len(count) +
                                          3 * (kMaxRankTiles - 1)));
  L->base.resize(count);
  for (int i = 0; i < count; ++i) {
    std::string why;
    cpd_status s = plan_workspace(&ps[i], &os[i], &(*plans)[i], &why);
    if (s == CPD_OK && (*plans)[i].grid) {
      why = "batched members use the persistent step (B <= " +
            std::to_string(CPD_MAX_PERSISTENT_BATCH) + ", LDS within 160 KiB)";
      s = CPD_E_INVALID;
    }
    if (s == CPD_OK && os[i].rescale_every != 0) {
      why = "rescale_every applies to single handles only (must be 0 in a batch)";
      s = CPD_E_INVALID;
    }
    if (s != CPD_OK) {
      set_error("member " + std::to_string(i) + ": " + why);
      return s;
    }
    if (os[i].fit_every != os[0].fit_every || os[i].fit_every < 1) {
      set_error("members must share fit_every >= 1");
      return CPD_E_INVALID;
    }
    if (os[i].storage != os[0].storage) {
      set_error("members must share the storage type");
      return CPD_E_INVALID;
    }
    L->base[i] = off;
    off = align_up(off + (*plans)[i].total);
  }
  L->total = off;
  return CPD_OK;
}

hipError_t launch_groups(cpd_batch* b, const StepArgs& a, hipStream_t main) {
  // the first class runs on the caller's stream, the others one after the
  // other on the side stream, forked from and joined back into the caller's
  // stream (classes are independent of each other)
  if (b->groups.size() == 1) {
    const Group& g = b->groups[0];
    return launch_chain_kernel(b->d_descs + g.first, g.count, g.rt, g.lds, a, main);
  }
  hipError_t e = hipEventRecord(b->fork, main);
  if (e != hipSuccess) return e;
  e = hipStreamWaitEvent(b->side, b->fork, 0);
  if (e != hipSuccess) return e;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const Group& g = b->groups[gi];
    e = launch_chain_kernel(b->d_descs + g.first, g.count, g.rt, g.lds, a,
                            gi == 0 ? main : b->side);
    if (e != hipSuccess) return e;
  }
  e = hipEventRecord(b->join, b->side);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(main, b->join, 0);
}

cpd_status read_states(cpd_batch* b) {
  hipError_t e = hipMemcpyAsync(b->states.data(), b->d_states, sizeof(ChainState) * b->count,
                                hipMemcpyDeviceToHost, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(states)");
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return CPD_OK;
}

cpd_status first_error(cpd_batch* b) {
  for (int i = 0; i < b->count; ++i) {
    const cpd_status s = b->states[b->pos[i]].status;
    if (s != 0) {
      describe_status(s);
      set_error("member " + std::to_string(i) + ": " + cpd_last_error());
      return s;
    }
  }
  return CPD_OK;
}

hipError_t upload_descs(cpd_batch* b) {
  return hipMemcpyAsync(b->d_descs, b->descs.data(), sizeof(ChainDesc) * b->count,
                        hipMemcpyHostToDevice, b->stream);
}

// Bring every member back to its initial factors: A = A0, S = 0, state
// cleared (t = 0), distributions rebuilt.
cpd_status restart_members(cpd_batch* b, const float* const* A0) {
  hipError_t e = hipMemsetAsync(b->d_states, 0, sizeof(ChainState) * b->count, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(states)");
  for (int i = 0; i < b->count; ++i) {
    const ChainDesc& d = b->descs[b->pos[i]];
    for (int k = 0; k < d.N; ++k) {
      const size_t fb = sizeof(float) * (size_t)d.dims[k] * d.R;
      e = hipMemcpyAsync(d.A[k], A0[(size_t)i * CPD_MAX_MODES + k], fb, hipMemcpyHostToDevice,
                         b->stream);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(A0)");
      e = hipMemsetAsync(d.S[k], 0, fb, b->stream);
      if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(S)");
    }
  }
  StepArgs a{};
  a.op = OP_REFRESH;
  e = launch_groups(b, a, b->stream);
  if (e != hipSuccess) return hip_fail(e, "refresh kernel");
  return CPD_OK;
}

// Time every candidate K-split of every mode on the members themselves
// (steps with that mode forced), keep the fastest per member and mode.
cpd_status tune(cpd_batch* b) {
  constexpr int kTuneSteps = 24;
  const int cands[] = {1, 2, 4, 8};
  int maxN = 0;
  for (int i = 0; i < b->count; ++i) maxN = std::max(maxN, b->ps[i].N);
  auto key = [&](int i, int k) {
    return std::make_tuple(b->ps[i].dims[k], b->ps[i].R, b->ps[i].B, b->os[i].storage);
  };
  std::vector<int> cached(b->count * CPD_MAX_MODES, 0);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < b->count; ++i)
      for (int k = 0; k < b->ps[i].N; ++k) {
        auto it = g_tuned.find(key(i, k));
        if (it != g_tuned.end()) cached[i * CPD_MAX_MODES + k] = it->second;
      }
  }
  // warm-up launch (instruction caches, first-touch of the copies)
  StepArgs a{};
  a.op = OP_STEP;
  a.nsteps = 4;
  hipError_t e = launch_groups(b, a, b->stream);
  if (e != hipSuccess) return hip_fail(e, "tuning kernel");
  for (int m = 0; m < maxN; ++m) {
    std::vector<std::vector<int>> opts(b->count);
    int rounds = 0;
    for (int i = 0; i < b->count; ++i) {
      if (m >= b->ps[i].N || b->os[i].ksplit[m] > 0 || cached[i * CPD_MAX_MODES + m] > 0) continue;
      const int mx = max_ksplit(b->ps[i].dims[m], b->os[i].storage, b->ps[i].B, b->ps[i].R);
      for (int c : cands)
        if (c <= mx) opts[i].push_back(c);
      if (opts[i].size() > 1) rounds = std::max(rounds, (int)opts[i].size());
    }
    if (rounds == 0) continue;
    std::vector<int64_t> best_ticks(b->count, INT64_MAX);
    std::vector<int> best(b->count, 0);
    for (int r = 0; r < rounds; ++r) {
      for (int i = 0; i < b->count; ++i)
        if (opts[i].size() > 1)
          b->descs[b->pos[i]].ksplit[m] = opts[i][std::min<size_t>(r, opts[i].size() - 1)];
      e = upload_descs(b);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(descs)");
      a.nsteps = kTuneSteps;
      a.force_mode1 = m + 1;
      e = launch_groups(b, a, b->stream);
      if (e != hipSuccess) return hip_fail(e, "tuning kernel");
      cpd_status s = read_states(b);
      if (s != CPD_OK) return s;
      for (int i = 0; i < b->count; ++i) {
        if (opts[i].size() <= 1 || r >= (int)opts[i].size()) continue;
        const int64_t tk = b->states[b->pos[i]].ticks;
        if (tk < best_ticks[i]) {
          best_ticks[i] = tk;
          best[i] = opts[i][r];
        }
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < b->count; ++i) {
      if (opts[i].size() <= 1) continue;
      b->descs[b->pos[i]].ksplit[m] = best[i];
      g_tuned[key(i, m)] = best[i];
    }
  }
  for (int i = 0; i < b->count; ++i)
    for (int k = 0; k < b->ps[i].N; ++k)
      if (cached[i * CPD_MAX_MODES + k] > 0) b->descs[b->pos[i]].ksplit[k] = cached[i * CPD_MAX_MODES + k];
  e = upload_descs(b);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(descs)");
  return CPD_OK;
}

void destroy_batch(cpd_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

hipError_t launch_fit_all(cpd_batch* b, hipStream_t stream) {
  return launch_fit(b->d_descs, b->d_fitmap, b->count, b->fit, b->dtype, true, stream);
}

// One round: every class steps fit_every steps and then checks the fit of
// its own members, on the class's stream (the first class on main, the
// others on the side stream, forked from and joined back into main).
hipError_t launch_round(cpd_batch* b, hipStream_t main) {
  StepArgs a{};
  a.op = OP_STEP;
  a.nsteps = b->fit_every;
  const bool fork = b->groups.size() > 1;
  hipError_t e = hipSuccess;
  if (fork) {
    e = hipEventRecord(b->fork, main);
    if (e != hipSuccess) return e;
    e = hipStreamWaitEvent(b->side, b->fork, 0);
    if (e != hipSuccess) return e;
  }
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const Group& g = b->groups[gi];
    hipStream_t s = gi == 0 ? main : b->side;
    e = launch_chain_kernel(b->d_descs + g.first, g.count, g.rt, g.lds, a, s);
    if (e != hipSuccess) return e;
    e = launch_fit(b->d_descs + g.first, g.d_fitmap, g.count, g.fit, b->dtype, true, s);
    if (e != hipSuccess) return e;
  }
  if (!fork) return hipSuccess;
  e = hipEventRecord(b->join, b->side);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(main, b->join, 0);
}

cpd_status build_graph(cpd_batch* b) {
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t e1 = launch_round(b, b->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (e1 != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e1 != hipSuccess ? e1 : e, "graph capture");
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graph = g;
  b->exec = x;
  return CPD_OK;
}

}  // namespace

extern "C" {

cpd_status cpd_batch_workspace_size(const cpd_problem* ps, const cpd_options* os, int32_t count,
                                    size_t* bytes) {
  try {
    if (!bytes) {
      set_error("bytes is null");
      return CPD_E_INVALID;
    }
    std::vector<WsPlan> plans;
    BatchLayout L;
    cpd_status s = plan_batch(ps, os, count, &plans, &L);
    if (s != CPD_OK) return s;
    *bytes = L.total;
    return CPD_OK;
  } catch (...) {
    set_error("unexpected exception");
    return CPD_E_INVALID;
  }
}

cpd_status cpd_batch_create(const cpd_problem* ps, const cpd_options* os, int32_t count,
                            const void* const* X, int32_t x_dtype, int32_t x_space,
                            const float* const* A0, void* ws, size_t ws_bytes, void* stream,
                            int32_t tune_flag, cpd_batch** out) {
  try {
    if (!out || !X || !A0 || !ws) {
      set_error("null argument");
      return CPD_E_INVALID;
    }
    *out = nullptr;
    std::vector<WsPlan> plans;
    BatchLayout L;
    cpd_status s = plan_batch(ps, os, count, &plans, &L);
    if (s != CPD_OK) return s;
    s = check_input_kinds(x_dtype, x_space);
    if (s != CPD_OK) return s;
    if (((uintptr_t)ws) % kAlign) {
      set_error("workspace must be 256-byte aligned");
      return CPD_E_INVALID;
    }
    if (ws_bytes < L.total) {
      set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
      return CPD_E_OOM;
    }
    for (int i = 0; i < count; ++i) {
      if (!X[i]) {
        set_error("member " + std::to_string(i) + ": null tensor");
        return CPD_E_INVALID;
      }
      for (int k = 0; k < ps[i].N; ++k)
        if (!A0[(size_t)i * CPD_MAX_MODES + k]) {
          set_error("member " + std::to_string(i) + ": null initial factor");
          return CPD_E_INVALID;
        }
    }
    cpd_batch* b = new (std::nothrow) cpd_batch();
    if (!b) {
      set_error("out of host memory");
      return CPD_E_OOM;
    }
    auto fail = [&](cpd_status r) {
      (void)hipStreamSynchronize(b->stream);
      destroy_batch(b);
      return r;
    };
    b->count = count;
    b->stream = (hipStream_t)stream;
    b->ws = (char*)ws;
    b->ps.assign(ps, ps + count);
    b->os.assign(os, os + count);
    b->plans = plans;
    b->base = L.base;
    b->dtype = os[0].storage;
    b->fit_every = os[0].fit_every;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return fail(hip_fail(e, "hipGetDevice"));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) == hipSuccess &&
        khz > 0)
      b->wall_hz = 1e3 * khz;
    e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
    e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e != hipSuccess) return fail(hip_fail(e, "hipEventCreate"));
    e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
    if (e != hipSuccess) return fail(hip_fail(e, "hipEventCreate"));

    // order members by rank-tile class
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return (ps[x].R + 15) / 16 < (ps[y].R + 15) / 16;
    });
    b->pos.assign(count, 0);
    for (int q = 0; q < count; ++q) b->pos[order[q]] = q;
    b->d_descs = (ChainDesc*)(b->ws + L.descs);
    b->d_states = (ChainState*)(b->ws + L.states);
    b->descs.resize(count);
    b->states.resize(count);
    for (int q = 0; q < count; ++q) {
      const int i = order[q];
      const int rt = (ps[i].R + 15) / 16;
      if (b->groups.empty() || b->groups.back().rt != rt) b->groups.push_back(Group{rt, q, 0, 0});
      Group& g = b->groups.back();
      g.count++;
      g.lds = std::max(g.lds, plans[i].lds);
    }
    if (b->groups.size() > (size_t)kMaxRankTiles) {
      set_error("more rank-tile classes than the persistent step has");
      return fail(CPD_E_INVALID);
    }
    e = hipMemsetAsync(b->ws, 0, L.states + sizeof(ChainState) * count, b->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemsetAsync"));
    for (int i = 0; i < count; ++i) {
      const int q = b->pos[i];
      ChainDesc& d = b->descs[q];
      char* mb = b->ws + L.base[i];
      fill_desc(&ps[i], &os[i], plans[i], mb, &d);
      d.state = b->d_states + q;
      d.autostop = 1;
      d.step_limit = os[i].max_steps > 0 ? os[i].max_steps : 0;
      d.fit_target = os[i].fit_target;
      s = init_member(&ps[i], &os[i], X[i], x_dtype, x_space, A0 + (size_t)i * CPD_MAX_MODES,
                      plans[i], mb, b->stream, &d, b->d_descs + q);
      if (s != CPD_OK) {
        set_error("member " + std::to_string(i) + ": " + cpd_last_error());
        return fail(s);
      }
    }
    StepArgs a{};
    a.op = OP_REFRESH;
    e = launch_groups(b, a, b->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "refresh kernel"));
    if (tune_flag) {
      s = tune(b);
      if (s != CPD_OK) return fail(s);
      s = restart_members(b, A0);
      if (s != CPD_OK) return fail(s);
    }
    // all members' tables, then each class's own (the same block split of
    // each member, a function of its tensor alone, over the class's
    // descriptors); one copy
    size_t ntab = fit_table_len(count);
    for (const Group& g : b->groups) ntab += fit_table_len(g.count);
    std::vector<int32_t> fitmap(ntab);
    b->d_fitmap = (int32_t*)(b->ws + L.fitmap);
    b->fit = plan_fit(b->descs.data(), count, fitmap.data());
    size_t at = fit_table_len(count);
    for (Group& g : b->groups) {
      g.fit = plan_fit(b->descs.data() + g.first, g.count, fitmap.data() + at);
      g.d_fitmap = b->d_fitmap + at;
      at += fit_table_len(g.count);
    }
    e = hipMemcpyAsync(b->d_fitmap, fitmap.data(), sizeof(int32_t) * fitmap.size(),
                       hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpyAsync(fit tables)"));
    e = launch_fit(b->d_descs, b->d_fitmap, count, b->fit, b->dtype, false, b->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "norm kernels"));
    s = read_states(b);
    if (s != CPD_OK) return fail(s);
    s = first_error(b);
    if (s != CPD_OK) return fail(s);
    *out = b;
    return CPD_OK;
  } catch (...) {
    set_error("unexpected exception in cpd_batch_create");
    return CPD_E_INVALID;
  }
}

cpd_status cpd_batch_step(cpd_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int64_t chunk = (int64_t)1 << 20;
  for (int64_t done = 0; done < nsteps; done += chunk) {
    StepArgs a{};
    a.op = OP_STEP;
    a.nsteps = std::min(chunk, nsteps - done);
    e = launch_groups(b, a, b->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel");
  }
  return CPD_OK;
}

cpd_status cpd_batch_fits(cpd_batch* b, double* fits) {
  if (!b || !fits) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = launch_fit_all(b, b->stream);
  if (e != hipSuccess) return hip_fail(e, "fit kernels");
  cpd_status s = read_states(b);
  if (s != CPD_OK) return s;
  for (int i = 0; i < b->count; ++i) fits[i] = b->states[b->pos[i]].fit;
  return first_error(b);
}

cpd_status cpd_batch_run(cpd_batch* b, int64_t max_rounds, int32_t* remaining) {
  if (!b || max_rounds < 0) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (!b->exec) {
    cpd_status s = build_graph(b);
    if (s != CPD_OK) return s;
  }
  // rounds are replayed in groups; the host looks at the members between
  // groups (a member that is done costs its workgroup one early exit)
  constexpr int64_t kPollEvery = 4;
  int32_t left = b->count;
  for (int64_t r = 0; r < max_rounds && left > 0;) {
    const int64_t n = std::min(kPollEvery, max_rounds - r);
    for (int64_t q = 0; q < n; ++q) {
      e = hipGraphLaunch(b->exec, b->stream);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    r += n;
    cpd_status s = read_states(b);
    if (s != CPD_OK) return s;
    left = 0;
    for (int q = 0; q < b->count; ++q) left += b->states[q].done ? 0 : 1;
  }
  if (remaining) *remaining = left;
  return first_error(b);
}

cpd_status cpd_batch_sync(cpd_batch* b) {
  if (!b) {
    set_error("null batch");
    return CPD_E_INVALID;
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  cpd_status s = read_states(b);
  if (s != CPD_OK) return s;
  return first_error(b);
}

cpd_status cpd_batch_member_info(cpd_batch* b, int32_t i, cpd_member_info* out) {
  if (!b || !out || i < 0 || i >= b->count) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  cpd_status s = read_states(b);
  if (s != CPD_OK) return s;
  const ChainState& st = b->states[b->pos[i]];
  const ChainDesc& d = b->descs[b->pos[i]];
  std::memset(out, 0, sizeof(*out));
  out->t = st.t;
  out->fit = st.fit;
  out->done = st.done;
  out->status = st.status;
  out->t_done = st.t_done;
  out->seconds_done =
      st.done && st.clock_done >= st.clock_start ? (st.clock_done - st.clock_start) / b->wall_hz : 0.0;
  for (int k = 0; k < d.N; ++k) out->ksplit[k] = d.ksplit[k];
  return CPD_OK;
}

cpd_status cpd_batch_read_factors(cpd_batch* b, int32_t i, int32_t n, float* dst,
                                  int32_t dst_space) {
  if (!b || !dst || i < 0 || i >= b->count || n < 0 || n >= b->ps[i].N) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const ChainDesc& d = b->descs[b->pos[i]];
  const size_t bytes = sizeof(float) * (size_t)d.dims[n] * d.R;
  e = hipMemcpyAsync(dst, d.A[n], bytes,
                     dst_space == CPD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                     b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(factor)");
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return CPD_OK;
}

cpd_status cpd_batch_destroy(cpd_batch* b) {
  if (!b) return CPD_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  destroy_batch(b);
  return CPD_OK;
}

}  // extern "C"
