// C ABI of libcpdmi: single-decomposition handles.
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cpd_runtime.hpp"

namespace cpdmi {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

cpd_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return CPD_E_HIP;
}

static size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

cpd_status plan_workspace(const cpd_problem* p, const cpd_options* o, WsPlan* w, std::string* why) {
  if (!p || !o || !w) {
    *why = "null argument";
    return CPD_E_INVALID;
  }
  if (p->N < 2 || p->N > kMaxModes) {
    *why = "N must be in [2, " + std::to_string(kMaxModes) + "]";
    return CPD_E_INVALID;
  }
  if (p->R < 1 || p->R > kMaxRank) {
    *why = "R must be in [1, " + std::to_string(kMaxRank) + "]";
    return CPD_E_INVALID;
  }
  if (p->B < 1 || p->B > CPD_MAX_BATCH) {
    *why = "B must be in [1, " + std::to_string(CPD_MAX_BATCH) + "]";
    return CPD_E_INVALID;
  }
  if (o->sampler < 0 || o->sampler > 2 || o->rule < 0 || o->rule > 2) {
    *why = "unknown sampler or rule";
    return CPD_E_INVALID;
  }
  if (o->storage != CPD_F32 && o->storage != CPD_BF16) {
    *why = "storage must be CPD_F32 or CPD_BF16";
    return CPD_E_INVALID;
  }
  if (o->path < CPD_PATH_AUTO || o->path > CPD_PATH_GRID) {
    *why = "path must be CPD_PATH_AUTO, CPD_PATH_PERSISTENT or CPD_PATH_GRID";
    return CPD_E_INVALID;
  }
  if (o->rescale_every < 0) {
    *why = "rescale_every must be >= 0";
    return CPD_E_INVALID;
  }
  int64_t total = 1;
  for (int k = 0; k < p->N; ++k) {
    if (p->dims[k] < 1 || p->dims[k] > CPD_MAX_DIM) {
      *why = "dims must be in [1, " + std::to_string(CPD_MAX_DIM) + "]";
      return CPD_E_INVALID;
    }
    total *= p->dims[k];
    if (total > (int64_t)1 << 40) {
      *why = "tensor too large";
      return CPD_E_INVALID;
    }
  }
  const size_t es = o->storage == CPD_BF16 ? 2 : 4;
  for (int n = 0; n < p->N; ++n) {
    const size_t copy_bytes =
        es * (size_t)(total / p->dims[n]) * (size_t)round_up(p->dims[n], kLdAlign);
    if (copy_bytes > ((size_t)1 << 32) - 256) {
      *why = "each mode-major copy of the tensor must stay below 4 GiB";
      return CPD_E_INVALID;
    }
  }
  // the persistent step when it fits (or is asked for), else the grid step;
  // ranks beyond 64 run on the grid step only, with the kernels compiled for
  // kWideRt rank tiles
  const int RT = (p->R + 15) / 16;
  const bool wide_rank = RT > kMaxRankTiles;
  const int GRT = wide_rank ? kWideRt : RT;
  if (wide_rank && o->sampler == CPD_SAMPLER_LEVERAGE) {
    *why = "the leverage sampler takes R <= " + std::to_string(16 * kMaxRankTiles);
    return CPD_E_INVALID;
  }
  const LdsPlan lp = lds_plan(p->N, p->dims, p->R, p->B, wide_rank ? kMaxRankTiles : RT);
  const bool fits =
      !wide_rank && p->B <= CPD_MAX_PERSISTENT_BATCH && lp.total <= kLdsBudget;
  w->grid = o->path == CPD_PATH_GRID || (o->path == CPD_PATH_AUTO && !fits);
  w->lds = w->grid ? 0 : lp.total;
  if (!w->grid && !fits) {
    *why = wide_rank ? "the persistent step takes R <= " + std::to_string(16 * kMaxRankTiles)
           : p->B > CPD_MAX_PERSISTENT_BATCH
               ? "the persistent step takes B <= " + std::to_string(CPD_MAX_PERSISTENT_BATCH)
               : "problem needs " + std::to_string(lp.total) +
                     " bytes of LDS per workgroup (limit 163840): reduce B, R or the mode sizes";
    return CPD_E_INVALID;
  }
  w->wide_fb = w->wide_blocks = 0;
  w->gather_lds = w->refresh_lds = 0;
  if (w->grid) {
    int fb = wide_fibres(p->B);
    while (fb > kFibrePad && gather_plan(p->N, p->dims, GRT, fb).total > kLdsBudget) fb -= kFibrePad;
    w->gather_lds = gather_plan(p->N, p->dims, GRT, fb).total;
    w->refresh_lds = refresh_plan(p->N, p->dims, p->R, GRT).total;
    if (w->gather_lds > kLdsBudget || w->refresh_lds > kLdsBudget) {
      *why = "the grid step needs " + std::to_string(std::max(w->gather_lds, w->refresh_lds)) +
             " bytes of LDS per block (limit 163840): reduce R or the mode sizes";
      return CPD_E_INVALID;
    }
    w->wide_fb = fb;
    w->wide_blocks = (p->B + fb - 1) / fb;
  } else {
    // the all-mode CDF rebuild (init, state writes, rescaling) uses the grid
    // path's one-block-per-mode refresh where its LDS plan fits
    const size_t rl = refresh_plan(p->N, p->dims, p->R, RT).total;
    w->refresh_lds = rl <= kLdsBudget ? rl : 0;
  }
  for (int k = 0; k < p->N; ++k) {
    const int ks = o->ksplit[k];
    if (w->grid) {
      if (ks != 0) {
        *why = "ksplit applies to the persistent step only (must be 0 on the grid path)";
        return CPD_E_INVALID;
      }
      continue;
    }
    const int mx = max_ksplit(p->dims[k], o->storage, p->B, p->R);
    if (ks < 0 || ks > mx) {
      *why = "ksplit[" + std::to_string(k) + "] must be 0 (default) or in [1, " +
             std::to_string(mx) + "] for this mode";
      return CPD_E_INVALID;
    }
  }
  size_t off = 0;
  w->state = off;
  off = align_up(off + sizeof(ChainState) + 64);
  w->desc = off;
  off = align_up(off + sizeof(ChainDesc));
  w->parts = off;
  off = align_up(off + sizeof(double) * kFitParts);
  w->fitmap = off;
  off = align_up(off + sizeof(int32_t) * fit_table_len(1));
  w->wide_info = w->wide_part = 0;
  if (w->grid) {
    w->wide_info = off;
    off = align_up(off + sizeof(WideInfo));
    w->wide_part = off;
    // parts per block and mode as the gather kernel splits them
    const int vw = o->storage == CPD_BF16 ? 2 : 1;
    const int nck = w->wide_fb / (4 * chunk_steps(vw, (p->R + 15) / 16));
    size_t per_block = 0;
    for (int k = 0; k < p->N; ++k) {
      const int nst = (p->dims[k] + 16 * vw - 1) / (16 * vw);
      per_block = std::max(per_block, (size_t)wide_kparts(nst, nck) * p->R * p->dims[k]);
    }
    off = align_up(off + sizeof(float) * (size_t)w->wide_blocks * per_block);
  }
  for (int k = 0; k < p->N; ++k) {
    const size_t fb = sizeof(float) * (size_t)p->dims[k] * p->R;
    w->A[k] = off;
    off = align_up(off + fb);
    w->S[k] = off;
    off = align_up(off + fb);
    w->C[k] = off;
    off = align_up(off + sizeof(double) * p->dims[k]);
  }
  for (int n = 0; n < p->N; ++n) {
    w->ld[n] = (int32_t)round_up(p->dims[n], kLdAlign);
    w->rows[n] = total / p->dims[n];
    w->X[n] = off;
    off = align_up(off + es * (size_t)w->rows[n] * w->ld[n]);
  }
  w->total = off;
  return CPD_OK;
}

void fill_desc(const cpd_problem* p, const cpd_options* o, const WsPlan& w, char* base,
               ChainDesc* d) {
  std::memset(d, 0, sizeof(*d));
  d->N = p->N;
  d->R = p->R;
  d->B = p->B;
  d->RT = (p->R + 15) / 16;
  for (int k = 0; k < p->N; ++k) {
    d->dims[k] = p->dims[k];
    d->ld[k] = w.ld[k];
    d->ksplit[k] = o->ksplit[k] > 0 ? o->ksplit[k] : host_ksplit(p->dims[k], o->storage, p->B, p->R);
    d->vw[k] = host_vw(p->dims[k], o->storage);
    d->X[k] = base + w.X[k];
    d->A[k] = (float*)(base + w.A[k]);
    d->S[k] = (float*)(base + w.S[k]);
    d->C[k] = (double*)(base + w.C[k]);
  }
  d->dtype = o->storage;
  d->sampler = o->sampler;
  d->rule = o->rule;
  d->nonneg = o->nonneg;
  d->alpha = (float)o->alpha;
  d->eta = (float)o->eta;
  d->b = (float)o->b;
  d->beta = o->beta;
  d->gamma = o->gamma;
  d->key0 = p->seed;
  d->key1 = p->stream_id;
  d->state = (ChainState*)(base + w.state);
  d->parts = (double*)(base + w.parts);
  d->active = 1;
  d->autostop = 0;
  d->step_limit = 0;
  d->fit_target = 0.0;
}

// Copy the tensor and the initial factors of one decomposition into its
// workspace (zeroed first) and write its descriptor to d_desc.  Does not
// build the distributions.  Enqueued on `stream`; host input is staged
// synchronously in chunks.
cpd_status init_member(const cpd_problem* p, const cpd_options* o, const void* X, int x_dtype,
                       int x_space, const float* const* A0, const WsPlan& w, char* base,
                       hipStream_t stream, ChainDesc* desc, ChainDesc* d_desc) {
  hipError_t e = hipMemsetAsync(base, 0, w.total, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(workspace)");
  e = hipMemcpyAsync(d_desc, desc, sizeof(ChainDesc), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(desc)");
  for (int k = 0; k < p->N; ++k) {
    e = hipMemcpyAsync(desc->A[k], A0[k], sizeof(float) * (size_t)p->dims[k] * p->R,
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(A0)");
  }
  if (x_space == CPD_DEVICE) {
    e = launch_layout_from_dense(X, x_dtype, *desc, stream);
    if (e != hipSuccess) return hip_fail(e, "layout kernels");
    return CPD_OK;
  }
  // host input: rounded to the storage type on the host into two pinned
  // chunks (alternating, so conversion overlaps the copy of the previous
  // chunk), copied densely into the region of copy 1 (it holds at least
  // prod(dims) elements and is rebuilt afterwards), then spread into the
  // padded rows of copy 0 on the device and transposed into copies 1..N-1.
  const int64_t total = w.rows[0] * p->dims[0];
  const size_t es = o->storage == CPD_BF16 ? 2 : 4;
  const int64_t chunk = ((int64_t)8 << 20) / (int64_t)es;  // elements per chunk
  void* hb[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto release = [&]() {
    for (int q = 0; q < 2; ++q) {
      if (ev[q]) (void)hipEventDestroy(ev[q]);
      if (hb[q]) (void)hipHostFree(hb[q]);
    }
  };
  for (int q = 0; q < 2; ++q) {
    e = hipHostMalloc(&hb[q], (size_t)chunk * es, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[q], hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(stream);
      release();
      return hip_fail(e, "pinned staging");
    }
  }
  char* staged = (char*)desc->X[1];
  int q = 0;
  for (int64_t e0 = 0; e0 < total; e0 += chunk, q ^= 1) {
    const int64_t cnt = std::min(chunk, total - e0);
    e = hipEventSynchronize(ev[q]);  // the copy that last read this chunk is done
    if (e != hipSuccess) break;
    for (int64_t i = 0; i < cnt; ++i) {
      const float v = x_dtype == CPD_F64 ? (float)((const double*)X)[e0 + i]
                                         : ((const float*)X)[e0 + i];
      if (es == 2) ((uint16_t*)hb[q])[i] = f32_to_bf16_rne(v);
      else ((float*)hb[q])[i] = v;
    }
    e = hipMemcpyAsync(staged + (size_t)e0 * es, hb[q], (size_t)cnt * es, hipMemcpyHostToDevice,
                       stream);
    if (e != hipSuccess) break;
    e = hipEventRecord(ev[q], stream);
    if (e != hipSuccess) break;
  }
  hipError_t es2 = hipStreamSynchronize(stream);
  release();
  if (e != hipSuccess) return hip_fail(e, "staging copy of X");
  if (es2 != hipSuccess) return hip_fail(es2, "hipStreamSynchronize");
  e = launch_copy0_from_staged(staged, *desc, stream);
  if (e != hipSuccess) return hip_fail(e, "layout kernels");
  e = launch_layout_from_copy0(*desc, stream);
  if (e != hipSuccess) return hip_fail(e, "layout kernels");
  return CPD_OK;
}

cpd_status check_input_kinds(int x_dtype, int x_space) {
  if (x_dtype != CPD_F32 && x_dtype != CPD_F64) {
    set_error("x_dtype must be CPD_F32 or CPD_F64");
    return CPD_E_INVALID;
  }
  if (x_space != CPD_HOST && x_space != CPD_DEVICE) {
    set_error("x_space must be CPD_HOST or CPD_DEVICE");
    return CPD_E_INVALID;
  }
  return CPD_OK;
}

}  // namespace cpdmi

using namespace cpdmi;

struct cpd_handle {
  cpd_problem p;
  cpd_options o;
  int device;
  hipStream_t stream;
  char* ws;
  WsPlan plan;
  ChainDesc desc;       // host mirror of the device descriptor
  ChainDesc* d_desc;    // in the workspace
  int32_t* d_mode;      // scratch int in the state block
  int32_t* d_fitmap;    // fit block tables in the workspace
  FitPlan fit;
  // grid path: kGridGraphSteps steps captured once (on a private stream,
  // since the handle's may be the null stream) and replayed by cpd_step
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // step counter as issued from the host (steps of cpd_step / cpd_step_replay
  // since init or the last cpd_write_state): where rescale_every falls
  int64_t t_host = 0;
};

static constexpr int kGridGraphSteps = 16;

// The distributions of every mode from the current factors.
static hipError_t refresh_all(cpd_handle* h) {
  // one block per mode where the refresh kernel's LDS plan fits (it always
  // does on the grid path), else the step kernel's own refresh in one block;
  // both run the same refresh code, so the CDFs are the same
  if (h->plan.refresh_lds > 0)
    return launch_wide_refresh(h->d_desc, h->desc.RT, h->plan.refresh_lds, nullptr, -1, h->p.N,
                               h->stream);
  StepArgs a{};
  a.op = OP_REFRESH;
  return launch_chain_kernel(h->d_desc, 1, h->desc.RT, h->plan.lds, a, h->stream);
}

static WideArgs wide_args(cpd_handle* h, int op) {
  WideArgs a{};
  a.op = op;
  a.fb = h->plan.wide_fb;
  a.tsplit = wide_tsplit(h->plan.wide_blocks);
  a.part = (float*)(h->ws + h->plan.wide_part);
  a.info = (WideInfo*)(h->ws + h->plan.wide_info);
  return a;
}

// Update and CDF refresh of the grid step whose gather was just enqueued.
static hipError_t wide_finish(cpd_handle* h, const WideArgs& a) {
  int imax = 0;
  for (int k = 0; k < h->p.N; ++k) imax = std::max(imax, h->p.dims[k]);
  hipError_t e = launch_wide_update(h->d_desc, a.part, h->plan.wide_blocks, h->plan.wide_fb,
                                    a.info, imax * h->p.R, h->stream);
  if (e != hipSuccess || h->o.sampler == CPD_SAMPLER_UNIFORM) return e;
  return launch_wide_refresh(h->d_desc, h->desc.RT, h->plan.refresh_lds, a.info, -2, 1,
                             h->stream);
}

static hipError_t wide_steps(cpd_handle* h, int64_t nsteps, hipStream_t stream) {
  const WideArgs a = wide_args(h, OP_STEP);
  int imax = 0;
  for (int k = 0; k < h->p.N; ++k) imax = std::max(imax, h->p.dims[k]);
  for (int64_t i = 0; i < nsteps; ++i) {
    hipError_t e = launch_wide_gather(h->d_desc, h->desc.RT, h->o.storage, h->plan.wide_blocks,
                                      h->plan.gather_lds, a, stream);
    if (e == hipSuccess)
      e = launch_wide_update(h->d_desc, a.part, h->plan.wide_blocks, h->plan.wide_fb, a.info,
                             imax * h->p.R, stream);
    if (e == hipSuccess && h->o.sampler != CPD_SAMPLER_UNIFORM)
      e = launch_wide_refresh(h->d_desc, h->desc.RT, h->plan.refresh_lds, a.info, -2, 1, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static cpd_status build_step_graph(cpd_handle* h) {
  hipError_t e = hipSuccess;
  if (!h->cap) e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const hipError_t e1 = wide_steps(h, kGridGraphSteps, h->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(h->cap, &g);
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
  h->graph = g;
  h->exec = x;
  return CPD_OK;
}

static void release_graph(cpd_handle* h) {
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  h->exec = nullptr;
  h->graph = nullptr;
  h->cap = nullptr;
}

static cpd_status read_state(cpd_handle* h, ChainState* st) {
  hipError_t e = hipMemcpyAsync(st, h->ws + h->plan.state, sizeof(ChainState), hipMemcpyDeviceToHost,
                                h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state)");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return CPD_OK;
}

namespace cpdmi {
void describe_status(cpd_status s) {
  switch (s) {
    case CPD_OK: break;
    case CPD_E_RANK_DEFICIENT: set_error("a factor is rank deficient (leverage scores undefined)"); break;
    case CPD_E_DEGENERATE: set_error("all sampling weights of a factor are zero or not finite"); break;
    case CPD_E_DIVERGED: set_error("a factor became non-finite (step too large?)"); break;
    case CPD_E_INVALID: set_error("a replayed index is outside its mode"); break;
    default: set_error("device error " + std::to_string(s));
  }
}
}  // namespace cpdmi

static cpd_status device_status(cpd_handle* h) {
  ChainState st;
  cpd_status s = read_state(h, &st);
  if (s != CPD_OK) return s;
  describe_status(st.status);
  return st.status;
}

static cpd_status set_device(cpd_handle* h) {
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return CPD_OK;
}

extern "C" {

const char* cpd_last_error(void) { return g_last_error.c_str(); }

const char* cpd_version(void) { return "libcpdmi 0.1 (gfx950)"; }

cpd_status cpd_workspace_size(const cpd_problem* p, const cpd_options* o, size_t* bytes) {
  try {
    if (!bytes) {
      set_error("bytes is null");
      return CPD_E_INVALID;
    }
    WsPlan w;
    std::string why;
    cpd_status s = plan_workspace(p, o, &w, &why);
    if (s != CPD_OK) {
      set_error(why);
      return s;
    }
    *bytes = w.total;
    return CPD_OK;
  } catch (...) {
    set_error("unexpected exception");
    return CPD_E_INVALID;
  }
}

cpd_status cpd_init(const cpd_problem* p, const cpd_options* o, const void* X, int32_t x_dtype,
                    int32_t x_space, const float* const* A0, void* ws, size_t ws_bytes,
                    void* stream, cpd_handle** out) {
  try {
    if (!out || !X || !A0 || !ws) {
      set_error("null argument");
      return CPD_E_INVALID;
    }
    *out = nullptr;
    WsPlan w;
    std::string why;
    cpd_status s = plan_workspace(p, o, &w, &why);
    if (s != CPD_OK) {
      set_error(why);
      return s;
    }
    s = check_input_kinds(x_dtype, x_space);
    if (s != CPD_OK) return s;
    if (((uintptr_t)ws) % kAlign) {
      set_error("workspace must be 256-byte aligned");
      return CPD_E_INVALID;
    }
    if (ws_bytes < w.total) {
      set_error("workspace too small: need " + std::to_string(w.total) + " bytes");
      return CPD_E_OOM;
    }
    for (int k = 0; k < p->N; ++k)
      if (!A0[k]) {
        set_error("null initial factor");
        return CPD_E_INVALID;
      }
    cpd_handle* h = new (std::nothrow) cpd_handle();
    if (!h) {
      set_error("out of host memory");
      return CPD_E_OOM;
    }
    h->p = *p;
    h->o = *o;
    h->stream = (hipStream_t)stream;
    h->ws = (char*)ws;
    h->plan = w;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
      delete h;
      return hip_fail(e, "hipGetDevice");
    }
    fill_desc(p, o, w, h->ws, &h->desc);
    h->d_desc = (ChainDesc*)(h->ws + w.desc);
    h->d_mode = (int32_t*)(h->ws + w.state + sizeof(ChainState));
    auto fail = [&](hipError_t err, const char* what) {
      cpd_status r = hip_fail(err, what);
      (void)hipStreamSynchronize(h->stream);
      delete h;
      return r;
    };
    s = init_member(p, o, X, x_dtype, x_space, A0, w, h->ws, h->stream, &h->desc, h->d_desc);
    if (s != CPD_OK) {
      (void)hipStreamSynchronize(h->stream);
      delete h;
      return s;
    }
    int32_t fitmap[6];
    h->fit = plan_fit(&h->desc, 1, fitmap);
    h->d_fitmap = (int32_t*)(h->ws + w.fitmap);
    e = hipMemcpyAsync(h->d_fitmap, fitmap, sizeof fitmap, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return fail(e, "hipMemcpyAsync(fit table)");
    if (w.grid) {
      e = prepare_wide_kernels(h->desc.RT, o->storage);
      if (e != hipSuccess) return fail(e, "grid kernel attributes");
    }
    e = refresh_all(h);
    if (e != hipSuccess) return fail(e, "refresh kernel");
    e = launch_fit(h->d_desc, h->d_fitmap, 1, h->fit, o->storage, false, h->stream);
    if (e != hipSuccess) return fail(e, "norm kernels");
    s = device_status(h);
    if (s != CPD_OK) {
      delete h;
      return s;
    }
    *out = h;
    return CPD_OK;
  } catch (...) {
    set_error("unexpected exception in cpd_init");
    return CPD_E_INVALID;
  }
}

cpd_status cpd_sample(cpd_handle* h, uint64_t t, int32_t* mode, int32_t* idx_dev, double* p_dev) {
  if (!h || !mode || !idx_dev || !p_dev) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  hipError_t e;
  if (h->plan.grid) {
    WideArgs a = wide_args(h, OP_SAMPLE);
    a.sample_t = t;
    a.out_idx = idx_dev;
    a.out_p = p_dev;
    a.out_mode = h->d_mode;
    e = launch_wide_gather(h->d_desc, h->desc.RT, h->o.storage, h->plan.wide_blocks,
                           h->plan.gather_lds, a, h->stream);
  } else {
    StepArgs a{};
    a.op = OP_SAMPLE;
    a.sample_t = t;
    a.out_idx = idx_dev;
    a.out_p = p_dev;
    a.out_mode = h->d_mode;
    e = launch_chain_kernel(h->d_desc, 1, h->desc.RT, h->plan.lds, a, h->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "sample kernel");
  e = hipMemcpyAsync(mode, h->d_mode, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(mode)");
  return device_status(h);
}

static cpd_status step_plain(cpd_handle* h, int64_t nsteps) {
  cpd_status s = CPD_OK;
  if (h->plan.grid) {
    // whole groups of steps as graph replays (three launches per step would
    // otherwise be bound by the host), the rest launched directly
    int64_t done = 0;
    if (nsteps >= kGridGraphSteps) {
      if (!h->exec) {
        s = build_step_graph(h);
        if (s != CPD_OK) return s;
      }
      for (; done + kGridGraphSteps <= nsteps; done += kGridGraphSteps) {
        hipError_t e = hipGraphLaunch(h->exec, h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      }
    }
    hipError_t e = wide_steps(h, nsteps - done, h->stream);
    if (e != hipSuccess) return hip_fail(e, "grid step kernels");
    return CPD_OK;
  }
  const int64_t chunk = (int64_t)1 << 20;
  for (int64_t done = 0; done < nsteps; done += chunk) {
    StepArgs a{};
    a.op = OP_STEP;
    a.nsteps = std::min(chunk, nsteps - done);
    hipError_t e = launch_chain_kernel(h->d_desc, 1, h->desc.RT, h->plan.lds, a, h->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel");
  }
  return CPD_OK;
}

// Column rescaling, then the distributions of every mode from the
// rescaled factors (uniform ones do not depend on them).
static cpd_status rescale_now(cpd_handle* h) {
  hipError_t e = launch_rescale(h->d_desc, h->p.R, h->stream);
  if (e != hipSuccess) return hip_fail(e, "rescale kernel");
  if (h->o.sampler == CPD_SAMPLER_UNIFORM) return CPD_OK;
  e = refresh_all(h);
  if (e != hipSuccess) return hip_fail(e, "refresh kernel");
  return CPD_OK;
}

cpd_status cpd_step(cpd_handle* h, int64_t nsteps) {
  if (!h || nsteps < 0) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  const int64_t k = h->o.rescale_every;
  if (k <= 0) {
    s = step_plain(h, nsteps);
    if (s == CPD_OK) h->t_host += nsteps;
    return s;
  }
  // runs of steps up to the next multiple of k, each followed by a rescale
  for (int64_t done = 0; done < nsteps;) {
    const int64_t run = std::min(nsteps - done, k - h->t_host % k);
    s = step_plain(h, run);
    if (s != CPD_OK) return s;
    h->t_host += run;
    done += run;
    if (h->t_host % k == 0) {
      s = rescale_now(h);
      if (s != CPD_OK) return s;
    }
  }
  return CPD_OK;
}

cpd_status cpd_rescale(cpd_handle* h) {
  if (!h) {
    set_error("null handle");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  return rescale_now(h);
}

cpd_status cpd_step_replay(cpd_handle* h, int32_t mode, const int32_t* idx_dev) {
  if (!h || !idx_dev || mode < 0 || mode >= h->p.N) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  hipError_t e;
  if (h->plan.grid) {
    WideArgs a = wide_args(h, OP_REPLAY);
    a.replay_mode = mode;
    a.replay_idx = idx_dev;
    e = launch_wide_gather(h->d_desc, h->desc.RT, h->o.storage, h->plan.wide_blocks,
                           h->plan.gather_lds, a, h->stream);
    if (e == hipSuccess) e = wide_finish(h, a);
  } else {
    StepArgs a{};
    a.op = OP_REPLAY;
    a.replay_mode = mode;
    a.replay_idx = idx_dev;
    e = launch_chain_kernel(h->d_desc, 1, h->desc.RT, h->plan.lds, a, h->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "replay kernel");
  h->t_host += 1;
  if (h->o.rescale_every > 0 && h->t_host % h->o.rescale_every == 0) return rescale_now(h);
  return CPD_OK;
}

cpd_status cpd_sync(cpd_handle* h) {
  if (!h) {
    set_error("null handle");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  return device_status(h);
}

cpd_status cpd_fit(cpd_handle* h, double* fit) {
  if (!h || !fit) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  hipError_t e = launch_fit(h->d_desc, h->d_fitmap, 1, h->fit, h->o.storage, true, h->stream);
  if (e != hipSuccess) return hip_fail(e, "fit kernels");
  ChainState st;
  s = read_state(h, &st);
  if (s != CPD_OK) return s;
  *fit = st.fit;
  if (st.status != 0) return device_status(h);
  return CPD_OK;
}

cpd_status cpd_get_step(cpd_handle* h, int64_t* t) {
  if (!h || !t) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  ChainState st;
  cpd_status s = read_state(h, &st);
  if (s != CPD_OK) return s;
  *t = st.t;
  return CPD_OK;
}

cpd_status cpd_read_factors(cpd_handle* h, int32_t n, float* dst, int32_t dst_space) {
  if (!h || !dst || n < 0 || n >= h->p.N) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  hipError_t e = hipMemcpyAsync(dst, h->desc.A[n], sizeof(float) * (size_t)h->p.dims[n] * h->p.R,
                                dst_space == CPD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(factor)");
  return device_status(h);
}

cpd_status cpd_read_cdf(cpd_handle* h, int32_t n, double* dst) {
  if (!h || !dst || n < 0 || n >= h->p.N) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  hipError_t e = hipMemcpyAsync(dst, h->desc.C[n], sizeof(double) * (size_t)h->p.dims[n],
                                hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(cdf)");
  return device_status(h);
}

struct StateHeader {
  char magic[8];
  int32_t version, N, R, pad;
  int32_t dims[kMaxModes];
  int64_t t;
};

static size_t state_bytes(const cpd_handle* h) {
  size_t n = sizeof(StateHeader);
  for (int k = 0; k < h->p.N; ++k) n += 2 * sizeof(float) * (size_t)h->p.dims[k] * h->p.R;
  return n;
}

cpd_status cpd_read_state(cpd_handle* h, void* buf, size_t* bytes) {
  if (!h || !bytes) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  const size_t need = state_bytes(h);
  if (!buf) {
    *bytes = need;
    return CPD_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    set_error("state buffer too small");
    return CPD_E_INVALID;
  }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  ChainState st;
  s = read_state(h, &st);
  if (s != CPD_OK) return s;
  StateHeader hd{};
  std::memcpy(hd.magic, "CPDSTATE", 8);
  hd.version = 1;
  hd.N = h->p.N;
  hd.R = h->p.R;
  for (int k = 0; k < h->p.N; ++k) hd.dims[k] = h->p.dims[k];
  hd.t = st.t;
  char* out = (char*)buf;
  std::memcpy(out, &hd, sizeof hd);
  size_t off = sizeof hd;
  for (int k = 0; k < h->p.N; ++k) {
    const size_t fb = sizeof(float) * (size_t)h->p.dims[k] * h->p.R;
    hipError_t e = hipMemcpyAsync(out + off, h->desc.A[k], fb, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state A)");
    off += fb;
    e = hipMemcpyAsync(out + off, h->desc.S[k], fb, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state S)");
    off += fb;
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  *bytes = need;
  return CPD_OK;
}

cpd_status cpd_write_state(cpd_handle* h, const void* buf, size_t bytes) {
  if (!h || !buf) {
    set_error("null argument");
    return CPD_E_INVALID;
  }
  const size_t need = state_bytes(h);
  StateHeader hd;
  if (bytes < need) {
    set_error("state buffer too small");
    return CPD_E_INVALID;
  }
  std::memcpy(&hd, buf, sizeof hd);
  if (std::memcmp(hd.magic, "CPDSTATE", 8) != 0 || hd.version != 1 || hd.N != h->p.N ||
      hd.R != h->p.R) {
    set_error("state does not match this problem");
    return CPD_E_INVALID;
  }
  for (int k = 0; k < h->p.N; ++k)
    if (hd.dims[k] != h->p.dims[k]) {
      set_error("state does not match this problem");
      return CPD_E_INVALID;
    }
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  const char* in = (const char*)buf;
  size_t off = sizeof hd;
  for (int k = 0; k < h->p.N; ++k) {
    const size_t fb = sizeof(float) * (size_t)h->p.dims[k] * h->p.R;
    hipError_t e = hipMemcpyAsync(h->desc.A[k], in + off, fb, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state A)");
    off += fb;
    e = hipMemcpyAsync(h->desc.S[k], in + off, fb, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state S)");
    off += fb;
  }
  ChainState st{};
  st.t = hd.t;
  h->t_host = hd.t;
  hipError_t e = hipMemcpyAsync(h->ws + h->plan.state, &st, sizeof(int64_t) + sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state t)");
  e = refresh_all(h);
  if (e != hipSuccess) return hip_fail(e, "refresh kernel");
  return device_status(h);
}

// The exact variance is evaluated for R <= 64.
static bool variance_rank_ok(const cpd_handle* h) {
  if (h->p.R <= 16 * kMaxRankTiles) return true;
  set_error("the exact variance takes R <= " + std::to_string(16 * kMaxRankTiles));
  return false;
}

cpd_status cpd_variance_workspace_size(cpd_handle* h, int32_t n, size_t* bytes) {
  if (!h || !bytes || n < 0 || n >= h->p.N) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  if (!variance_rank_ok(h)) return CPD_E_INVALID;
  *bytes = variance_scratch_bytes(h->desc, n);
  return CPD_OK;
}

cpd_status cpd_variance(cpd_handle* h, int32_t n, int32_t sampler, void* ws, size_t ws_bytes,
                        double* out) {
  if (!h || !out || !ws || n < 0 || n >= h->p.N || sampler < 0 || sampler > 2 ||
      ((uintptr_t)ws & (kAlign - 1))) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  if (!variance_rank_ok(h)) return CPD_E_INVALID;
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  s = device_status(h);
  if (s != CPD_OK) return s;
  // the sampler's CDFs are rebuilt one block per mode where that kernel's
  // LDS plan fits (always on the grid path)
  return variance_eval(h->desc, h->plan.lds, h->plan.refresh_lds, n, sampler, h->stream, out, ws,
                       ws_bytes);
}

cpd_status cpd_variance_noalloc(cpd_handle* h, int32_t n, int32_t sampler, double* out) {
  if (!h || !out || n < 0 || n >= h->p.N || sampler < 0 || sampler > 2) {
    set_error("bad argument");
    return CPD_E_INVALID;
  }
  if (!variance_rank_ok(h)) return CPD_E_INVALID;
  cpd_status s = set_device(h);
  if (s != CPD_OK) return s;
  s = device_status(h);
  if (s != CPD_OK) return s;
  const size_t need = variance_scratch_bytes(h->desc, n);
  if (need > kVarStaticScratch) {
    set_error("cpd_variance_noalloc: this mode needs " + std::to_string(need) +
              " bytes of scratch, above the static " + std::to_string(kVarStaticScratch));
    return CPD_E_INVALID;
  }
  void* ws = nullptr;
  s = variance_static_scratch(&ws);
  if (s != CPD_OK) return s;
  return variance_eval(h->desc, h->plan.lds, h->plan.refresh_lds, n, sampler, h->stream, out, ws,
                       kVarStaticScratch);
}

cpd_status cpd_destroy(cpd_handle* h) {
  if (!h) return CPD_OK;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  release_graph(h);
  delete h;
  return CPD_OK;
}

}  // extern "C"
