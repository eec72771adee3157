// Host-side runtime pieces shared by the single-decomposition API, the
// batched path and the server: workspace planning and kernel launchers.
#pragma once

#include <string>

#include "cpd_internal.hpp"
#include "wide_internal.hpp"

namespace cpdmi {

hipError_t launch_chain_kernel(const ChainDesc* descs, int nchains, int rt, size_t lds_bytes,
                               const StepArgs& args, hipStream_t stream);
hipError_t launch_layout_from_dense(const void* X, int in_dtype, const ChainDesc& d,
                                    hipStream_t stream);
hipError_t launch_layout_from_copy0(const ChainDesc& d, hipStream_t stream);
hipError_t launch_copy0_from_staged(const void* staged, const ChainDesc& d, hipStream_t stream);
// Fit work split over a set of decompositions.  Three block tables of
// nchains + 1 prefix sums each (fit_table_len entries in all): the blocks of
// every decomposition, then the same for the decompositions whose inner pass
// stages little LDS ("light") and for the others ("heavy"), 0 blocks for the
// rest.  The partial pass runs as one launch per non-empty group, so a few
// decompositions that need much LDS do not lower the occupancy of all.
struct FitPlan {
  int32_t blocks[2];  // light, heavy
  size_t lds[2];      // dynamic LDS of the inner pass per group
  int32_t passes;     // inner passes over 64 ranks each (2 when some R > 64)
};
inline int fit_table_len(int nchains) { return 3 * (nchains + 1); }
FitPlan plan_fit(const ChainDesc* host_descs, int nchains, int32_t* tables);
// d_tables: device copy of the tables of plan_fit.
hipError_t launch_fit(const ChainDesc* d_descs, const int32_t* d_tables, int nchains,
                      const FitPlan& fp, int dtype, bool inner, hipStream_t stream);

// Grid-wide step (wide_step.hip).  Gather: nblocks slices of a.fb fibres,
// a.tsplit blocks per slice, wide_kparts parts of -G^T per slice; update: the parts of every entry of mode n summed
// and applied (launched over max_rows * R entries); refresh: the CDF of mode `mode` (-1: every
// one of the nmodes modes, one block each; -2: the mode in info).
hipError_t launch_wide_gather(const ChainDesc* d_desc, int rt, int dtype, int nblocks,
                              size_t lds_bytes, const WideArgs& a, hipStream_t stream);
hipError_t launch_wide_update(const ChainDesc* d_desc, const float* part, int nblocks, int fb,
                              const WideInfo* info, int max_entries, hipStream_t stream);
hipError_t launch_wide_refresh(const ChainDesc* d_desc, int rt, size_t lds_bytes,
                               const WideInfo* info, int mode, int nmodes, hipStream_t stream);
// Column rescaling of every factor (rescale.hip): one block per rank
// component, R blocks.
hipError_t launch_rescale(const ChainDesc* d_desc, int R, hipStream_t stream);
// Sets the dynamic-LDS limits of the grid kernels for (rt, dtype); called
// before any of them is captured into a graph.
hipError_t prepare_wide_kernels(int rt, int dtype);

// Offsets of every region of one decomposition's workspace.
struct WsPlan {
  size_t state, desc, parts, fitmap;
  int grid;                 // 1: the grid-wide step (CPD_PATH_GRID)
  int wide_fb, wide_blocks; // grid path: fibres per gather block, gather blocks
  size_t wide_info, wide_part;      // grid path: WideInfo, block parts
  size_t gather_lds, refresh_lds;   // grid path: dynamic LDS of its kernels
  size_t A[kMaxModes], S[kMaxModes], C[kMaxModes];
  size_t X[kMaxModes];
  int32_t ld[kMaxModes];
  int64_t rows[kMaxModes];  // J_n
  size_t total;
  size_t lds;               // dynamic LDS of the step kernel
};

// Validates the problem; returns CPD_OK or CPD_E_INVALID with a message.
cpd_status plan_workspace(const cpd_problem* p, const cpd_options* o, WsPlan* out,
                          std::string* why);

// Fill a descriptor for a workspace at `base` (device address).
void fill_desc(const cpd_problem* p, const cpd_options* o, const WsPlan& w, char* base,
               ChainDesc* d);

cpd_status init_member(const cpd_problem* p, const cpd_options* o, const void* X, int x_dtype,
                       int x_space, const float* const* A0, const WsPlan& w, char* base,
                       hipStream_t stream, ChainDesc* desc, ChainDesc* d_desc);
cpd_status check_input_kinds(int x_dtype, int x_space);

// Message for a sticky device status (sets the thread's last error).
void describe_status(cpd_status s);

// Exact variance of the sampled gradient of mode n (variance.hip).
// grid_refresh_lds > 0: the distributions are rebuilt by the grid path's
// refresh kernel (one block per mode, with that LDS) instead of the
// persistent kernel.
// The scratch is caller-owned device memory of at least
// variance_scratch_bytes(host_desc, n) bytes (CPD_E_OOM otherwise).
size_t variance_scratch_bytes(const ChainDesc& host_desc, int n);
// Bytes of the static scratch of cpd_variance_noalloc (one array per device),
// and its device address on the current device (looked up once per device).
constexpr size_t kVarStaticScratch = 20u << 20;
cpd_status variance_static_scratch(void** ptr);
cpd_status variance_eval(const ChainDesc& host_desc, size_t lds, size_t grid_refresh_lds, int n,
                         int sampler, hipStream_t stream, double* out3, void* scratch,
                         size_t scratch_bytes);

void set_error(const std::string& msg);
cpd_status hip_fail(hipError_t e, const char* what);

}  // namespace cpdmi
