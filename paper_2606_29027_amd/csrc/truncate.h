// HTACA final truncation (Supplement B), one problem or a group of
// independent problems.
#pragma once
#include <functional>
#include <vector>

#include "slar_internal.h"

namespace slar {

slar_status truncate_run(hipStream_t s, Workspace* ws, const slar_lowrank& in, double tol, int rmax,
                         slar_ht* out);
size_t truncate_scratch_elems(const GridDev& G);

// One problem of a grouped truncation: its own workspace, input factors and
// output tensor.  st ends as truncate_run's status for the same inputs.
struct TruncJob {
  Workspace* ws = nullptr;
  slar_lowrank in{};
  slar_ht* out = nullptr;
  slar_status st = SLAR_OK;
  // host decisions between phases
  int r = 0;
  double theta = 0.0;
  bool capped = false;
};

// each(fn) calls fn(j, stream) for every job index j, on streams that first
// wait for the work already on the group stream; the group stream then
// waits for everything fn enqueued.  Returns SLAR_OK or an error of its own.
using TruncEach = std::function<slar_status(const std::function<void(int, hipStream_t)>&)>;

// Device bytes (and pinned host bytes, same layout) for a group of `count`.
size_t truncate_group_bytes(int count);

// Every job truncated as by truncate_run (same kernels, arguments and
// summation orders, so bit-identical results), with the single-block
// factorisations of all jobs (Cholesky, core SVD, Gram eigenpairs, basis
// completion) in one launch per phase on s and the host decisions taken
// after one gathered read per phase.  dmem / hmem: truncate_group_bytes
// of device / pinned host memory.  Returns once every job's work is done;
// per-job statuses in jobs[j].st.
slar_status truncate_group(hipStream_t s, std::vector<TruncJob>& jobs, double tol, int rmax,
                           const TruncEach& each, void* dmem, void* hmem);

}  // namespace slar
