// HTACA final truncation (Supplement B), one problem or a group of
// independent problems.
#pragma once
#include <vector>

#include "slar_internal.h"

namespace slar {

slar_status truncate_run(hipStream_t s, Workspace* ws, const slar_lowrank& in, double tol, int rmax,
                         slar_ht* out);
size_t truncate_scratch_elems(const GridDev& G);

// One problem of a grouped truncation: its own workspace, input factors,
// output tensor and (may be null) output frames.  st ends as truncate_run's
// status for the same inputs.
struct TruncJob {
  Workspace* ws = nullptr;
  slar_lowrank in{};
  slar_ht* out = nullptr;
  slar_frames* frames = nullptr;   // ld >= the rank cap
  slar_status st = SLAR_OK;
  // host decisions between phases
  int r = 0;
  double theta = 0.0;
  bool capped = false;
};

// Device bytes (and pinned host bytes, same layout) for a group of `count`.
size_t truncate_group_bytes(int count);

// Every job truncated as by truncate_run, followed by frames_from_ht into
// job.frames when given (same kernel bodies, arguments and summation
// orders, so bit-identical results): each step is one grouped launch over
// all jobs on s (group.h), and the host takes the rank decisions of all
// jobs after one gathered read of the singular values and one of the
// eigenvalues.  dmem / hmem: truncate_group_bytes of device / pinned host
// memory.  Returns once every job's work is done; per-job statuses in
// jobs[j].st (an error of a grouped launch fails every job).
slar_status truncate_group(hipStream_t s, std::vector<TruncJob>& jobs, double tol, int rmax, void* dmem,
                           void* hmem);

}  // namespace slar
