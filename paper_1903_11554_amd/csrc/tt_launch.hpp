// Launch interface between the host translation unit and the per-integrand-class
// kernel translation units (each class is compiled separately, in parallel).
#pragma once

#include <hip/hip_runtime.h>

namespace ttx {

struct ProbDesc;

struct LaunchArgs {
  ProbDesc* desc;
  const int2* bond_tasks;
  int nbond;
  const int2* core_tasks;
  int ncore;
  int nprob;
  int mbucket;        // compile-time bound on the number of modes (0: streaming, any number)
  hipStream_t stream;
  int32_t* sweep_ctr; // two launch counters of the sweep kernel (zero between launches)
  int group;          // workgroups per superblock search (1 for the extended precisions)
};

enum { LAUNCH_START = 0, LAUNCH_INIT_UPDATE = 1, LAUNCH_SWEEP = 2, LAUNCH_ALS = 3 };

// what = LAUNCH_*; rbucket (8, 16, 32, 64) bounds every rank reachable in a sweep.
void launch_paper(const LaunchArgs& a, int what, int rbucket);
void launch_uform(const LaunchArgs& a, int what, int rbucket);
void launch_synth(const LaunchArgs& a, int what, int rbucket);
void launch_any(const LaunchArgs& a, int what, int rbucket);
void launch_paper_dd(const LaunchArgs& a, int what, int rbucket);   // double-double, paper form
void launch_paper_qd(const LaunchArgs& a, int what, int rbucket);   // quad-double, paper form

}  // namespace ttx
