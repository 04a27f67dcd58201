// Kernel instantiations for one integrand class (TT_FAM = FAM_PAPER, FAM_UFORM,
// FAM_SYNTH or FAM_ANY) and one number type (TT_INST_DD = 0: double, 1:
// double-double, paper form only), compiled once per combination.
#include "tt_kernels.hpp"
#include "tt_launch.hpp"

#ifndef TT_FAM
#error "compile with -DTT_FAM=<integrand class>"
#endif
#ifndef TT_INST_DD
#define TT_INST_DD 0
#endif
#ifndef TT_INST_QD
#define TT_INST_QD 0
#endif
#if (TT_INST_DD || TT_INST_QD) && TT_FAM != 0
#error "the double-double and quad-double kernels exist for the paper-form class only"
#endif

namespace ttx {
namespace {

#if TT_INST_QD
using Real = qd;
#elif TT_INST_DD
using Real = dd;
#else
using Real = double;
#endif

template <int MAXM, int RMAX>
void sweep(const LaunchArgs& a) {
  // group workgroups per superblock, then one per core
  const int group = a.group < 1 ? 1 : a.group;
  hipLaunchKernelGGL((k_sweep<Real, TT_FAM, MAXM, RMAX>), dim3(group * a.nbond + a.ncore), dim3(kSweepBlock), 0,
                     a.stream, a.desc, a.bond_tasks, a.nbond, a.core_tasks, a.sweep_ctr, group);
}

template <int MAXM>
void by_rank(const LaunchArgs& a, int what, int rb) {
  if (what == LAUNCH_START) {
    hipLaunchKernelGGL((k_start<Real, TT_FAM, MAXM>), dim3(a.nprob), dim3(kBlock), 0, a.stream, a.desc);
    return;
  }
  if (what == LAUNCH_ALS) {   // double precision only (the host rejects the other precisions)
#if !TT_INST_DD && !TT_INST_QD
    hipLaunchKernelGGL((k_als<TT_FAM, MAXM>), dim3(a.nprob), dim3(kSweepBlock), 0, a.stream, a.desc);
#endif
    return;
  }
  if (what == LAUNCH_INIT_UPDATE) {
    hipLaunchKernelGGL((k_update<Real, TT_FAM, MAXM, 8>), dim3(a.ncore), dim3(kSweepBlock), 0, a.stream,
                       a.desc, a.core_tasks, 1);
    return;
  }
  switch (rb) {
#if TT_INST_QD
    case 8:
    case 16: sweep<MAXM, 16>(a); break;
    default: sweep<MAXM, 32>(a); break;   // quad-double ranks are at most 32
#else
    case 8: sweep<MAXM, 8>(a); break;
    case 16: sweep<MAXM, 16>(a); break;
    case 32: sweep<MAXM, 32>(a); break;
    default: sweep<MAXM, 64>(a); break;
#endif
  }
}

// Mode buckets: the paper-form class in double (the Ising workloads) has fine
// buckets, since every mode a kernel is compiled for beyond the problem's costs
// a guarded loop step per run; the other classes share 8, 16, 32.  Bucket 0 is
// the streaming path for more modes than the registers hold (double only,
// paper-form and synthetic integrands).
void dispatch(const LaunchArgs& a, int what, int rb) {
#if TT_INST_QD
  by_rank<16>(a, what, rb);   // quad-double: one mode bucket (compile time grows fast with each)
#elif TT_FAM == 0 && !TT_INST_DD
  switch (a.mbucket) {
    case 0: by_rank<0>(a, what, rb); break;
    case 4: by_rank<4>(a, what, rb); break;
    case 8: by_rank<8>(a, what, rb); break;
    case 10: by_rank<10>(a, what, rb); break;
    case 12: by_rank<12>(a, what, rb); break;
    case 16: by_rank<16>(a, what, rb); break;
    case 24: by_rank<24>(a, what, rb); break;
    default: by_rank<32>(a, what, rb); break;
  }
#else
  switch (a.mbucket) {
#if !TT_INST_DD && TT_FAM != 1
    case 0: by_rank<0>(a, what, rb); break;
#endif
    case 8: by_rank<8>(a, what, rb); break;
    case 16: by_rank<16>(a, what, rb); break;
    default: by_rank<32>(a, what, rb); break;
  }
#endif
}

}  // namespace

#if TT_INST_QD
void launch_paper_qd(const LaunchArgs& a, int what, int rb) { dispatch(a, what, rb); }
#elif TT_INST_DD
void launch_paper_dd(const LaunchArgs& a, int what, int rb) { dispatch(a, what, rb); }
#elif TT_FAM == 0
void launch_paper(const LaunchArgs& a, int what, int rb) { dispatch(a, what, rb); }
#elif TT_FAM == 1
void launch_uform(const LaunchArgs& a, int what, int rb) { dispatch(a, what, rb); }
#elif TT_FAM == 2
void launch_synth(const LaunchArgs& a, int what, int rb) { dispatch(a, what, rb); }
#else
void launch_any(const LaunchArgs& a, int what, int rb) { dispatch(a, what, rb); }
#endif

}  // namespace ttx
