/*
 * ttcross.h — C ABI of the MI355X (gfx950) tensor-train cross integration library.
 *
 * The library computes integrals over [0,1]^m of a built-in integrand by the
 * tensor-product Gauss--Legendre rule (Dolgov & Savostyanov, arXiv:1903.11554,
 * Sec. 4.1, eq. quad_product), approximating the weighted tensor
 *     B(i_1..i_m) = w_{i_1} ... w_{i_m} f(t_{i_1}, ..., t_{i_m})
 * (weights folded in, last paragraph of Sec. 4.1) by the TT cross formula
 * eq. tt (Sec. 3.2).  The index sets grow by the dimension-parallel greedy
 * cross of Alg. 6 (Sec. 3.4) with one superblock per GPU workgroup: every
 * superblock runs one step of Alg. 2 (random then rook pivoting, eq. rook)
 * against the previous sweep's index sets, and accepted pivots are appended
 * after the sweep.  The integral is the product of 2m-1 matrices of Sec. 4.1.
 * Inside a job the folded weights are the rule's times 2^s, s the integer
 * nearest log2 n (their mean becomes about 1; exact, so no decision changes),
 * and the chain of matrices is rescaled by exact powers of two: the values of
 * B that the pivot log reports carry the factor 2^(s m); the integral does not.
 *
 * All compute runs in HIP kernels on the device; the host code only validates,
 * allocates and launches.  Every function returns a tt_status (or a plain value
 * where stated); no C++ exception crosses this boundary, and outputs are left
 * untouched when an error is returned (one exception: TT_ENUMERIC from
 * tt_cross_sweep and tt_cross_run, which still fill the per-integral infos).
 *
 * Ownership: the library owns every device buffer it allocates (index sets,
 * cores, interpolation cores, logs); they live from tt_cross_init to
 * tt_cross_free.  Callers own tt_problem structs and their params arrays,
 * which are copied at init.  Pointers documented as "device" must point to
 * device memory of the context's GPU; all others are host pointers.
 *
 * Thread safety: a tt_job must be used from one host thread at a time; a
 * tt_ctx may be shared, calls that enqueue work serialise on its stream.
 */
#ifndef TTCROSS_H
#define TTCROSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TT_OK = 0,
  TT_CONVERGED = 1,      /* every integral of the job met its stopping rule            */
  TT_NOT_CONVERGED = 2,  /* work remains (more sweeps needed)                          */
  TT_PENDING = 3,        /* a served request has not finished yet                      */
  TT_EINVAL = -1,        /* invalid argument (see each function)                       */
  TT_ENOMEM = -2,        /* device allocation failed or footprint over the limit       */
  TT_EDEVICE = -3,       /* a HIP runtime call failed                                  */
  TT_ENUMERIC = -4       /* non-finite integrand value, zero start, singular cross     */
} tt_status;

/* Integrand families.
 * Paper form (Sec. 5.1, eqs. c, d, e): m = d-1 modes, variables x_2..x_d in [0,1];
 *   C_d = 2 int B_d, D_d = 2 int A_d B_d, E_d = 2 int A_d (factor 2 included).
 * u-form: m = d modes, the (0,inf)^d form of C_d and D_d mapped by u = x/(1-x).
 * Synthetic: m = d modes on [0,1]^d, params = a[0..d) followed by b[0..d):
 *   PROD_EXP = prod_j exp(-a_j x_j); SUM2_EXP_COS = prod exp(-a_j x_j) + prod cos(b_j x_j). */
typedef enum {
  TT_ISING_C = 1, TT_ISING_D = 2, TT_ISING_E = 3,
  TT_ISING_C_U = 11, TT_ISING_D_U = 12,
  TT_PROD_EXP = 21, TT_SUM2_EXP_COS = 22
} tt_integrand;

/* Number type of a job's whole computation.
 * TT_FP64: IEEE double throughout.
 * TT_DD: double-double (a value is an unevaluated sum hi + lo of two doubles,
 *   about 32 significant digits), standing in for the quadruple and multiple
 *   precision runs of Sec. 5.2: nodes, weights, integrand values, interpolation
 *   cores, the pivot errors and the quadrature are all double-double; the pivot
 *   choice and the acceptance test compare the leading double.  Paper-form
 *   integrands (TT_ISING_C, TT_ISING_D, TT_ISING_E) only.
 * TT_QD: quad-double (four doubles of decreasing magnitude, about 61 significant
 *   digits), the precision beyond the paper's quadruple: every value as for
 *   TT_DD; each operation rounds the exact sum of its operands' components (or of
 *   their exact partial products) to four components.  Paper-form integrands, at
 *   most TT_QD_MAX_MODES modes and rank TT_QD_MAX_RANK; tt_cross_init, sweep, run,
 *   integrate, tt_batch_run and the state exports (tt_job_history_parts,
 *   tt_job_nodes_parts give all four components); the other entry points reject it.
 * All integrals of one job must use the same precision. */
typedef enum { TT_FP64 = 0, TT_DD = 1, TT_QD = 2 } tt_precision;
#define TT_QD_MAX_MODES 16
#define TT_QD_MAX_RANK 32

/* Stop reasons reported in tt_info.reason.  TT_STOP_ERROR: the integral was
 * stopped because a sweep raised one of the err_flags bits (its value is not a
 * result of the stopping rule and must not be used as one). */
enum { TT_RUNNING = 0, TT_STOP_CONVERGED = 1, TT_STOP_RANK_CAP = 2, TT_STOP_MAX_SWEEPS = 3,
       TT_STOP_ERROR = 4 };

/* Library limits (a problem beyond them is rejected with TT_EINVAL).
 * Jobs take up to TT_MAX_MODES modes.  Above TT_MAX_REG_MODES the kernels read
 * the coordinates of every point from the index-set rows in device memory one
 * at a time (the paper's 1023-mode C_1024 of Sec. 5.3 is such a job); that path
 * covers the paper-form and synthetic integrands in TT_FP64.  Double-double
 * jobs, the u-form integrands, tt_eval_points/tt_eval_fibers, tt_mc_integrate
 * and the serving loop take at most TT_MAX_REG_MODES modes. */
#define TT_MAX_MODES 1024
#define TT_MAX_REG_MODES 32
#define TT_MAX_RANK 64
#define TT_MAX_NODES 256

typedef struct {
  int32_t integrand;   /* tt_integrand                                                   */
  int32_t d;           /* Ising: the paper's d (number of u variables); synthetic: dim    */
  int32_t n_nodes;     /* Gauss--Legendre nodes per mode on [0,1], 1..TT_MAX_NODES        */
  int32_t rank_cap;    /* maximum TT rank of every bond, 1..TT_MAX_RANK                   */
  double  tol;         /* relative tolerance > 0 (pivot acceptance and stopping rule)     */
  int32_t precision;   /* tt_precision                                                    */
  int32_t max_sweeps;  /* 0 selects 4*rank_cap; at most 1024                              */
  uint64_t seed;       /* key of the SplitMix64 counter-based sample generator            */
  const double *params;/* synthetic families: 2*d doubles (a then b); NULL otherwise      */
  int32_t stop_rule;   /* tt_stop_rule; 0 (TT_STOP_REL2) for the default                    */
  int32_t reserved;    /* 0                                                               */
} tt_problem;

/* The stopping rule (the paper measures "internal convergence" without defining
 * it, Sec. 5.2-5.5).  Both rules also stop on a sweep that accepts no pivot,
 * when every bond is at rank_cap, and at max_sweeps.
 *   TT_STOP_REL2:   converged after two consecutive sweeps whose relative change
 *                   of the integral is <= tol;
 *   TT_STOP_STRICT: that alone does not stop: the integral runs until a sweep
 *                   accepts no pivot (no superblock error above tol * its largest
 *                   |B|), every bond is at the cap, or max_sweeps. */
typedef enum { TT_STOP_REL2 = 0, TT_STOP_STRICT = 1 } tt_stop_rule;

/* Per-integral result and progress. value is the current TT quadrature. */
typedef struct {
  int32_t sweeps;      /* sweeps done                                                     */
  int32_t max_rank;    /* largest bond rank                                               */
  int32_t reason;      /* TT_RUNNING or a TT_STOP_* code                                  */
  int32_t err_flags;   /* bits: non-finite value (1), singular cross (2), zero start (4),
                          internal rank bucket overflow (8), a wait inside a sweep
                          (a core update's for its neighbouring searches, or a
                          superblock's workgroups' for each other) timed out (16)         */
  int64_t evals;       /* integrand evaluations so far (start, samples, fibers, cores)    */
  double  value;       /* integral estimate (TT_DD: its leading double)                   */
  double  rel_change;  /* |I_s - I_{s-1}| / |I_s| of the last sweep                       */
  double  value_lo;    /* TT_DD: the low double of the estimate (value + value_lo); else 0 */
  double  value_mant;  /* the estimate is value_mant * 2^value_exp2 exactly (TT_DD: its    */
  int32_t value_exp2;  /*   leading double), 1/2 <= |value_mant| < 1 or 0; value and       */
  int32_t recomputes;  /*   value_lo are 0 or +-inf when the estimate leaves the double range;
                          recomputes: interpolation cores rebuilt from F_c with a pivoted
                          solve so far (double jobs whose crosses lost dominance)        */
  int32_t value_scale; /* E: above 32 modes every value of B the job forms (pivot log,
                          cores) is f W 2^(s m) 2^E, E fixed at the start so that its B
                          lies in [1/2, 1) (D_d falls below the double range from about
                          d = 512, Sec. 5.5); 0 up to 32 modes. value_mant/value_exp2
                          are unscaled.                                                   */
  int32_t reserved;
} tt_info;

/* One accepted-or-rejected pivot search of one superblock in one sweep.
 * row = alpha*n + i over (I_<=b-1 x nodes), col = j*r_{b+1} + beta over
 * (nodes x I_>b+1), with the ranks at the time of the search. */
typedef struct {
  int32_t row, col;    /* pivot position in the superblock (-1: not searched)            */
  int32_t accepted;    /* 1 if appended to the index sets                                 */
  int32_t iters;       /* rook (column,row) pairs used, 1..5; 0 if not searched            */
  double  err;         /* B - B~ at the pivot, B with the job's weights (times 2^(s m)
                          2^E, E = tt_info.value_scale); signed; TT_DD: leading double   */
  double  value;       /* B at the pivot (same scale; TT_DD: leading double)              */
  int32_t col_fresh;   /* 1 if the last column step of the rook loop was at `col`: its
                          values are the new column of the core left of the bond       */
  int32_t reserved;
} tt_pivot;

typedef struct tt_ctx tt_ctx;
typedef struct tt_job tt_job;

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run
 * on (e.g. PyTorch's current stream), or NULL for a library-owned stream.
 * Errors: TT_EINVAL (out == NULL), TT_EDEVICE (bad device / HIP failure). */
tt_status tt_ctx_create(int device, void *hip_stream, tt_ctx **out);
void tt_ctx_destroy(tt_ctx *ctx);

/* Bytes of device memory one problem needs at its rank cap (0 if invalid). */
size_t tt_job_footprint(const tt_problem *problem);

/* Start a job of `count` independent integrals (a batch: every kernel launch
 * serves all of them).  Generates the Gauss--Legendre nodes, draws the rank-1
 * start of each integral (largest |B| among 1024 SplitMix64 grid samples),
 * evaluates the first cores and the first quadrature value.  Synchronises.
 * Errors: TT_EINVAL (bad problem: d < 1, modes > TT_MAX_MODES (> TT_MAX_REG_MODES
 * for TT_DD and the u-form), n or rank out of
 * range, tol <= 0, unknown integrand or precision, TT_DD for an integrand
 * without a double-double path, precisions mixed in one job, missing params),
 * TT_ENOMEM, TT_EDEVICE, TT_ENUMERIC (all start samples zero or non-finite). */
tt_status tt_cross_init(tt_ctx *ctx, const tt_problem *problems, int32_t count, tt_job **out);

/* Enqueue n_sweeps sweeps of Alg. 6 for every integral not yet stopped, then
 * synchronise and fill info[count] (may be NULL).  Returns TT_CONVERGED when
 * every integral has stopped, TT_NOT_CONVERGED otherwise, and TT_ENUMERIC when
 * an integral has stopped with reason TT_STOP_ERROR (non-zero err_flags).  With
 * TT_ENUMERIC, unlike the other errors, info is still filled, so the caller can
 * see which integral failed and keep the others' results. */
tt_status tt_cross_sweep(tt_job *job, int32_t n_sweeps, tt_info *info);

/* Sweep until every integral stops (stopping rule, max_sweeps or a numeric
 * error); fills info.  Status as tt_cross_sweep. */
tt_status tt_cross_run(tt_job *job, tt_info *info);

/* One ALS maxvol refresh of the index sets of every integral still running, at
 * fixed ranks (Sec. 3.3, Alg. 3, with the row swaps of Alg. 1, Sec. 2.4): left
 * to right, bond b's left set becomes the maxvol rows of the r_{b-1} n x r_b
 * matrix B(I_<=b-1 x [n], I_>b) on the left set refreshed one step before; right
 * to left, its right set the maxvol columns of B(I_<=b, [n] x I_>b+1).  maxvol:
 * Gaussian elimination with partial pivoting, then Alg. 1 swaps while the
 * largest |B(:, I)^-1 B| exceeds 1.01 (at most 4 r swaps).  The sets stay nested;
 * the cores, the interpolation cores (recomputed from the cores in every later
 * sweep too) and the integral are rebuilt on them, and the integral replaces the
 * value after the last sweep (tt_job_history), so the next sweep's relative
 * change is taken from it.  Each bond's largest |B| takes the refresh's values
 * into account; every value evaluated counts in tt_info.evals.  TT_FP64 jobs
 * only: TT_EINVAL for double-double jobs.  TT_ENUMERIC (infos filled, the
 * integral stopped with TT_STOP_ERROR) if a matrix has lower rank than its bond
 * or a value is not finite. */
tt_status tt_cross_refresh(tt_job *job, tt_info *info);

/* A batch of count integrals solved together in one call: tt_cross_init,
 * tt_cross_run and tt_cross_free of one job (every kernel launch serves all of
 * them), info[count] filled with each integral's result.  Status as
 * tt_cross_run (TT_CONVERGED; TT_ENUMERIC with info filled if an integral
 * stopped on a numeric error), or an error of tt_cross_init. */
tt_status tt_batch_run(tt_ctx *ctx, const tt_problem *problems, int32_t count, tt_info *info);

/* Enqueue n_sweeps sweeps of Alg. 6 on the context stream and return at once:
 * no host synchronisation, no allocation, no memset, so the call may run while
 * the caller captures that stream into a HIP graph.  Every enqueued sweep uses
 * the kernels sized for the job's rank caps, so captured launches stay valid
 * however far a replayed graph advances the integrals; sweeps of integrals that
 * have stopped return at once.  Read the results with tt_cross_integrate after
 * the work has run.  Errors: TT_EINVAL (NULL job, n_sweeps < 0, or per-kernel
 * profiling switched on), TT_EDEVICE. */
tt_status tt_cross_enqueue(tt_job *job, int32_t n_sweeps);

/* Copy the integral values (count doubles, host) and infos (may be NULL). */
tt_status tt_cross_integrate(tt_job *job, double *values, tt_info *info);

/* Diagnostics for tests: the pivot log of integral k (sweeps x (m-1) records,
 * host buffer of `capacity` records, *written = records copied), the
 * integral after the start and after each sweep (sweeps+1 values: leading
 * doubles in `values`, low doubles in `values_lo` if not NULL, 0 for TT_FP64;
 * with exp2 not NULL, values and values_lo receive mantissas and exp2 the
 * powers of two, value = (values + values_lo) * 2^exp2, for integrals outside
 * the double range), and the
 * index sets: for bond b the left set I_<=b as rows of (b+1) node indices and
 * the right set I_>b as rows of (m-b-1) node indices, packed bond by bond
 * (left then right), each row in insertion order; ranks[m-1] receives r_b. */
tt_status tt_job_pivot_log(tt_job *job, int32_t k, tt_pivot *log, int64_t capacity, int64_t *written);
tt_status tt_job_history(tt_job *job, int32_t k, double *values, double *values_lo, int32_t *exp2,
                         int64_t capacity, int64_t *written);
tt_status tt_job_index_sets(tt_job *job, int32_t k, int32_t *ranks, int32_t *nodes,
                            int64_t capacity, int64_t *written);
/* Core c (0 <= c < m) of integral k at the current ranks, for tests: F_c =
 * B(I_<=c-1 x nodes, I_>c) as an (r_{c-1} n) x r_c row-major host array (row
 * alpha*n + i, the index sets in insertion order, B with the job's weights),
 * and for c < m-1 the interpolation core C_c = F_c M_c^-1 (M_c the rows I_<=c
 * of F_c) in the same layout; C may be NULL, and is left untouched for the last
 * core.  TT_DD: leading doubles.  *rows and *cols receive r_{c-1} n and r_c.
 * Errors: TT_EINVAL (bad k or c, NULL F/rows/cols, capacity below rows*cols). */
tt_status tt_job_core(tt_job *job, int32_t k, int32_t c, double *F, double *C, int64_t capacity,
                      int32_t *rows, int32_t *cols);

/* Gauss--Legendre nodes and weights of integral k as generated on the device, n
 * each: t and w rounded to double; t_lo and w_lo (may be NULL) receive the low
 * doubles of the double-double tables (t + t_lo, w + w_lo), for any precision. */
tt_status tt_job_nodes(tt_job *job, int32_t k, double *t, double *w, double *t_lo, double *w_lo);
/* The integral after the start and after every sweep (as tt_job_history with
 * exp2) and the job's unscaled nodes and weights, `parts` (1..4) components per
 * value, leading component first: 1 for TT_FP64, 2 for TT_DD and 4 for TT_QD
 * hold every component, further ones are 0.  values: capacity * parts doubles,
 * exp2: capacity int32 (value = (sum of the components) * 2^exp2); t, w: n * parts
 * doubles.  Errors: TT_EINVAL (parts outside 1..4, NULL outputs, capacity too
 * small). */
tt_status tt_job_history_parts(tt_job *job, int32_t k, int32_t parts, double *values, int32_t *exp2,
                               int64_t capacity, int64_t *written);
tt_status tt_job_nodes_parts(tt_job *job, int32_t k, int32_t parts, double *t, double *w);
void tt_cross_free(tt_job *job);

/* Standalone batched integrand evaluation (the fiber-evaluation kernel of the
 * sweep, exposed for parity checks and roofline measurement).
 * tt_eval_points: B at npts multi-indices; d_idx is a device int32 array of
 * npts*m node indices (row-major, one row per point), d_out a device double
 * array of npts values (TT_DD: 2*npts doubles, the pairs (hi, lo) of each
 * value in turn).  Asynchronous on the context stream.
 * tt_eval_fibers: B over the fiber set I_left x [n] x I_right at mode position
 * `pos` (0 <= pos < m): d_left is device int32 [r_left * pos] node indices,
 * d_right device int32 [r_right * (m-pos-1)]; d_out receives r_left*n*r_right
 * values in the order (alpha, i, beta), beta fastest (TT_DD: (hi, lo) pairs,
 * twice as many doubles).  Asynchronous.
 * Errors: TT_EINVAL (bad problem or sizes), TT_EDEVICE. */
tt_status tt_eval_points(tt_ctx *ctx, const tt_problem *problem, const int32_t *d_idx,
                         int64_t npts, double *d_out);
tt_status tt_eval_fibers(tt_ctx *ctx, const tt_problem *problem, int32_t pos,
                         const int32_t *d_left, int32_t r_left,
                         const int32_t *d_right, int32_t r_right, double *d_out);

/* Equal-weight quadratures of Sec. 4.2, the baselines the paper compares the
 * cross with: Monte Carlo (kind TT_MC_RANDOM, eq. mc) and a randomly shifted
 * rank-1 lattice rule (kind TT_MC_LATTICE, eq. qmc, x_i = frac(i q / N + s),
 * i = 1..N) for the caller's generating vector gen[m] (host, reduced mod N).
 * n_sets estimators of n_points points each (independent points, or
 * independent shifts of one lattice) are computed in one launch; estimates
 * (host, n_sets doubles) receives them, *mean their mean and *rel_err the
 * relative empirical standard deviation of eq. std.  The integrand is the
 * problem's f without weights (n_nodes, rank_cap and tol are not used; seed keys
 * the generator).  Double precision only.  Synchronises.
 * Errors: TT_EINVAL (invalid problem, n_points < 1 or >= 2^31, n_sets < 2 or
 * > 4096, missing gen for a lattice, TT_DD), TT_ENOMEM, TT_EDEVICE. */
enum { TT_MC_RANDOM = 0, TT_MC_LATTICE = 1 };
tt_status tt_mc_integrate(tt_ctx *ctx, const tt_problem *problem, int32_t kind, int64_t n_points,
                          int32_t n_sets, const int64_t *gen, double *estimates, double *mean,
                          double *rel_err);

/* For callers that cannot allocate device memory: code that runs under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same estimators as tt_mc_integrate (the same kernels, so the same bits for
 * the same arguments), with no allocation of any kind: the partial sums live
 * in a static device array of TT_MC_NOALLOC_MAX_PARTIALS doubles (1 MiB) that
 * the library holds on every GPU it runs on until the process ends, and gen
 * (host, m values, reduced mod N) and the synthetic parameters are passed by
 * value in the kernel arguments.  d_out is a device array of n_sets + 2
 * doubles that receives the estimates, then their mean, then the relative
 * empirical standard deviation (eq. std).  Asynchronous on the context stream:
 * no host synchronisation, no event, no memset.  All calls on one GPU share
 * its static array, so calls that overlap on one GPU (several streams or
 * contexts) race and must be serialised by the caller; the array holds the
 * last call's partial sums, and nothing in it needs clearing.
 * Errors: as tt_mc_integrate, plus TT_EINVAL when d_out is NULL or
 * n_sets * min(ceil(n_points / 256), 256) > TT_MC_NOALLOC_MAX_PARTIALS
 * (the partial sums would not fit), and TT_EDEVICE if the static array's
 * address could not be looked up when the context was created. */
#define TT_MC_NOALLOC_MAX_PARTIALS 131072
tt_status tt_mc_integrate_noalloc(tt_ctx *ctx, const tt_problem *problem, int32_t kind, int64_t n_points,
                                  int32_t n_sets, const int64_t *gen, double *d_out);

/* Optional per-kernel timing with HIP events recorded on the context stream
 * around every launch (adds two event records per launch).  tt_ctx_profile
 * switches it on or off and clears the totals; tt_ctx_kernel_time returns the
 * number of timed launches and their summed duration in ms for a kernel kind:
 * 0 sweep (pivot search, core updates, quadrature and stopping rule fused in
 * one launch per sweep), 1 core update at init, 2 quadrature at init,
 * 3 rank-1 start, 4 Gauss--Legendre nodes, 5 tt_eval_points, 6 tt_eval_fibers,
 * 7 tt_mc_integrate, 8 ALS refresh (tt_cross_refresh, with the rebuild of the cores).
 * Errors: TT_EINVAL (bad kind or NULL outputs). */
tt_status tt_ctx_profile(tt_ctx *ctx, int32_t enable);

/* Workgroups per superblock search for jobs created after the call
 * (a launch shape, not part of the method: every group size gives the same
 * values, pivots and evaluation counts bit for bit).  group 1..8 fixes it
 * (over any tuned choice); 0 returns to the tuned group, else the rule: as many
 * as keep at most two workgroups per compute unit in a sweep launch
 * (superblocks x group + cores <= 2 x compute units), at most 1, 2 or 3 for a
 * double launch sized for ranks up to 8, 16 or more, at most 6 for double-double
 * and quad-double.  A serving loop's launches take the rule
 * for their running set, or the group fixed when the server was created.
 * Errors: TT_EINVAL outside 0..8. */
tt_status tt_ctx_set_search_group(tt_ctx *ctx, int32_t group);
tt_status tt_ctx_kernel_time(tt_ctx *ctx, int32_t kind, int64_t *launches, double *total_ms);

/* Phase marks of the sweep kernel for integral k, recorded for jobs created
 * while profiling is on (otherwise *written = 0): for every sweep, one row of
 * 16 wall-clock marks per superblock b (row b: 0 start, 1 sets staged,
 * 2 samples done, 3 rook pivoting done, 4 search done, 7 end; and durations,
 * not marks, in 8, 9, 10: the samples' point loop, block argmax and exchange
 * between the superblock's workgroups, 11, 12, 13: the same summed over the
 * rook steps, 14: the rook steps' set-up), then one per
 * core c (row m-1+c: 0 start, 8 both neighbouring searches seen, 9 pivots
 * appended and sets staged, 10 new entries evaluated, 11 new rows of the
 * interpolation core solved, 12 cross LU bordered, 13 rank-1 update done,
 * 14 core summed, 5 update done, 6 quadrature done, 7 end); 0 where the
 * workgroup skipped a phase; in ticks of *clock_mhz MHz.  marks is a host
 * buffer of `capacity` int64; sweeps x (2m-1) x 16 values are written. */
tt_status tt_job_phase_times(tt_job *job, int32_t k, int64_t *marks, int64_t capacity, int64_t *written,
                             double *clock_mhz);

/* ---- Serving loop (continuous batching) --------------------------------------
 * For callers that submit integrals one at a time, as they arrive.  A server
 * owns a worker thread, one device arena of max_bytes and up to max_active
 * running integrals.  tt_server_submit queues one problem (any host thread)
 * and returns a ticket.  The worker admits queued problems in arrival order
 * while the arena has room for their footprint (tt_job_footprint) and fewer
 * than max_active run, initialises them, and launches sweeps in which every
 * running integral advances by one sweep of Alg. 6: one launch serves all of
 * them, whatever their d, tolerance, rank cap or age.  An integral that stops
 * leaves the running set at once and its memory and slot go to the next
 * request; the kernels publish its result to pinned host memory, so the loop
 * never waits for the device except to bound the sweeps in flight.  Every
 * result is bitwise the one tt_cross_run gives for the same problem alone.
 * Double precision only (TT_FP64).
 * tt_server_submit: TT_EINVAL (invalid problem, TT_DD), TT_ENOMEM (footprint
 *   above max_bytes: it could never be admitted).
 * tt_server_poll: TT_PENDING until the result exists, then TT_OK with info and
 *   the time from submission to completion in seconds (latency_s may be NULL);
 *   the ticket is then released.  TT_EINVAL for an unknown ticket.
 * tt_server_wait: as poll, blocking until the result exists.
 * tt_server_destroy: lets running integrals finish, drops queued ones. */
typedef struct tt_server tt_server;
typedef struct {
  int64_t submitted, completed;   /* requests so far                                         */
  int64_t queued, running;        /* now                                                     */
  int64_t max_running;            /* largest running set seen                                */
  int64_t sweep_launches;         /* sweep kernels launched                                  */
  int64_t admissions;             /* admission rounds (each initialises one group of requests) */
  double  busy_s;                 /* wall time with at least one integral running            */
} tt_server_stats;
tt_status tt_server_create(tt_ctx *ctx, size_t max_bytes, int32_t max_active, tt_server **out);
tt_status tt_server_submit(tt_server *server, const tt_problem *problem, uint64_t *ticket);
tt_status tt_server_poll(tt_server *server, uint64_t ticket, tt_info *info, double *latency_s);
tt_status tt_server_wait(tt_server *server, uint64_t ticket, tt_info *info, double *latency_s);
tt_status tt_server_get_stats(tt_server *server, tt_server_stats *out);
void tt_server_destroy(tt_server *server);

/* Autotuning of the kernel variants a job launches (no passage of the paper
 * defines these: they are launch shapes of this library, not part of the method).
 * A job's kernels come in variants that compute the same values bit for bit:
 *   mode_bucket  the number of modes the kernels are compiled for, at least the
 *                job's largest m (TT_FP64 paper form: 4, 8, 10, 12, 16, 24, 32;
 *                other classes and double-double: 8, 16, 32; 0 is the streaming
 *                kernel, any number of modes, double precision, paper form and
 *                synthetic classes);
 *   rank_policy  0: each sweep's kernel is sized for the ranks reachable in that
 *                sweep; 1: for the rank caps;
 *   search_group workgroups per superblock search (see
 *                tt_ctx_set_search_group), 0 for the rule's.
 * Without tuning a job takes the smallest mode bucket, policy 0 and the rule's
 * search group (the rule).  The candidates: every valid mode bucket with both
 * policies at the rule's group, and the rule's bucket and policy 0 with search
 * groups 1, 2, 4 and 6 (when tt_ctx_set_search_group has not fixed the
 * group).
 * tt_autotune runs the given job once per candidate variant (`reps` times each,
 * median wall time from tt_cross_init to the stopping rule), keeps only the
 * variants whose results equal the rule's bit for bit (every value, sweep count
 * and evaluation count), and records the fastest for the job's key (integrand
 * class, precision, largest m, largest rank cap) in the context: later jobs with
 * that key launch it.  If the environment variable TTCROSS_TUNE_CACHE names a
 * file, the context loads it at tt_ctx_create and tt_autotune rewrites it with
 * every key the context holds (text, one key per line).  tt_autotune must not run
 * concurrently with other calls on the same context.  Errors: TT_EINVAL for an
 * invalid problem set or reps < 1; the job's own errors (TT_ENUMERIC, ...) when
 * the rule variant fails; TT_EDEVICE if the cache file cannot be written. */
typedef struct {
  int32_t mode_bucket;   /* chosen variant                                            */
  int32_t rank_policy;
  int32_t rule_mode_bucket;
  int32_t candidates;    /* variants timed                                             */
  int32_t matching;      /* of those, variants whose results equal the rule's          */
  int32_t search_group;  /* chosen search group (0: the rule's)                        */
  double  rule_ms;       /* median time of the rule's variant                          */
  double  tuned_ms;      /* median time of the chosen variant                          */
} tt_tune_result;
tt_status tt_autotune(tt_ctx *ctx, const tt_problem *problems, int32_t count, int32_t reps,
                      tt_tune_result *out);

/* Synchronise the context stream. */
tt_status tt_ctx_synchronize(tt_ctx *ctx);

/* Human-readable name of a status code (static string). */
const char *tt_status_string(tt_status status);

#ifdef __cplusplus
}
#endif
#endif /* TTCROSS_H */
