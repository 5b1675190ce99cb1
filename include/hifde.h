/*
 * hifde.h -- C ABI of the MI355X (gfx950) implementation of the hierarchical
 * interpolative factorization for elliptic PDEs (HIF-DE; K. L. Ho and L. Ying,
 * "Hierarchical Interpolative Factorization for Elliptic Operators:
 * Differential Equations").
 *
 * Problem (Section 1, Eq. (1)-(2); Sections 3.1-3.2): -div(a grad u) + b u = f
 * on the unit square (dim = 2) or cube (dim = 3) with homogeneous Dirichlet
 * data, discretized by the five-/seven-point stencil with a on the staggered
 * links and b at the nodes.  There are n unknowns per side, N = n^dim, grid
 * spacing h = 1/(n+1), lexicographic order with x0 fastest.  The library
 * factors the sparse matrix A approximately as the generalized LDL form of
 * Section 4.1 (A ~= F = V_0^-T ... V_{L-1/2}^-T D V_{L-1/2}^-1 ... V_0^-1,
 * Algorithm 4.1) and applies F^-1, directly or as the preconditioner of
 * conjugate gradients (Section 5).
 *
 * Conventions shared by every call:
 *   - Every function returns a hifde_status (0 on success, < 0 on error); the
 *     message of the last failing call on the calling thread is returned by
 *     hifde_last_error().  No C++ exception crosses this interface.
 *   - Device pointers are HIP device pointers on the current device; host
 *     pointers are plain host memory.  Each argument says which it is.
 *   - hip_stream is a hipStream_t passed as void*; NULL means the default
 *     stream.  All device work of a call is ordered on that stream; calls that
 *     return results to host memory synchronize it.
 *   - Handles own every buffer they allocate and are released by the matching
 *     *_free call.  Inputs are copied during the call and stay owned by the
 *     caller.  A handle must not be used from two threads at once; distinct
 *     handles are independent.
 */
#ifndef HIFDE_H
#define HIFDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hifde_tree_s* hifde_tree_t;
typedef struct hifde_factor_s* hifde_factor_t;

typedef enum {
  HIFDE_OK = 0,
  HIFDE_EINVAL = -1,   /* invalid argument                                  */
  HIFDE_ENOMEM = -2,   /* device or host allocation failed                  */
  HIFDE_EDEVICE = -3,  /* a HIP runtime call failed                         */
  HIFDE_ENOTSPD = -4,  /* a diagonal block had a non-positive pivot (with
                          HIFDE_INDEFINITE: a zero or non-finite one)     */
  HIFDE_ENOCONV = -5,  /* PCG or GMRES missed the tolerance within maxit   */
  HIFDE_ESTATE = -6    /* handle in the wrong state for this call           */
} hifde_status;

typedef enum {
  HIFDE_FP64 = 0,      /* every step in double precision                    */
  HIFDE_MIXED = 1,     /* cell/group steps and F^-1 in float; the top block
                          factorization, residuals and PCG in double         */
  HIFDE_MIXED_ELIM64 = 2 /* as HIFDE_MIXED, but the cell eliminations of
                          Lemma 2.1 (LDL^T, W and the Schur update of each
                          front) run in double; their apply form is rounded
                          to float for the sweeps.  For strongly varying
                          coefficients, where float Schur complements lose
                          the small differences of large terms            */
} hifde_precision;

enum {
  HIFDE_USE_RANK_MODEL = 1u,    /* size and launch each level's skeleton-front
                                   eliminations from the rank predictor's
                                   output before the IDs return (needs
                                   hifde_set_rank_model on the tree)        */
  HIFDE_DEBUG_DETERMINISM = 4u, /* factor every level twice, compare bitwise */
  HIFDE_AUTOTUNE = 8u,          /* time every launch variant of each unseen
                                   size bucket (trailing-update tiles of the
                                   LDL^T on FMA or matrix cores; ID grid or
                                   persistent queue) on a snapshot of its
                                   data and keep the fastest in the tree;
                                   later factorizations of the tree reuse
                                   the choices with or without this flag   */
  HIFDE_NO_GRAPH = 16u,         /* apply F^-1 by direct kernel launches; by
                                   default the launches of one application
                                   are captured once per right-hand-side
                                   count into a HIP graph and replayed      */
  HIFDE_PRESIZE_WORST_CASE = 64u, /* as HIFDE_USE_RANK_MODEL with every rank
                                   assumed 0 (the largest possible fronts):
                                   the comparison point of the predictor    */
  HIFDE_SWEEP_ROW_TILES = 128u, /* F^-1 sweeps in the row-tile form only (no
                                   whole-front launches, interpolation as
                                   separate launches); the results are
                                   bitwise the same                         */
  HIFDE_INDEFINITE = 256u,      /* A may be indefinite (b < 0, Helmholtz-type
                                   problems, Section 5): the LDL^T of every
                                   diagonal block accepts negative pivots
                                   (no pivoting; a zero or non-finite pivot
                                   fails with HIFDE_ENOTSPD).  Solve with
                                   hifde_gmres; hifde_pcg refuses the factor */
  HIFDE_SKETCH_ID = 512u,       /* randomized compression (Section 4.3): a
                                   group with |c^N| > |c| + 16 takes the ID
                                   of Phi A_{c^N,c}, Phi the (|c| + 16) x
                                   |c^N| Gaussian matrix drawn from
                                   Philox4x32-10 (key 0x9E3779B97F4A7C15,
                                   counter (row, column, group key, level),
                                   Box-Muller in the working type); same
                                   rank rule.  Fewer rows
                                   for the pivoted QR, plus one product on
                                   the matrix cores                        */
  HIFDE_RETRY_FP64 = 1024u      /* a float factorization (HIFDE_MIXED or
                                   HIFDE_MIXED_ELIM64) that fails on a pivot
                                   is done again in double (HIFDE_FP64):
                                   rounding in float can turn a small
                                   positive eigenvalue of a Schur complement
                                   negative.  hifde_stats reports the
                                   precision used and the retry.  A failure
                                   in double is reported as usual          */
};

/* Maximum number of tree levels reported by hifde_stats. */
#define HIFDE_MAX_LEVELS 24

typedef struct {
  int64_t N;                        /* number of unknowns                     */
  int32_t dim, levels;              /* dimension and tree depth L             */
  int64_t top_size;                 /* |s_L|, the unknowns left at level L    */
  int64_t factor_bytes;             /* m_f: device bytes of the stored factor */
  double factor_flops;              /* algorithmic flops of the factorization */
  double factor_ms;                 /* wall time of the last hifde_factor     */
  double solve_bytes;               /* algorithmic bytes of one F^-1 sweep    */
  int64_t cells[HIFDE_MAX_LEVELS];  /* cells eliminated at level l            */
  int64_t groups[HIFDE_MAX_LEVELS]; /* groups at level l+1/2                  */
  int64_t skel_in[HIFDE_MAX_LEVELS];  /* unknowns entering level l+1/2 groups  */
  int64_t skel_out[HIFDE_MAX_LEVELS]; /* skeletons kept at level l+1/2         */
  int32_t max_front[HIFDE_MAX_LEVELS];/* largest |p|+|c^N| of a level-l cell   */
  int64_t rank_groups;              /* groups launched from predicted ranks   */
  double rank_mae;                  /* mean |predicted - actual| of their k   */
  int64_t rebuckets;                /* levels eliminated again because a rank
                                       left the launched bound               */
  int64_t skel_panels;              /* 32-pivot panel sweeps launched for the
                                       skeleton fronts (all levels)          */
  int64_t tuned;                    /* size buckets the autotuner timed      */
  double level_ms[HIFDE_MAX_LEVELS];  /* host wall time from the start of the
                                       factorization to the end of level
                                       l + 1/2 (the host has its ranks and
                                       has queued the level's work)          */
  double top_ms;                    /* device time of the top block (level L:
                                       assembly, LDL^T in double, apply form) */
  int32_t precision;                /* hifde_precision the factor holds      */
  int32_t retried;                  /* 1: HIFDE_RETRY_FP64 redid it in double */
} hifde_stats_t;

/* Index sets of one (fractional) level, for comparison with other
 * implementations.  level2 = 2l selects the cells of level l (lists 0 = p,
 * the eliminated unknowns, and 1 = c^N, the front); level2 = 2l+1 selects the
 * groups of level l+1/2 (lists 0 = c, 1 = c^N, 2 = skeletons, 3 = redundant);
 * level2 = 2L selects the top block (one entry, list 0 = s_L).  Every list is
 * sorted ascending and holds global unknown indices. */
typedef struct {
  int64_t count;      /* number of cells or groups                           */
  int64_t total[4];   /* total length of each list over all entries          */
  int64_t* ids;       /* [count] cell or group keys (host, caller-owned)     */
  int64_t* offs[4];   /* [count+1] start of each entry in lists[i]           */
  int32_t* lists[4];  /* concatenated lists (host, caller-owned)             */
} hifde_sets_t;

/* Build the tree of Sections 3.1-3.2 and 4.1-4.2: n unknowns per side, boxes
 * of leaf * 2^l unknowns per side at level l, L = log2(ceil(n/leaf)) levels,
 * the top one a single box.  When leaf does not divide n the last box along
 * each axis is shorter (e.g. the paper's n = 2^k - 1 grids); the number of
 * leaf boxes per side, ceil(n/leaf), must be a power of two (otherwise a
 * short corner box could be left with nothing to eliminate).  The first
 * `skip_levels` fractional levels are not skeletonized (Section 5).
 * Host-only; no device work.  The tree also keeps, for reuse by its later
 * factorizations, the device memory of factorizations that were freed; it
 * is released when the tree and all its factorizations are freed (or, when
 * a device allocation fails, before it is retried).
 * EINVAL: dim not 2 or 3, leaf < 2, ceil(n/leaf) not a power of two >= 2,
 * skip_levels < 0, N >= 2^31. */
int hifde_build_tree(int dim, int64_t n, int64_t leaf, int skip_levels,
                     hifde_tree_t* out);

/* Cap on the device memory the tree's factorizations and their solves may
 * hold together (bytes; 0 removes the cap, the default).  It counts the
 * blocks the tree's memory pool has taken from the device, including those
 * kept for reuse after a factorization was freed (which are released first
 * when the cap would be exceeded).  A call that would go over it fails with
 * HIFDE_ENOMEM, frees what it took, and leaves the tree usable.  Host-only.
 * EINVAL: NULL tree, bytes < 0. */
int hifde_tree_set_memory_limit(hifde_tree_t tree, int64_t bytes);

/* Factor A (Algorithm 4.1).  a[k] (k < dim) are DEVICE pointers to double
 * arrays of the link coefficients along axis k: n+1 links along axis k and n
 * along the others, x0 fastest (link j along axis k joins x_k = j-1 and
 * x_k = j).  b is a DEVICE pointer to N doubles or NULL (b = 0).  eps is the
 * relative ID tolerance of Section 2.2; eps = 0 disables skeletonization
 * (the multifrontal method, Algorithm 3.1).  The returned factor keeps no
 * reference to a or b.
 * A zero coefficient on boundary links (link 0 or n along an axis) makes
 * that part of the boundary zero-flux (Neumann) rather than Dirichlet.
 * EINVAL: eps outside [0, 1), NULL a[k], a not positive on an interior link,
 * negative on a boundary link or not finite (checked on the device),
 * non-finite b.  ENOTSPD: a pivot of a diagonal
 * block was not positive (with HIFDE_INDEFINITE: was zero or not finite);
 * hifde_last_error() names the level and block.
 * The pivots of each level are read with that level's skeleton ranks, so
 * the factorization stops at the level after the failing block (at the end
 * when no level is skeletonized).  ENOMEM: the device, or the tree's cap
 * (hifde_tree_set_memory_limit), ran out of memory. */
int hifde_factor(hifde_tree_t tree, const double* const* a, const double* b,
                 double eps, hifde_precision prec, uint32_t flags,
                 void* hip_stream, hifde_factor_t* out);

/* u = F^-1 f for nrhs right-hand sides (the factored application of
 * Section 4.1).  f and u are DEVICE pointers to N x nrhs column-major double
 * arrays with leading dimensions ldf, ldu >= N; f may equal u.
 * EINVAL: nrhs < 1, ld < N, NULL pointers. */
int hifde_solve(hifde_factor_t F, int64_t nrhs, const double* f, int64_t ldf,
                double* u, int64_t ldu, void* hip_stream);

/* Solve A u = f by conjugate gradients preconditioned with F^-1 (Section 5),
 * from u = 0, in double precision, one independent iteration per column,
 * until ||f - A u|| <= tol ||f|| (recursive residual) or maxit iterations.
 * The mixed-precision factor uses the flexible (Polak-Ribiere) update.
 * f, u: DEVICE, N x nrhs column-major; f may equal u when ldf == ldu (no
 * other overlap).  iters[nrhs], relres[nrhs]: HOST,
 * filled with the iteration count and the true relative residual
 * ||f - A u|| / ||f|| of each column.
 * ENOCONV: some column missed tol; iters, relres and u hold the last iterate.
 * ESTATE: F was factored with HIFDE_INDEFINITE (conjugate gradients needs a
 * definite operator: use hifde_gmres). */
int hifde_pcg(hifde_factor_t F, int64_t nrhs, const double* f, int64_t ldf,
              double* u, int64_t ldu, double tol, int maxit, int* iters,
              double* relres, void* hip_stream);

/* Solve A u = f by GMRES with F^-1 as right preconditioner (the paper's
 * solver for indefinite problems, Section 5), from u = 0, in double
 * precision, one independent iteration per column.  Each step takes
 * z_k = F^-1 v_k and A z_k, orthogonalizes against the basis by modified
 * Gram-Schmidt and updates the Hessenberg least-squares problem by Givens
 * rotations; every `restart` steps (and at the end) u += Z y with the kept
 * z_k (for the fixed linear F^-1 the same as F^-1 (V y); for the float
 * factor it keeps A Z = V H exact in double, the flexible form), and the
 * next cycle starts from the true residual.  It stops when the residual
 * estimate reaches tol ||f|| (or the true residual does, at a restart) or
 * after maxit steps in all.  Any factor works (definite or not).
 * f, u: DEVICE, N x nrhs column-major; f may equal u when ldf == ldu (no
 * other overlap).  iters[nrhs], relres[nrhs]: HOST, filled with the step
 * count and the true relative residual ||f - A u|| / ||f|| of each column.
 * Device memory: (restart + 1) N nrhs doubles for the basis and restart
 * N nrhs elements of the factor's sweep type (float or double) for the z_k.
 * EINVAL: nrhs < 1, ld < N, NULL pointers, restart < 1, maxit < 1, tol not
 * finite and positive.  ENOCONV: some column missed tol; iters, relres and u hold
 * the last iterate. */
int hifde_gmres(hifde_factor_t F, int64_t nrhs, const double* f, int64_t ldf,
                double* u, int64_t ldu, double tol, int restart, int maxit,
                int* iters, double* relres, void* hip_stream);

/* y = A x with the assembled stencil (the operator PCG and GMRES use).  DEVICE,
 * N x nrhs column-major. */
int hifde_matvec(hifde_factor_t F, int64_t nrhs, const double* x, int64_t ldx,
                 double* y, int64_t ldy, void* hip_stream);

/* Kernel timing.  Launches of the selected kernel classes are bracketed by
 * HIP events on the stream they run on (while profiling, F^-1 runs as direct
 * launches, not as the captured graph, except with HIFDE_PROF_SWEEP_UP_ONE
 * as the only class: that first kernel of each application always runs as a
 * direct launch before the graph of the rest); hifde_profile_read reports, per
 * class, the launches timed, their summed event time and their algorithmic
 * traffic and flops (the bytes of the stored factor blocks, index lists and
 * vector rows the launch must touch, and the multiply-adds the sweep
 * formulas of Section 4.1 need), so that achieved bandwidth can be compared
 * with the device's.  Profiling adds two event records per timed launch. */
enum {
  HIFDE_PROF_SWEEP_UP = 0,    /* upward steps of cells and skeleton fronts:
                                 z_p = D^-1 L^-1 x_p, x_q -= W^T L^-1 x_p
                                 (Lemma 2.1; Lemma 2.4 after the interpolation),
                                 launches of the row-tile form               */
  HIFDE_PROF_SWEEP_DOWN = 1,  /* downward steps: x_p = L^-T (z_p - W x_q),
                                 row-tile form                               */
  HIFDE_PROF_INTERP = 2,      /* interpolation steps of skeletonized groups:
                                 x_r -= T^T x_s (up), x_s -= T x_r (down)    */
  HIFDE_PROF_TOP = 3,         /* both steps of the top block (double)       */
  HIFDE_PROF_SWEEP_UP_WHOLE = 4,    /* upward steps, launches of the
                                       whole-front form (one work-group per
                                       front: levels of many small fronts)  */
  HIFDE_PROF_SWEEP_DOWN_WHOLE = 5,  /* downward steps, whole-front form     */
  HIFDE_PROF_GROUP_UP = 6,    /* upward steps of skeleton fronts with their
                                 interpolation x_r -= T^T x_s in the same
                                 launch (whole-front form of groups)        */
  HIFDE_PROF_GROUP_DOWN = 7,  /* downward steps of skeleton fronts with
                                 x_s -= T x_r in the same launch            */
  HIFDE_PROF_SWEEP_UP_ONE = 8,   /* upward steps of the level-0 cells, both
                                    colors in one whole-front launch; the
                                    x_q updates go to a contribution buffer.
                                    Its bytes count the stored factor once
                                    and every front's p and q vector rows
                                    once per right-hand side              */
  HIFDE_PROF_CONTRIB_ADD = 9,    /* x_q -= the contributions of that launch,
                                    in color order                          */
  HIFDE_PROF_CLASSES = 10
};

typedef struct {
  int64_t launches;   /* launches timed since the last read                   */
  double ms;          /* summed HIP-event durations                          */
  double bytes;       /* algorithmic bytes of those launches                 */
  double flops;       /* algorithmic flops of those launches                 */
} hifde_prof_t;

/* Start timing the classes in class_mask (bit c = class c) at tree level
 * `level` (-1: every level); class_mask = 0 stops.  Counters are kept until
 * read. */
int hifde_profile(hifde_factor_t F, uint32_t class_mask, int level);

/* Waits for the timed launches of class cls, adds them up into *out (HOST)
 * and clears the class's counters. */
int hifde_profile_read(hifde_factor_t F, int cls, hifde_prof_t* out);

/* ---- Skeleton-rank predictor ------------------------------------------
 * A 3-layer tanh perceptron HIFDE_RANK_FEATURES -> 64 -> 64 -> 1 (float)
 * predicts log2(1 + k), k the skeleton count of a group at level l+1/2,
 * from the group's features (level, |c|, |c^N|, eps, dimension and the
 * statistics of log10 a on the stencil links at c and at c^N).  With
 * HIFDE_USE_RANK_MODEL, hifde_factor sizes and launches the skeleton-front
 * eliminations of a level from the predicted ranks before the IDs'
 * results reach the host; the tolerance-driven IDs still decide every
 * skeleton, and a front whose actual rank leaves the launched bound is
 * eliminated again after the IDs return (counted in hifde_stats).
 * Parameters (HIFDE_RANK_PARAMS floats): W1 (64 x F, row-major), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (1 x 64), b3 (1).  All pointers of the hifde_mlp
 * calls are DEVICE pointers; work is ordered on hip_stream. */
#define HIFDE_RANK_FEATURES 16
#define HIFDE_RANK_HIDDEN 64
#define HIFDE_RANK_PARAMS (64 * 16 + 64 + 64 * 64 + 64 + 64 + 1)

/* Bytes of device workspace hifde_mlp_grad needs for nbatch samples. */
int hifde_mlp_workspace(int64_t nbatch, int64_t* bytes);

/* out[b] = network(feat[b, :]) for nbatch samples (feat row-major). */
int hifde_mlp_forward(const float* params, int64_t nbatch, const float* feat,
                      float* out, void* hip_stream);

/* Gradient of the mean squared error (1/B) sum_b (out[b] - target[b])^2
 * with respect to params into grad (HIFDE_RANK_PARAMS floats) and the loss
 * into *loss (one float, device).  Sums over the batch run in a fixed
 * order.  work: hifde_mlp_workspace(nbatch) bytes. */
int hifde_mlp_grad(const float* params, int64_t nbatch, const float* feat,
                   const float* target, float* grad, float* loss, void* work,
                   void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the gradient of
 * hifde_mlp_grad without the work argument.  The workspace is a static
 * device array of (4 * HIFDE_RANK_HIDDEN + 2) * 4 bytes per sample for up to
 * HIFDE_MLP_NOALLOC_MAX_BATCH samples (1032 bytes each, 8.45 MB in all),
 * which each device holds from the first call on it until the process ends.
 * The call allocates nothing.  All calls on one device share that array:
 * calls that overlap in time on one device (two streams, two threads) race
 * and give undefined results.  Results equal those of hifde_mlp_grad.
 * EINVAL: NULL pointers, nbatch < 1 or nbatch > HIFDE_MLP_NOALLOC_MAX_BATCH. */
#define HIFDE_MLP_NOALLOC_MAX_BATCH 8192
int hifde_mlp_grad_noalloc(const float* params, int64_t nbatch, const float* feat,
                           const float* target, float* grad, float* loss,
                           void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, epsilon 1e-8, bias-corrected;
 * step counts from 1) on params with moments m, v. */
int hifde_mlp_adam(float* params, const float* grad, float* m, float* v,
                   int64_t step, float lr, void* hip_stream);

/* Features of the groups of level `level` + 1/2 of a factorization into
 * feat (DEVICE, cap x HIFDE_RANK_FEATURES) and, when target is not NULL,
 * the log2(1 + k) of the skeleton counts the factorization chose (DEVICE,
 * cap): training data drawn from the method itself.  *ngroups (HOST) gets
 * the number of groups; feat = NULL only reports it. */
int hifde_rank_features(hifde_factor_t F, int level, float* feat, float* target,
                        int64_t cap, int64_t* ngroups, void* hip_stream);

/* Weights (HOST, HIFDE_RANK_PARAMS floats) used by later hifde_factor calls
 * on this tree with HIFDE_USE_RANK_MODEL; NULL removes the model. */
int hifde_set_rank_model(hifde_tree_t tree, const float* weights, int64_t nweights);

/* Statistics of a factor (HOST out). */
int hifde_stats(hifde_factor_t F, hifde_stats_t* out);

/* Index sets of one level (see hifde_sets_t).  Call once with every pointer
 * in *out NULL to obtain count and totals, then again with caller-allocated
 * host buffers of those sizes.  Works on factors and on replayed plans. */
int hifde_export_sets(hifde_factor_t F, int level2, hifde_sets_t* out);

/* Host-only replay of the tree and index-set construction: the skeletons of
 * every level l+1/2 are taken from redundant_level (HOST, N int32: 2l+1 if
 * the unknown is redundant at level l+1/2, any other value otherwise)
 * instead of being computed.  The result supports hifde_export_sets and
 * hifde_stats only.  Needs no GPU. */
int hifde_plan_replay(hifde_tree_t tree, const int32_t* redundant_level,
                      hifde_factor_t* out);

/* Free a tree (its factorizations stay valid) or a factor (waits for the
 * device to finish before its memory returns to the tree's pool). */
void hifde_tree_free(hifde_tree_t tree);
void hifde_factor_free(hifde_factor_t F);
const char* hifde_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HIFDE_H */
