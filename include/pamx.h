/*
 * pamx.h -- C ABI of the MI355X (gfx950) k-medoids library.
 *
 * The library implements PAM (Kaufman & Rousseeuw) with the SWAP
 * improvements of Schubert & Rousseeuw, "Fast and Eager k-Medoids
 * Clustering", arXiv 2008.05171:
 *   - BUILD, the greedy initialisation                   (Sec. 2, Alg. 1)
 *   - FastPAM1 SWAP: one pass per candidate over all objects gives the
 *     change of all k swaps at once (Sec. 3.1, Alg. 3, Eq. better-change3);
 *     it performs exactly the swaps of PAM SWAP           (Sec. 2, Alg. 2)
 *   - eager FastPAM2 SWAP: the best swap of every medoid from one pass,
 *     applied one after another in the same iteration     (Sec. 3.2)
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller (for instance
 *     torch tensors on the GPU).  Scalar outputs (td, stats) are HOST
 *     pointers, written after the call has synchronised its stream.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Every call returns after the work on `stream` has finished.
 *   - The library allocates no device memory.  Scratch space is the caller's
 *     workspace `ws` of `ws_bytes` bytes, 256-byte aligned, sized by
 *     pamx_workspace_bytes() for the same arguments (pamx_swap_noalloc uses
 *     a fixed scratch array of the library instead).
 *   - Dissimilarities are a row-major n x n matrix with leading dimension
 *     `ld` >= n (elements): D[o*ld + c] = d(x_o, x_c).  D must be symmetric,
 *     non-negative and have a zero diagonal (Sec. 2 requires only a
 *     dissimilarity; symmetry lets the library read row c for column c).
 *     Element type PAMX_I32 (exact int64 sums) or PAMX_F32.
 *   - Medoids are object indices in SLOT order.  A swap keeps the slot: the
 *     new medoid takes the slot of the medoid it replaces.  labels[o] is the
 *     slot of o's nearest medoid (smallest slot on distance ties).
 *   - Ties: BUILD takes the smallest candidate index among equal changes;
 *     SWAP takes the smallest (change, slot, candidate) in lexicographic
 *     order, which is the order of Alg. 2's loops, so FastPAM1 reproduces
 *     PAM exactly on integer dissimilarities.
 *   - A swap is applied only if it lowers TD strictly (Alg. 2 and 3 stop
 *     when the best change is >= 0).
 *   - Return value: PAMX_OK (0), PAMX_WARN_MAXITER (1: results valid, the
 *     iteration cap was reached), or a negative PAMX_ERR_* code; then
 *     pamx_last_error() describes it.  Argument errors are detected on the
 *     host before any device work is enqueued.
 *   - Results are deterministic: no floating-point atomics are used, so the
 *     same inputs give bitwise identical outputs.
 */
#ifndef PAMX_H
#define PAMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types */
#define PAMX_I32 1
#define PAMX_F32 2

/* input kinds of pamx_fit */
#define PAMX_INPUT_D 0 /* an n x n dissimilarity matrix */
#define PAMX_INPUT_X 1 /* n points of `dim` coordinates, row-major */

/* metrics for points */
#define PAMX_L1 1 /* Manhattan: int32 points give exact int32 distances
                     (coordinate ranges must sum to at most INT32_MAX - 1) */
#define PAMX_L2 2 /* Euclidean: float32 points */

/* SWAP variants */
#define PAMX_FASTPAM1 1 /* best swap per iteration (Alg. 3)               */
#define PAMX_FASTPAM2 2 /* best swap per medoid, applied eagerly (Sec. 3.2); the
                           eager application runs over the whole device under a
                           cooperative launch, or in one work-group when the
                           device has none or the environment sets
                           PAMX_COOPERATIVE=0 (equal results either way);
                           PAMX_EAGER_GRID=g caps the cooperative grid at g
                           work-groups (equal results) */
#define PAMX_FASTERPAM 3 /* FasterPAM (Alg. 4, Sec. 3.2): the candidates are
                            visited in index order, cyclically; each takes its
                            best slot (smallest on ties) and is swapped in at
                            once when that lowers TD; the run ends after a
                            full cycle of n positions without a swap.  The
                            device scores a window of consecutive candidates
                            in one pass and applies the first improving one,
                            which is the swap the sequential scan makes, so
                            the swaps are Alg. 4's exactly (PAMX_I32) or
                            with FP64 sums of the FP32 matrix (PAMX_F32, a
                            swap taken when its change is below minus the
                            summation bound).  max_iter caps the passes.
                            The window pass groups its object chunks by
                            their length; the environment variable
                            PAMX_FP_GROUP=1, 2 or 4 (read on every call)
                            fixes the chunks per work-group (equal results
                            on PAMX_I32; PAMX_F32 sums may round
                            differently). */

/* accumulation of the loss changes for PAMX_F32 dissimilarities */
#define PAMX_ACC_F64 0 /* FP64 sums (default)                              */
#define PAMX_ACC_F32 1 /* FP32 sums; candidates whose change lies within a
                          rigorous FP32 error bound of the best are scored
                          again in FP64 before the swap is chosen          */

/* how pamx_fit obtains distances of PAMX_F32 points */
#define PAMX_DIST_STORED 0 /* the n x n FP32 matrix is computed once into the
                              workspace (Gram term on FP32 MFMA)              */
#define PAMX_DIST_BF16 1   /* mixed-precision form: no matrix; every pass
                              recomputes distances of split-BF16 centred
                              points on the BF16 matrix cores, sums loss
                              changes in FP64 (or FP32 with PAMX_ACC_F32),
                              and re-scores in FP64 (from the FP32 points)
                              every candidate whose rigorous error bound
                              reaches the best one, so BUILD and SWAP take
                              the decisions of FP64 arithmetic.
                              FastPAM1 only; dim <= 64, k <= 4096.            */

/* pamx_options.chunk: time the SWAP pass for several chunk lengths on the
 * caller's matrix (after BUILD, with its medoids) and keep the fastest; the
 * workspace must then be sized with the same option.  For pamx_fit_batched
 * it times the batched launch for several team sizes (work-groups per large
 * instance) on the first call of each instance shape and keeps the fastest
 * for the process; the results do not depend on the team sizes. */
#define PAMX_CHUNK_TUNE (-1)

/* return codes */
#define PAMX_OK 0
#define PAMX_WARN_MAXITER 1
#define PAMX_ERR_ARG (-1)
#define PAMX_ERR_WORKSPACE (-2)
#define PAMX_ERR_HIP (-3)
#define PAMX_ERR_INVALID_MEDOIDS (-4)
#define PAMX_ERR_UNSUPPORTED (-5)

typedef struct pamx_options {
    int32_t variant;            /* PAMX_FASTPAM1 (default) or PAMX_FASTPAM2   */
    int32_t accum;              /* PAMX_ACC_F64 (default) or PAMX_ACC_F32     */
    int32_t max_iter;           /* SWAP iterations (searches; FasterPAM: passes
                                   over the candidates) cap; default 10000  */
    int32_t build_exclude_self; /* 0 (default): a BUILD candidate's own drop to
                                   distance 0 counts in its change, so each step
                                   adds the point that lowers TD most; 1: the
                                   literal loop bounds of Alg. 1 (x_c skipped) */
    int32_t trace_cap;          /* capacity of `trace` in records (0: none)   */
    int32_t chunk;              /* objects per pass work-group; 0 = automatic,
                                   PAMX_CHUNK_TUNE = timed on the first call for
                                   this device and shape (stored matrix), then
                                   reused for the life of the process         */
    int32_t profile;            /* 1: time every BUILD / SWAP pass kernel with
                                   HIP events on `stream` (pamx_stats)       */
    int32_t dist_mode;          /* PAMX_DIST_STORED (default) or PAMX_DIST_BF16 */
    int32_t graph;              /* stored matrix, profile 0: 1 = one SWAP
                                   search is captured as a HIP graph (kept per
                                   host thread for the last 4 argument sets) and
                                   replayed on a library stream ordered after
                                   and before `stream` by events; 0 (default) =
                                   every kernel launched directly (measured
                                   faster: a replay costs more than the launches
                                   it replaces)                              */
    int32_t window;             /* PAMX_FASTERPAM: largest number of candidates
                                   scored per pass (rounded up to whole 1024-
                                   or 256-candidate tiles; a pass after a swap
                                   scores one tile, each pass without a swap
                                   doubles the width up to this); 0 (default)
                                   = 16 tiles                                */
    void *trace;                /* optional DEVICE array of pamx_swap_record:
                                   every applied swap in order               */
} pamx_options;

typedef struct pamx_swap_record {
    int32_t slot;   /* medoid slot that was replaced */
    int32_t cand;   /* object that became the medoid */
    double delta;   /* change of TD of the swap (exact for PAMX_I32) */
} pamx_swap_record;

typedef struct pamx_stats {
    int32_t iterations; /* SWAP searches performed (PAM: swaps + 1 when converged;
                           FasterPAM: passes over the candidates begun) */
    int32_t swaps;      /* swaps applied */
    int32_t converged;  /* 1 if the last search found no improving swap */
    int32_t rescored;   /* candidates scored again in FP64 (PAMX_ACC_F32) */
    double td_build;    /* TD after BUILD (pamx_fit) */
    double td;          /* final TD, summed afresh (FP64; exact for PAMX_I32) */
    double ms_dist, ms_build, ms_swap, ms_total; /* device time per phase */
    int64_t pass_pairs; /* candidate-object pairs read by SWAP passes */
    int64_t build_pairs;/* candidate-object pairs read by BUILD passes */
    double ms_swap_pass;   /* profile=1: summed duration of the SWAP pass kernels */
    double ms_build_pass;  /* profile=1: summed duration of the full BUILD passes
                              (every step of the BUILD-from-scratch form; the
                              first two steps of the stored-matrix form) */
    int32_t n_swap_pass;   /* profile=1: SWAP pass launches that did work */
    int32_t n_build_pass;  /* profile=1: full BUILD pass launches */
    double ms_build_delta; /* profile=1: summed duration of the incremental BUILD
                              passes (stored matrix, steps 3..k) */
    int64_t build_rows;    /* matrix rows read by the incremental BUILD passes */
    int32_t n_build_delta; /* profile=1: incremental BUILD pass launches */
    int32_t chunk;         /* object chunk length of the SWAP passes */
    int64_t scan_positions;/* PAMX_FASTERPAM: candidate positions visited
                              (iterations = passes begun = ceil(positions / n)) */
    int32_t windows;       /* PAMX_FASTERPAM: window passes run */
    int32_t window;        /* PAMX_FASTERPAM: largest window (candidates) */
} pamx_stats;

/* Fills `opt` with the defaults listed above. */
void pamx_default_options(pamx_options *opt);

/* Workspace bytes needed by pamx_build / pamx_swap / pamx_fit for these
 * arguments.  input_kind PAMX_INPUT_X includes room for the n x n matrix
 * (row stride rounded up to 64 elements).  Returns 0 or PAMX_ERR_ARG. */
int pamx_workspace_bytes(int64_t n, int32_t k, int32_t dim, int32_t input_kind,
                         int32_t dtype, const pamx_options *opt, size_t *bytes);

/* Dissimilarity matrix of n points (Sec. 2: PAM consumes a matrix).
 *   X      device, n x dim row-major; PAMX_I32 with PAMX_L1 (exact), or
 *          PAMX_F32 with PAMX_L2 (Euclidean of the mean-centred points,
 *          the Gram term on MFMA; pamx_fit computes the same bits).
 *   D      device, n x ld output of the same element type; ld >= n,
 *          a multiple of 4.  Diagonal written as 0, D symmetric bitwise.
 *   ws     device scratch, 4-byte aligned, of at least 4*dim bytes for
 *          PAMX_F32 (the coordinate means) or 8*dim bytes for PAMX_I32 (the
 *          coordinate ranges); PAMX_ERR_WORKSPACE otherwise.
 * PAMX_I32 points whose per-coordinate ranges (max - min) sum past
 * INT32_MAX - 1 are refused with PAMX_ERR_ARG before any distance is
 * formed: such points could have L1 distances outside int32 (INT32_MAX is
 * the "no medoid" sentinel).  pamx_fit and pamx_fit_batched check their
 * integer points the same way.  This check waits for the stream. */
int pamx_dist(const void *X, int32_t dtype, int64_t n, int32_t dim, int32_t metric,
              void *D, int64_t ld, void *ws, size_t ws_bytes, void *stream);

/* BUILD (Alg. 1): k initial medoids in slot order (the order picked).
 *   D        device dissimilarities (see conventions)
 *   medoids  device int32[k] output
 *   td       host double output: TD of the k medoids, summed afresh */
int pamx_build(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
               const pamx_options *opt, int32_t *medoids, double *td,
               void *ws, size_t ws_bytes, void *stream);

/* SWAP (Alg. 3, or eager FastPAM2) from the given medoids to a local
 * optimum: no single swap lowers TD (Sec. 2).
 *   medoids  device int32[k], read and overwritten, slot order; entries must
 *            be distinct and in [0, n), else PAMX_ERR_INVALID_MEDOIDS
 *   labels   device int32[n] output (may be NULL)
 *   td       host double output (may be NULL)
 *   stats    host output (may be NULL) */
int pamx_swap(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
              const pamx_options *opt, int32_t *medoids, int32_t *labels, double *td,
              pamx_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* pamx_swap without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Arguments, results and errors are those of pamx_swap,
 * and the same kernels run, so the results equal pamx_swap's bit for bit.
 * The scratch is a fixed device array of PAMX_NOALLOC_SCRATCH_BYTES inside
 * the library: each GPU it runs on holds one copy until the process ends,
 * and every call on that GPU reuses it, so calls that overlap on one GPU
 * (other streams, other host threads) race and must not be made.  Arguments
 * whose workspace (pamx_workspace_bytes(n, k, 0, PAMX_INPUT_D, dtype, opt))
 * exceeds that size return PAMX_ERR_WORKSPACE before any device work.
 * opt->profile, opt->graph and chunk = PAMX_CHUNK_TUNE are refused
 * (PAMX_ERR_ARG): each would create HIP events or graphs.  The stats'
 * durations (ms_*) are 0.  Allocates nothing: no hipMalloc, no hipFree, no
 * event creation. */
#define PAMX_NOALLOC_SCRATCH_BYTES (64ll << 20) /* 64 MiB per GPU */
int pamx_swap_noalloc(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                      const pamx_options *opt, int32_t *medoids, int32_t *labels, double *td,
                      pamx_stats *stats, void *stream);

/* Whole fit (Sec. 2: PAM consumes a dissimilarity matrix; Alg. 1 BUILD, then
 * SWAP as Alg. 3 FastPAM1, the eager FastPAM2 reading of Sec. 3.2, or Alg. 4
 * FasterPAM; TD by Eq. td): distances (for points), BUILD, SWAP, labels, TD.
 *   XorD  device: n x n matrix (input_kind PAMX_INPUT_D, ld = n) or n x dim
 *         points (PAMX_INPUT_X; the matrix is written into the workspace).
 *   medoids device int32[k] output, slot order; labels device int32[n]
 *         output (may be NULL); td, stats host outputs (may be NULL).
 * Errors as for pamx_build and pamx_swap; PAMX_I32 points as for pamx_dist. */
int pamx_fit(const void *XorD, int32_t input_kind, int32_t dtype, int64_t n, int32_t dim,
             int32_t metric, int32_t k, const pamx_options *opt, int32_t *medoids,
             int32_t *labels, double *td, pamx_stats *stats, void *ws, size_t ws_bytes,
             void *stream);

/* FastCLARANS (Sec. 3.4): one randomized local search from `medoids`
 * (DEVICE int32[k], slot order; read, then overwritten with the result).
 * draws: DEVICE int32[len], random object indices chosen by the caller,
 * taken in order.  A draw that is a current medoid is skipped; any other is
 * a candidate scored against all k slots at once (its best slot, smallest on
 * ties) and swapped in when that lowers TD (PAMX_F32: below minus the FP64
 * summation bound).  Draws that do not improve count as failures, a swap
 * resets the count; the search ends after `maxneighbor` failures in a row
 * (the paper uses 2.5% of n - k) -> PAMX_OK, or when the list runs out ->
 * PAMX_WARN_MAXITER.  Several searches ("numlocal"): pamx_clarans_numlocal.
 * The device scores a window of draws per pass and applies the first
 * improving one, so the swaps are those of the sequential search (exactly
 * for PAMX_I32).
 * labels, td, stats as for pamx_swap (stats: swaps, converged; windows =
 * passes; scan_positions = draws evaluated).  Workspace:
 * pamx_workspace_bytes(n, k, 0, PAMX_INPUT_D, dtype, opt, ...).  A draw
 * outside [0, n) returns PAMX_ERR_ARG (checked on the device first). */
int pamx_clarans(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                 const int32_t *draws, int64_t len, int64_t maxneighbor,
                 const pamx_options *opt, int32_t *medoids, int32_t *labels, double *td,
                 pamx_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- Best of several local searches.  Each search runs from its own
 * start, one after another on `stream`; the local optimum of smallest TD is
 * kept (the lowest search index on ties) and written to medoids (DEVICE
 * int32[k], slot order) and labels (DEVICE int32[n], may be NULL).  td:
 * host, the kept TD.  stats: the kept search's (ms_total covers the call).
 * each_td: host double[R] (may be NULL), every search's TD.  best: host
 * int32 (may be NULL), the kept search.  Every start must hold k distinct
 * indices in [0, n), else PAMX_ERR_INVALID_MEDOIDS.  Returns the kept
 * search's code (PAMX_OK or PAMX_WARN_MAXITER) or the first error.
 * Workspace (256-byte aligned): pamx_best_of_workspace_bytes, the SWAP
 * workspace plus the current search's medoids and labels. */
int pamx_best_of_workspace_bytes(int64_t n, int32_t k, int32_t dtype, const pamx_options *opt,
                                 size_t *bytes);

/* Restarts (Sec. 3.3: cheap starts -- uniform random, distance-weighted or
 * LAB -- each followed by SWAP; the paper finds random starts with FasterPAM
 * fastest at equal quality, Sec. 4.3, Tab. 1): R SWAP runs (opt->variant:
 * FastPAM1, eager FastPAM2 or FasterPAM) from starts (DEVICE int32[R*k],
 * start r at r*k), each exactly as pamx_swap from that start. */
int pamx_swap_restarts(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                       int32_t restarts, const int32_t *starts, const pamx_options *opt,
                       int32_t *medoids, int32_t *labels, double *td, pamx_stats *stats,
                       double *each_td, int32_t *best, void *ws, size_t ws_bytes, void *stream);

/* FastCLARANS with numlocal searches (Sec. 3.4; Sec. 2.1 for CLARANS's
 * numlocal): search r starts from starts[r*k .. r*k+k) (DEVICE int32) and
 * takes draws[r*len .. r*len+len) (DEVICE int32), each exactly as
 * pamx_clarans with those arguments.  opt->trace_cap must be 0. */
int pamx_clarans_numlocal(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                          int32_t numlocal, const int32_t *starts, const int32_t *draws,
                          int64_t len, int64_t maxneighbor, const pamx_options *opt,
                          int32_t *medoids, int32_t *labels, double *td, pamx_stats *stats,
                          double *each_td, int32_t *best, void *ws, size_t ws_bytes,
                          void *stream);

/* ---- Bichromatic medoids (facility location, Sec. 5): consumers and
 * possible locations are separate sets.  D: DEVICE n_cons x n_loc matrix
 * (row-major, row stride ld >= n_loc) of consumer-to-location
 * dissimilarities (finite, non-negative, no symmetry needed).  The k
 * medoids are location indices in slot order; TD sums each consumer's
 * distance to its nearest medoid; labels (DEVICE int32[n_cons] or NULL)
 * hold slots.  pamx_fit_rect runs BUILD (Alg. 1: first the location with
 * the smallest summed distance to all consumers -- the bichromatic medoid
 * of Sec. 5 -- then each step the location that lowers TD most; no
 * self-term, as no location is a consumer) and FastPAM1 SWAP with the
 * arithmetic and tie rules of pamx_fit; pamx_swap_rect starts from the
 * medoids given (DEVICE int32[k], read and overwritten).  The workspace
 * (pamx_rect_workspace_bytes) also holds the transposed matrix (each
 * location's distances to all consumers).  opt: FastPAM1 with a stored
 * matrix only (else PAMX_ERR_UNSUPPORTED); build_exclude_self does not
 * apply.  With n_cons = n_loc and a symmetric zero-diagonal D the results
 * equal pamx_fit / pamx_swap on that matrix. */
int pamx_rect_workspace_bytes(int64_t n_cons, int64_t n_loc, int32_t k, int32_t dtype,
                              const pamx_options *opt, size_t *bytes);
int pamx_fit_rect(const void *D, int32_t dtype, int64_t n_cons, int64_t n_loc, int64_t ld,
                  int32_t k, const pamx_options *opt, int32_t *medoids, int32_t *labels,
                  double *td, pamx_stats *stats, void *ws, size_t ws_bytes, void *stream);
int pamx_swap_rect(const void *D, int32_t dtype, int64_t n_cons, int64_t n_loc, int64_t ld,
                   int32_t k, const pamx_options *opt, int32_t *medoids, int32_t *labels,
                   double *td, pamx_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- Faster initialisations (Sec. 3.3).  Both write k object indices in
 * slot order to `medoids` (DEVICE int32[k]) for pamx_swap, and take their
 * random draws as inputs.  D, dtype, n, ld as for pamx_build (symmetric).
 * The work is enqueued on `stream` (pamx_init_lab first synchronizes once
 * to check its sample indices).  Host-detectable argument errors return
 * before any device work.  Integer matrices give the same medoids as the
 * plain definition; FP32 ones sum in FP64 in a fixed order.
 *
 * Workspace (256-byte aligned): pamx_init_workspace_bytes(n, m); m = the
 * subsample size for pamx_init_lab, 0 for pamx_init_dw. */
int pamx_init_workspace_bytes(int64_t n, int32_t m, size_t *bytes);

/* Distance-weighted seeding (the k-means++ idea with the distance to the
 * nearest seed as weight, the "distance weighted" initialisation of
 * Sec. 3.3).  u: DEVICE double[k], uniforms in [0, 1).  The first seed is
 * floor(u[0] n); seed t is the first object, in index order, whose running
 * sum of weights exceeds u[t] W (W the sum of all weights); seeds weigh 0.
 * When W = 0 (every object coincides with a seed) the smallest-index
 * non-seed is taken. */
int pamx_init_dw(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                 const double *u, int32_t *medoids, void *ws, size_t ws_bytes, void *stream);

/* LAB, linear approximative BUILD (Sec. 3.3): BUILD whose step t looks only
 * at samples[t*m .. t*m+m-1] (DEVICE int32, distinct indices in [0, n); the
 * paper draws 10 + ceil(sqrt(n)) non-medoid points per step).  The
 * non-medoid members are the candidates, in listed order (first strict
 * minimum wins), the members are the objects of the change; exclude_self as
 * pamx_options.build_exclude_self.  If every member is a medoid the
 * smallest-index non-medoid is taken.  An index outside [0, n) returns
 * PAMX_ERR_ARG (checked on the device before the first step). */
int pamx_init_lab(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                  const int32_t *samples, int32_t m, int32_t exclude_self, int32_t *medoids,
                  void *ws, size_t ws_bytes, void *stream);

typedef struct pamx_batch_stats {
    int32_t iterations;   /* SWAP searches over all instances */
    int32_t swaps;        /* swaps over all instances */
    int32_t best_inst;    /* instance with the smallest full-data TD (lowest id on ties),
                             -1 when full-data TD was not requested */
    int32_t team_scale;   /* team sizes used, in percent of the cost-balanced ones
                             (0: no teams); chosen by timing with
                             opt->chunk = PAMX_CHUNK_TUNE, else 100 */
    double ms_pam;        /* device time of the batched BUILD + SWAP launch */
    double ms_assign;     /* device time of the full-data TD kernels */
    double ms_total;
    int64_t pairs;        /* candidate-object pairs evaluated: two full BUILD steps, the
                             rows of changed objects in later BUILD steps, and every
                             non-medoid candidate against every object per SWAP search */
} pamx_batch_stats;

/* Workspace bytes of pamx_fit_batched for n_inst instances. */
int pamx_batched_workspace_bytes(int32_t n_inst, int64_t N, size_t *bytes);

/* Batched CLARA (Sec. 2.1; with FastPAM1 inside, Sec. 3.4): n_inst
 * independent PAM runs (BUILD + FastPAM1 SWAP) on subsamples of N points in
 * one persistent launch, then the TD of every run's medoids over all N
 * points.  Distances are computed on the fly (L2 for PAMX_F32 points, exact
 * L1 for PAMX_I32 points); no n'^2 matrix is stored.
 *   X           device, N x dim points, 1 <= dim <= 16
 *   sample_off  HOST int64[n_inst+1], sample_off[0] = 0, nondecreasing;
 *               instance j uses points sample_idx[sample_off[j] .. sample_off[j+1])
 *   sample_idx  device int32 point indices in [0, N) (checked on the device:
 *               PAMX_ERR_ARG), distinct within an instance
 *   k_inst      HOST int32[n_inst], 1 <= k_j <= min(n'_j, 256), n'_j <= 2048
 *   opt         max_iter and build_exclude_self are used (variant: FastPAM1)
 *   medoids     device int32[sum k_j]: instance j's medoids (global point
 *               indices, slot order) start at sum_{j'<j} k_j'
 *   td_sample   HOST double[n_inst]: TD of each run on its own sample
 *   td_full     HOST double[n_inst] or NULL: TD over all N points; when
 *               given, stats->best_inst is the CLARA result
 * Large instances run as teams of up to 8 work-groups under a cooperative
 * launch (same results as one work-group each); setting the environment
 * variable PAMX_COOPERATIVE=0 (read on every call) turns teams off.  A team
 * that fails to meet within its bounded wait returns PAMX_ERR_HIP. */
int pamx_fit_batched(const void *X, int32_t dtype, int64_t N, int32_t dim, int32_t metric,
                     int32_t n_inst, const int64_t *sample_off, const int32_t *sample_idx,
                     const int32_t *k_inst, const pamx_options *opt, int32_t *medoids,
                     double *td_sample, double *td_full, pamx_batch_stats *stats,
                     void *ws, size_t ws_bytes, void *stream);

/* Validation of a dissimilarity matrix.  PAM's arithmetic (Sec. 2) and the
 * shortcuts of FastPAM assume D symmetric with a zero diagonal, finite and
 * non-negative; pamx_build / pamx_swap / pamx_fit do not check this.
 *   D       device, n x ld, PAMX_I32 or PAMX_F32
 *   ws      device scratch of at least 8 bytes (two counters, overwritten)
 *   flags   HOST out: bitwise OR of the PAMX_DIS_* bits found (0: valid)
 *   count   HOST out, may be NULL: number of offending unordered pairs
 *           {i, j}, i <= j (a diagonal entry is the pair {i, i})
 * Reads every entry once; returns 0, PAMX_ERR_ARG / PAMX_ERR_WORKSPACE for
 * bad arguments (before any device work), PAMX_ERR_HIP. */
#define PAMX_DIS_ASYMMETRIC 1   /* D[i][j] != D[j][i] as values (a NaN never equals its mirror) */
#define PAMX_DIS_DIAGONAL   2   /* D[i][i] != 0 */
#define PAMX_DIS_NEGATIVE   4   /* an entry below 0 */
#define PAMX_DIS_NONFINITE  8   /* a NaN or infinite entry (PAMX_F32) */
int pamx_check_dissimilarity(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t *flags,
                             int64_t *count, void *ws, size_t ws_bytes, void *stream);

/* Measurement (not part of the method): the read rate the SWAP pass's access
 * pattern can reach.  A plain streaming read of rows [0, n) of a row-major
 * matrix of 4-byte elements in the pass's launch shape: work-groups of 256
 * lanes over 1024-column tiles, one 16-byte non-temporal load per lane and
 * row with four rows in flight, rows in chunks of `chunk`.  Columns
 * [0, n rounded up to a multiple of 4) are read; 4 n^2 bytes over the time
 * of one call is the reference the pass's own rate is compared with.
 *   D      device, ld % 4 == 0, 16-byte aligned, read as FP32
 *   sums   device float[sums_len], sums_len >= ceil(n / 1024) * ceil(n / chunk):
 *          per work-group sums of what it read (overwritten)
 * Asynchronous on stream.  Returns 0, PAMX_ERR_ARG for bad arguments
 * (before any device work), PAMX_ERR_HIP. */
int pamx_read_probe(const void *D, int64_t n, int64_t ld, int32_t chunk, float *sums,
                    int64_t sums_len, void *stream);

/* Measurement (not part of the method): the store rate the FP32 distance
 * kernel's output pattern can reach.  Writes `value` to D[r][c] for r, c in
 * [0, n) in exactly the launch shape and store pattern of the distance
 * kernel (64 x 64 tiles, eight per work-group along the row, each store
 * instruction two 128-byte row pieces, streaming stores), with no loads and
 * no arithmetic; 4 n^2 bytes over the time of one call is the reference the
 * distance kernel's rate is compared with.
 *   D      device, n x ld FP32 (ld >= n), 4-byte aligned; entries beyond
 *          column n - 1 are not touched
 * Asynchronous on stream.  Returns 0, PAMX_ERR_ARG for bad arguments
 * (before any device work; n at most 65535 * 64), PAMX_ERR_HIP. */
int pamx_write_probe(void *D, int64_t n, int64_t ld, float value, void *stream);

/* Message for the last non-zero return on this thread ("" if none). */
const char *pamx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PAMX_H */
