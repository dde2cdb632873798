// pamx_internal.h -- shared declarations of the gfx950 k-medoids library:
// device state, workspace layout, value traits and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdlib>
#include <stdint.h>
#include <climits>
#include <cmath>

#include "pamx.h"

namespace pamx {

constexpr int kWG = 256;          // threads per work-group in pass kernels
// Chunk length from which the pass (and the reference read in its shape)
// issues each block's rows before summing the previous block (measured on the
// 40 GB matrix, 20000-row chunks: faster; on the 1.6 GB one, 800-row chunks:
// slower)
#ifndef PAMX_PF_CHUNK
#define PAMX_PF_CHUNK 4096
#endif
constexpr int32_t kPfChunk = PAMX_PF_CHUNK;
constexpr int kObjBlk = 256;      // objects per block in segment kernels
constexpr int kFpGroup = kWG / 64; // FasterPAM window pass: most chunks per work-group (one per wave)
constexpr int kMaxK = 16000;      // largest k accepted (slot histogram and offsets in LDS)
constexpr int kBMaxDim = 16;      // batched instances: largest point dimension
constexpr int kBMaxK = 256;       // batched instances: largest k
constexpr int kBMaxN = 2048;      // batched instances: largest sample (2 candidates per lane)
constexpr int kBTeamMax = 8;      // batched instances: largest team of work-groups per instance

// Accumulator and "infinity" per element type.  Integer dissimilarities are
// summed exactly in int64; float32 ones in FP64 (or FP32 with re-scoring).
template <typename T> struct VT;
template <> struct VT<float> {
    using acc = double;
    __host__ __device__ static constexpr float inf() { return __builtin_huge_valf(); }
    __host__ __device__ static constexpr double acc_inf() { return __builtin_huge_val(); }
};
template <> struct VT<int32_t> {
    using acc = long long;
    __host__ __device__ static constexpr int32_t inf() { return INT_MAX; }
    __host__ __device__ static constexpr long long acc_inf() { return LLONG_MAX; }
};

template <typename T> using AccT = typename VT<T>::acc;

// Device-resident state of one BUILD or SWAP run.  Every iteration kernel
// reads `done` first and returns at once when it is set, so the host can
// enqueue several iterations ahead and poll rarely.
struct alignas(64) DevState {
    int32_t iter;        // SWAP searches performed
    int32_t swaps;       // swaps applied
    int32_t done;        // converged or capped: later iteration kernels idle
    int32_t capped;      // max_iter reached
    int32_t max_iter;
    int32_t empty_slot;  // smallest slot without assigned objects, or k
    int32_t swapped;     // this iteration applied a FastPAM1 swap
    int32_t new_slot;    // slot replaced this iteration
    int32_t new_med;     // object that became the medoid
    int32_t old_med;     // object that stopped being a medoid
    int32_t bad_medoids; // input medoids duplicated or out of range
    int32_t trace_cap;
    int32_t rescored;    // candidates scored again in FP64
    int32_t n_list;      // length of the re-score list
    int32_t best_i, best_c;
    double best_v;       // FP64 best change (float path)
    long long best_vi;   // int64 best change (int path)
    double td;           // running TD (float path)
    long long td_i;      // running TD (int path)
    double margin;       // FP32 error bound used for re-scoring
    double f32_best;     // FP32 best change before re-scoring
    long long n_chg;     // BUILD: objects whose nearest distance dropped this step
    long long build_rows;// BUILD: rows read by the incremental passes
    // FasterPAM scan (Alg. 4)
    int32_t fp;          // 1: the run is a FasterPAM scan (max_iter caps passes)
    int32_t seg_skip;    // 1: no swap since the segments were built
    long long fp_pos;    // next scan position
    long long fp_visited;// positions visited
    long long fp_quiet;  // positions visited since the last swap
    long long fp_limit;  // max_iter * n
    long long fw_base;   // window of the next pass: [fw_base, fw_end)
    long long fw_end;
    int32_t fw_tiles;    // its width in candidate tiles
    long long fp_cols;   // candidate columns scored by the window passes
    int32_t sync_err;    // a bounded grid-barrier wait of the eager apply expired
};

// Lexicographic "a is better than b" on (value, slot, candidate).
template <typename A>
__device__ __forceinline__ bool lex_less(A va, int ia, int ca, A vb, int ib, int cb) {
    if (va != vb) return va < vb;
    if (ia != ib) return ia < ib;
    return ca < cb;
}

// ---- small device helpers shared by the kernel files
__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ int32_t vmin(int32_t a, int32_t b) { return min(a, b); }
// median of (d, lo, hi) for lo <= hi
__device__ __forceinline__ float vmed3(float d, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(d, lo, hi);
}
__device__ __forceinline__ int32_t vmed3(int32_t d, int32_t lo, int32_t hi) {
    return max(lo, min(d, hi));
}

// lexicographic (value, index) "a < b"
template <typename A>
__device__ __forceinline__ bool lt2(A va, int ia, A vb, int ib) {
    return va < vb || (va == vb && ia < ib);
}

// Block-wide lexicographic argmin over (v, i, c); result in thread 0.
template <typename A, int NT>
__device__ void block_argmin3(A &v, int &i, int &c) {
    __shared__ A sv[NT];
    __shared__ int si[NT], sc[NT];
    const int t = threadIdx.x;
    sv[t] = v; si[t] = i; sc[t] = c;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w && lex_less(sv[t + w], si[t + w], sc[t + w], sv[t], si[t], sc[t])) {
            sv[t] = sv[t + w]; si[t] = si[t + w]; sc[t] = sc[t + w];
        }
        __syncthreads();
    }
    v = sv[0]; i = si[0]; c = sc[0];
    __syncthreads();
}

// Block-wide sum in a fixed tree order; result returned to every thread.
template <typename A, int NT>
__device__ A block_sum(A x) {
    __shared__ A s[NT];
    const int t = threadIdx.x;
    s[t] = x;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    const A r = s[0];
    __syncthreads();
    return r;
}

// Wave-wide lexicographic argmin over (v, i, c) by butterfly; every lane
// ends with the same result.
template <typename A>
__device__ __forceinline__ void wave_argmin3(A &v, int &i, int &c) {
    for (int w = 32; w >= 1; w >>= 1) {
        const A v2 = __shfl_xor(v, w);
        const int i2 = __shfl_xor(i, w), c2 = __shfl_xor(c, w);
        if (lex_less(v2, i2, c2, v, i, c)) { v = v2; i = i2; c = c2; }
    }
}

// Wave-wide sum by butterfly (fixed pattern, same value in every lane).
template <typename A>
__device__ __forceinline__ A wave_sum(A x) {
    for (int w = 32; w >= 1; w >>= 1) x += __shfl_xor(x, w);
    return x;
}

// Workspace layout (byte offsets, 256-aligned) for one (n, k, dtype) run.
struct Layout {
    int64_t n;           // objects (consumers of a rectangular matrix)
    int64_t nc;          // candidates (locations); = n for a square matrix
    int32_t k;
    int32_t dtype;
    int32_t vec;         // candidates per lane in pass kernels (4, or 1 if ld % 4)
    int32_t tile;        // candidates per pass work-group = kWG * vec
    int32_t n_ctiles;    // candidate tiles
    int32_t L;           // objects per pass work-group (chunk)
    int32_t Q;           // object chunks
    int32_t Qg;          // FasterPAM window pass: groups of fwG chunks (= Q otherwise)
    int64_t ncp;         // padded candidate count = n_ctiles * tile
    int32_t n_oblk;      // object blocks of kObjBlk
    int32_t n_mwg;       // merge work-groups = ceil(n / kWG)
    int32_t fw;          // FasterPAM: largest window (a multiple of tile), or 0
    int32_t fwL, fwQ;    // FasterPAM: object chunk length and count of the window pass
    int32_t fwG;         // FasterPAM: chunks per work-group of the window pass (1, 2 or 4)
    int32_t eg;          // FastPAM2: grid of the cooperative eager apply, 0 = one work-group
    int32_t sbS;         // FastPAM2: candidate ranges per slot in the best-candidate scan
    size_t esz;          // element size of D (4)
    size_t asz;          // accumulator size (8)
    // offsets
    size_t D;            // stored matrix (pamx_fit with points), or SIZE_MAX
    size_t mean;         // coordinate means of the points (L2 fit), or SIZE_MAX
    size_t near, sec, dn, ds, is_med;
    size_t srow, sdn, sds;
    size_t blkcnt, blkbase, seg_off, cdn;
    size_t ginfo;        // FasterPAM window pass: run map of each chunk group, or SIZE_MAX
    size_t tdp;          // per-block sums of dn and ds (2 per block of kObjBlk objects)
    size_t segtot;       // objects per slot (k)
    size_t part, part_i;
    size_t cand_v, cand_i, cand_a;
    size_t wg_v, wg_i, wg_c;
    size_t P, slot_v, slot_c;   // P: FastPAM2 only (SIZE_MAX otherwise), (k + Q) x ncp FP64
    bool has_p;
    size_t list, list_v, list_i, rlist;
    size_t cl_v, cl_i;   // FastCLARANS: changes and slots of a window of draws
    size_t mark;         // medoid check: one counter per candidate
    size_t egred;        // FastPAM2: per-work-group re-score sums of the eager apply
    size_t sb_v, sb_c;   // FastPAM2: per-range best candidates of every slot
    size_t DT;           // rectangular matrix: its transpose (candidate rows), or SIZE_MAX
    int64_t ldt;         // row stride of DT
    size_t state;
    size_t head;         // end of the regions that do not depend on the chunk length
    size_t total;
    int64_t ld_fit;      // row stride of the stored matrix in pamx_fit
};

// host helpers (pamx_api.cpp)
// ncand >= 0: a rectangular n x ncand matrix (objects x candidates), whose
// transpose the workspace holds; else square (ncand = n)
int make_layout(int64_t n, int32_t k, int32_t dim, int32_t input_kind, int32_t dtype,
                int64_t ld, const pamx_options *opt, Layout *L, const void *D,
                int64_t ncand = -1);
// Grid for the cooperative FastPAM2 eager apply over n objects on the
// current device (0: the device has no cooperative launch).
int32_t eager_grid(int64_t n, int32_t dtype);
// Cooperative launches (the FastPAM2 eager apply over the whole chip, teams
// of batched instances) unless the environment sets PAMX_COOPERATIVE=0,
// read on every call: the one-work-group forms then run, with equal results.
inline bool cooperative_allowed() {
    const char *e = std::getenv("PAMX_COOPERATIVE");
    return !(e && e[0] == '0');
}
// flags[0] |= PAMX_DIS_* bits, flags[1] += offending entries (zeroed by the caller)
hipError_t launch_check_dis(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t *flags,
                            hipStream_t s);
hipError_t launch_read_probe(const float *D, int64_t n, int64_t ld, int32_t L, float *sums,
                             hipStream_t s);
hipError_t launch_transpose(const void *D, int64_t ld, int64_t rows, int64_t cols, void *DT,
                            int64_t ldt, hipStream_t s);
// re-place the chunk-dependent regions (after L->head) for chunk length Lc
void set_chunk(Layout *L, int32_t Lc);
// FasterPAM: place them for the window pass (chunk fwL, fw partial columns)
void set_window(Layout *L);

// launchers (one per kernel family); each returns hipSuccess or an error.
hipError_t launch_dist_l1_i32(const int32_t *X, int64_t n, int32_t dim, int32_t *D, int64_t ld,
                              hipStream_t s);
// measurement: the FP32 distance kernel's stores alone (value v into D[r][c], r, c < n)
hipError_t launch_write_probe(float *D, int64_t n, int64_t ld, float v, hipStream_t s);
// mm[2*dim] (device scratch) receives the minimum and maximum of every
// coordinate of the integer points
hipError_t launch_range_i32(const int32_t *X, int64_t n, int32_t dim, int32_t *mm, hipStream_t s);
// mean[dim] (device scratch) receives the coordinate means; the distances are
// those of the centred points
hipError_t launch_dist_l2_f32(const float *X, int64_t n, int32_t dim, float *D, int64_t ld,
                              float *mean, hipStream_t s);

// Workspace layout of the mixed-precision (BF16 Gram, FP32 sums, FP64
// re-score) form for points.
struct RcLayout {
    int64_t n;
    int32_t k, KP, n_ctiles, L, Q, n_oblk;
    int64_t ncp;
    size_t Xb, nb, eo, dn64, ds64, dn32, ds32, sdn, sds, sthr, snb, R64, R32, part, part_i,
        cand_v, cand_b, wg_u, list, res_v, res_i, rlist, near, sec, srow, blkcnt, tdp, segtot, seg_off, cinfo,
        is_med, mx, eps0, bnd, mean, state, acur, lold, lnew, rs_part, total;
};
constexpr int kRcMaxDim = 64;     // precision form: largest point dimension
constexpr int kRcMaxK = 4096;     // precision form: largest k (per-slot FP64 sums in LDS)
hipError_t rc_prep_build(const float *X, int32_t dim, const RcLayout &R, int32_t k,
                         const pamx_options &opt, int32_t *medoids, void *ws, hipStream_t s,
                         const float *mean);
hipError_t rc_td(const RcLayout &R, void *ws, hipStream_t s);
hipError_t rc_swap_init(const float *X, int32_t dim, const RcLayout &R, const int32_t *medoids,
                        const pamx_options &opt, void *ws, hipStream_t s);
hipError_t rc_swap_iteration(const float *X, int32_t dim, const RcLayout &R, int32_t *medoids,
                             const pamx_options &opt, void *ws, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1);
hipError_t rc_finalize(const float *X, int32_t dim, const RcLayout &R, const int32_t *medoids,
                       int32_t *labels, void *ws, hipStream_t s);
hipError_t launch_mean_f32(const float *X, int64_t n, int32_t dim, float *mean, hipStream_t s);
int make_rc_layout(int64_t n, int32_t k, int32_t dim, const pamx_options *opt, RcLayout *R);

// Arguments of the batched (CLARA) kernels; all pointers are device pointers.
struct BatchArgs {
    const int64_t *soff;    // [n_inst+1] sample offsets
    const int32_t *sidx;    // sample point indices
    const int32_t *kin;     // [n_inst] k per instance
    const int64_t *moff;    // [n_inst+1] medoid offsets
    const int32_t *tk_inst; // [n_tick] instance of each queue ticket, largest estimated cost first
    const int32_t *tk_mem;  // [n_tick] team member of the ticket
    const int32_t *tsz;     // [n_inst] team size (work-groups) of each instance
    int32_t *bar;           // [n_inst] team arrival counters, zero before the launch
    unsigned long long *xch;   // [n_inst][2][kBTeamMax][2] team exchange slots
    int32_t n_inst, n_tick, max_iter, excl, n_max, k_max, grid, nblk;
    int32_t coop;           // teams present: cooperative launch
    int32_t *med_out;       // global indices of the medoids, instance-major
    double *td_out, *tdb_out, *part, *td_full;
    int32_t *it_out, *sw_out, *queue, *err;
    int32_t *rows_out;      // rows read by the incremental BUILD steps
};
size_t batched_lds_bytes_host(int n_max, int k_max, int dim, size_t esz);
// Work-groups of k_clara resident at once on the current device for this
// LDS size, and whether it has cooperative launch (teams need both).
int batched_resident(int32_t dim, size_t lds, int32_t dtype, int *coop);
constexpr int kBTeamSlots = kBTeamMax * 2 * 2;   // exchange words per instance (members x 2 parities x 2)
hipError_t launch_check_sidx(const int32_t *sidx, int64_t total, int64_t N, int32_t *err,
                             hipStream_t s);
template <typename T>
hipError_t launch_clara(const T *X, int64_t N, int32_t dim, const BatchArgs &a, hipStream_t s);
template <typename T>
hipError_t launch_full_assign(const T *X, int64_t N, int32_t dim, const BatchArgs &a, hipStream_t s);

// Workspace of the faster initialisations (init.hip): weights / nearest
// distances (two buffers), block sums (two buffers), medoid flags, the
// subsample changes and an error flag.
struct InitLayout {
    int32_t nblk;
    size_t dn0, dn1, bs0, bs1, is_med, vals, err, total;
};
InitLayout make_init_layout(int64_t n, int32_t m);
template <typename T>
hipError_t launch_init_dw(const T *D, int64_t ld, int64_t n, int32_t k, const double *u,
                          int32_t *med, void *ws, hipStream_t s);
hipError_t launch_init_zero(int32_t *p, hipStream_t s);
template <typename T>
hipError_t launch_init_lab(const T *D, int64_t ld, int64_t n, int32_t k, const int32_t *S,
                           int32_t m, int32_t excl, int32_t *med, void *ws, hipStream_t s);

template <typename T>
hipError_t run_build(const T *D, int64_t ld, const Layout &L, int32_t k, int32_t exclude_self,
                     int32_t *medoids, void *ws, hipStream_t s, hipEvent_t *ev);

template <typename T>
hipError_t enqueue_swap_init(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                             const pamx_options &opt, void *ws, hipStream_t s);
template <typename T>
hipError_t enqueue_swap_iteration(const T *D, int64_t ld, const Layout &L, int32_t *medoids,
                                  const pamx_options &opt, void *ws, hipStream_t s,
                                  hipEvent_t ev0, hipEvent_t ev1);
template <typename T>
hipError_t enqueue_tune_passes(const T *D, int64_t ld, const Layout &L, const pamx_options &opt,
                               void *ws, hipStream_t s, hipEvent_t *ev, int reps);
// FastCLARANS: state for a search over `len` draws, and one window step
template <typename T>
hipError_t enqueue_cl_init(const Layout &L, int64_t len, int64_t maxneighbor, void *ws,
                           hipStream_t s);
template <typename T>
hipError_t enqueue_cl_step(const T *D, int64_t ld, const Layout &L, const int32_t *draws,
                           int32_t *medoids, const pamx_options &opt, void *ws, hipStream_t s);
template <typename T>
hipError_t enqueue_finalize(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                            int32_t *labels, void *ws, hipStream_t s);

}  // namespace pamx
