// pamx_api.hip -- host side of the C ABI declared in include/pamx.h:
// argument validation (before any device work), workspace layout, and the
// orchestration of BUILD (Alg. 1) and SWAP (Alg. 3 / eager FastPAM2) of
// Schubert & Rousseeuw, arXiv 2008.05171.
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "pamx_internal.h"

namespace pamx {
template <typename T>
hipError_t enqueue_swap_caches(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                               void *ws, hipStream_t s);
}

using namespace pamx;

static thread_local char g_err[512] = "";

static int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(PAMX_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

extern "C" const char *pamx_last_error(void) { return g_err; }

extern "C" void pamx_default_options(pamx_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->variant = PAMX_FASTPAM1;
    opt->accum = PAMX_ACC_F64;
    opt->max_iter = 10000;
}

static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

namespace pamx {

// Chunk length (a multiple of 8 objects).  The pass grid (column tiles x
// object chunks) is kept at or just below two work-groups per compute unit
// (256 CUs): a grid slightly above that leaves a few CUs with a third
// work-group that holds the whole pass back (measured on the 20000-point
// workload: 520 work-groups 9% slower than 500).
static int32_t auto_chunk(int64_t n, int32_t n_ctiles) {
    int64_t Q = 512 / n_ctiles;
    const int64_t qmax = (n + 63) / 64;
    if (Q > qmax) Q = qmax;
    if (Q < 1) Q = 1;
    int64_t Lc = (n + Q - 1) / Q;
    Lc = (Lc + 7) & ~int64_t(7);
    return (int32_t)Lc;
}

// FasterPAM window pass: chunks per work-group for window chunks of Lw
// objects.  Short chunks are bound by the latency of their few blocks of
// rows and the merge of their many partials, so four chunks share a
// work-group (and one partial): SWAP phase 11.1 -> 10.5 ms at n = 20000
// (80-object chunks).  Long chunks stream, and one chunk per work-group (its
// four waves on the same rows, no merge through LDS) is faster: 102 against
// 107 ms at n = 100000 (392-object chunks).
// PAMX_FP_GROUP=1, 2 or 4 in the environment fixes it (equal results on
// integer distances; with floating point the group sums are added in another
// order and may round differently).
static int32_t fp_group(int64_t Lw) {
    if (const char *e = std::getenv("PAMX_FP_GROUP")) {
        const int g = std::atoi(e);
        if (g == 1 || g == 2 || g == 4) return g;
    }
    return Lw <= 128 ? 4 : 1;
}

int make_layout(int64_t n, int32_t k, int32_t dim, int32_t input_kind, int32_t dtype,
                int64_t ld, const pamx_options *opt, Layout *L, const void *D, int64_t ncand) {
    std::memset(L, 0, sizeof(*L));
    const bool rect = ncand >= 0;
    const int64_t nc = rect ? ncand : n;
    L->n = n;
    L->nc = nc;
    L->k = k;
    L->dtype = dtype;
    L->esz = 4;
    L->asz = 8;
    L->ld_fit = (n + 63) & ~int64_t(63);
    const int64_t ldx = (input_kind == PAMX_INPUT_X) ? L->ld_fit : ld;
    // 16-byte loads need 4 | ld and a 16-byte aligned matrix
    const bool aligned = (input_kind == PAMX_INPUT_X) || !D ||
                         (reinterpret_cast<uintptr_t>(D) & 15) == 0;
    L->vec = (ldx % 4 == 0 && aligned) ? 4 : 1;
    L->tile = kWG * L->vec;
    L->n_ctiles = (int32_t)((nc + L->tile - 1) / L->tile);
    L->ncp = (int64_t)L->n_ctiles * L->tile;
    int32_t Lc = (opt && opt->chunk > 0) ? opt->chunk : auto_chunk(n, L->n_ctiles);
    if (Lc > n) Lc = (int32_t)n;
    L->L = Lc;
    L->Q = (int32_t)((n + Lc - 1) / Lc);
    L->n_oblk = (int32_t)((n + kObjBlk - 1) / kObjBlk);
    L->n_mwg = (int32_t)((nc + kWG - 1) / kWG);
    const bool p2 = opt && opt->variant == PAMX_FASTPAM2;
    if (opt && opt->variant == PAMX_FASTERPAM) {
        // largest window: the requested width rounded up to whole tiles, else
        // 16 tiles; the pass is chunked for about one work-group per compute
        // unit on a one-tile window (the width after a swap): 256 chunks of
        // eight-row blocks measured 8 % faster than 512 (at most n / 64) of
        // four-row blocks at n = 20000 (smaller partials for the merge) and
        // the same at n = 100000
        int64_t m = (opt->window > 0) ? (opt->window + L->tile - 1) / L->tile : 16;
        if (m < 1) m = 1;
        if (m > L->n_ctiles) m = L->n_ctiles;
        if (m > 256) m = 256;
        L->fw = (int32_t)(m * L->tile);
        int64_t Q = 256;
        const int64_t qmax = (n + 63) / 64;
        if (Q > qmax) Q = qmax;
        if (Q < 1) Q = 1;
        int64_t Lw = (n + Q - 1) / Q;
        Lw = (Lw + 7) & ~int64_t(7);
        if (Lw > n) Lw = n;
        L->fwL = (int32_t)Lw;
        L->fwQ = (int32_t)((n + Lw - 1) / Lw);
        L->fwG = fp_group(Lw);
    }

    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = up256(off + (bytes ? bytes : 1)); return o; };
    L->D = SIZE_MAX;
    L->mean = SIZE_MAX;
    L->DT = SIZE_MAX;
    if (rect) {
        L->ldt = (n + 63) & ~int64_t(63);
        L->DT = take((size_t)nc * (size_t)L->ldt * 4);
    }
    if (input_kind == PAMX_INPUT_X) {
        L->D = take((size_t)n * (size_t)L->ld_fit * 4);
        L->mean = take((size_t)dim * (dtype == PAMX_F32 ? 4 : 8));   // means / ranges
    }
    L->near = take((size_t)n * 4);
    L->sec = take((size_t)n * 4);
    L->dn = take((size_t)n * 4);
    L->ds = take((size_t)n * 4);
    L->is_med = take((size_t)nc);
    L->mark = take((size_t)nc * 4);
    L->srow = take((size_t)n * 4);
    L->sdn = take((size_t)n * 4);
    L->sds = take((size_t)n * 4);
    L->blkcnt = take((size_t)L->n_oblk * k * 4);
    L->tdp = take((size_t)L->n_oblk * 2 * 8);
    L->segtot = take((size_t)k * 4);
    L->seg_off = take((size_t)(k + 1) * 4);
    L->cand_v = take(8);
    L->cand_i = take(8);
    L->cand_a = take((size_t)L->ncp * 8);
    // >= n_mwg, >= the SWAP merge grid (ncp / 64) and >= the window-merge grid (256)
    const size_t nwg = (size_t)(L->ncp / 16) > 256 ? (size_t)(L->ncp / 16) : 256;
    L->wg_v = take(nwg * 8);
    L->wg_i = take(nwg * 4);
    L->wg_c = take(nwg * 4);
    L->has_p = p2;   // P depends on the chunk count: placed with the chunk-dependent regions
    L->slot_v = take((size_t)k * 8);
    L->slot_c = take((size_t)k * 4);
    L->list = take((size_t)(n > k ? n : k) * 4);
    L->list_v = take(8);
    L->list_i = take(8);
    L->rlist = take((size_t)n * 4);
    L->cl_v = take(1024 * 8);
    L->cl_i = take(1024 * 4);
    L->egred = p2 ? take(2 * 1024 * 8 + 256) : SIZE_MAX;   // sums of two visits + barrier count
    // best-candidate scan: about 4096 work-groups in all, at least 1024
    // candidates each, at most 32 ranges per slot
    {
        int64_t S = 4096 / k;
        const int64_t smax = (nc + 1023) / 1024;
        if (S > smax) S = smax;
        if (S > 32) S = 32;
        if (S < 1) S = 1;
        L->sbS = (int32_t)S;
    }
    L->sb_v = p2 ? take((size_t)k * L->sbS * 8) : SIZE_MAX;
    L->sb_c = p2 ? take((size_t)k * L->sbS * 4) : SIZE_MAX;
    L->state = take(sizeof(DevState));
    L->head = off;
    set_chunk(L, L->L);
    return PAMX_OK;
}

// The regions whose size depends on the number of object chunks Q come last,
// so the chunk length can change between BUILD and SWAP (chunk tuning).
static void place_tail(Layout *L, int32_t Lc, int64_t cols, bool win = false) {
    if (Lc > L->n) Lc = (int32_t)L->n;
    if (Lc < 1) Lc = 1;
    L->L = Lc;
    L->Q = (int32_t)((L->n + Lc - 1) / Lc);
    // the window pass merges fwG consecutive chunks in each work-group; the
    // partials, DN parts and run map it leaves are per group
    L->Qg = win ? (L->Q + L->fwG - 1) / L->fwG : L->Q;
    size_t off = L->head;
    auto take = [&](size_t bytes) { size_t o = off; off = up256(off + (bytes ? bytes : 1)); return o; };
    L->blkbase = take((size_t)L->Q * 16);            // chunk carry map
    L->cdn = take((size_t)L->Q * 2 * 8);              // DN parts of carried segments
    L->ginfo = (win && L->fwG > 1) ? take((size_t)L->Qg * 16) : SIZE_MAX;
    L->part = take((size_t)L->Q * 4 * cols * 8);
    L->part_i = take((size_t)L->Q * cols * 4);
    // FastPAM2: one row per (chunk, segment) pair at segment + chunk (k + Q rows)
    L->P = L->has_p ? take(((size_t)L->k + L->Q) * L->ncp * 8) : SIZE_MAX;
    L->total = off;
}
void set_chunk(Layout *L, int32_t Lc) { place_tail(L, Lc, L->ncp); }
void set_window(Layout *L) { place_tail(L, L->fwL, L->fw, true); }

// Chunk lengths tried by the tuner: pass grids at or just below about 1, 1.5,
// 2, 3, 4, 6 and 8 work-groups per compute unit.
std::vector<int32_t> tune_chunks(const Layout &L) {
    static const int grid[] = {256, 384, 512, 768, 1024, 1536, 2048};
    const int64_t qmax = (L.n + 63) / 64;
    std::vector<int32_t> out;
    for (int g : grid) {
        int64_t Q = g / L.n_ctiles;
        if (Q > qmax) Q = qmax;
        if (Q < 1) Q = 1;
        int64_t Lc = (L.n + Q - 1) / Q;
        Lc = (Lc + 7) & ~int64_t(7);
        if (Lc > L.n) Lc = L.n;
        if (std::find(out.begin(), out.end(), (int32_t)Lc) == out.end()) out.push_back((int32_t)Lc);
    }
    return out;
}

// Workspace bytes for L: with chunk tuning, the largest tail over the chunk
// lengths the tuner may pick.
size_t layout_need(const Layout &L, const pamx_options *opt) {
    if (L.fw > 0) {
        Layout T = L;
        set_window(&T);
        return T.total > L.total ? T.total : L.total;
    }
    if (!opt || opt->chunk >= 0) return L.total;
    size_t need = L.total;
    for (int32_t Lc : tune_chunks(L)) {
        Layout T = L;
        set_chunk(&T, Lc);
        if (T.total > need) need = T.total;
    }
    return need;
}

int make_rc_layout(int64_t n, int32_t k, int32_t dim, const pamx_options *opt, RcLayout *R) {
    std::memset(R, 0, sizeof(*R));
    R->n = n;
    R->k = k;
    R->KP = ((dim + 15) / 16) * 16;
    R->n_ctiles = (int32_t)((n + 255) / 256);
    R->ncp = (int64_t)R->n_ctiles * 256;
    R->n_oblk = (int32_t)((n + kObjBlk - 1) / kObjBlk);
    int64_t Lc;
    if (opt && opt->chunk > 0) {
        Lc = opt->chunk;
    } else {
        int64_t Q = (1024 + R->n_ctiles - 1) / R->n_ctiles;   // ~4 work-groups per CU
        if (Q < 1) Q = 1;
        Lc = (n + Q - 1) / Q;
    }
    Lc = ((Lc + 31) / 32) * 32;
    if (Lc > n) Lc = n;
    R->L = (int32_t)Lc;
    R->Q = (int32_t)((n + Lc - 1) / Lc);
    const int64_t nmwg = (n + 255) / 256;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = up256(off + (bytes ? bytes : 1)); return o; };
    R->Xb = take((size_t)n * R->KP * 4);              // split rows: hi and lo, bf16
    R->nb = take((size_t)n * 4);
    R->eo = take((size_t)n * 8);
    R->dn64 = take((size_t)n * 8);
    R->ds64 = take((size_t)n * 8);
    R->dn32 = take((size_t)n * 4);
    R->ds32 = take((size_t)n * 4);
    R->sdn = take((size_t)n * 4);
    R->sds = take((size_t)n * 4);
    R->sthr = take((size_t)n * 4);
    R->snb = take((size_t)n * 4);
    R->R64 = take((size_t)k * 8);
    R->R32 = take((size_t)k * 4);
    R->part = take((size_t)R->Q * 4 * R->ncp * 8);
    R->part_i = take((size_t)R->Q * 4 * R->ncp * 4);
    R->cand_v = take((size_t)R->ncp * 8);
    R->cand_b = take((size_t)R->ncp * 8);
    R->wg_u = take((size_t)nmwg * 8);
    R->list = take((size_t)n * 4);
    R->res_v = take((size_t)n * 8);
    R->res_i = take((size_t)n * 4);
    R->rlist = take((size_t)n * 4);
    R->near = take((size_t)n * 4);
    R->sec = take((size_t)n * 4);
    R->srow = take((size_t)n * 4);
    R->blkcnt = take((size_t)R->n_oblk * k * 4);
    R->tdp = take((size_t)R->n_oblk * 2 * 8);
    R->segtot = take((size_t)k * 4);
    R->seg_off = take((size_t)(k + 1) * 4);
    R->cinfo = take((size_t)R->Q * 16);
    R->is_med = take((size_t)n);
    R->mx = take(2 * 8);
    R->eps0 = take(4 * 8);
    R->bnd = take(4 * 8);
    R->mean = take((size_t)dim * 4);
    R->state = take(sizeof(DevState));
    // FP64 BUILD: running A(c), list of objects whose dn dropped (old, new)
    R->acur = take((size_t)R->ncp * 8);
    R->lold = take((size_t)n * 8);
    R->lnew = take((size_t)n * 8);
    R->rs_part = take((size_t)4096 * (k + 1) * 8);   // FP64 re-score partials
    R->total = off;
    return PAMX_OK;
}

}  // namespace pamx

// ---------------------------------------------------------------- validation
static int check_common(int64_t n, int32_t k, int32_t dtype, const pamx_options *opt) {
    if (n < 1) return fail(PAMX_ERR_ARG, "n must be >= 1 (got %lld)", (long long)n);
    if (n > (int64_t)INT32_MAX - 1) return fail(PAMX_ERR_ARG, "n too large for int32 indices");
    if (k < 1) return fail(PAMX_ERR_ARG, "k must be >= 1 (got %d)", k);
    if (k > n) return fail(PAMX_ERR_ARG, "k (%d) must not exceed n (%lld)", k, (long long)n);
    if (k > kMaxK) return fail(PAMX_ERR_ARG, "k (%d) exceeds the supported maximum %d", k, kMaxK);
    if (dtype != PAMX_I32 && dtype != PAMX_F32)
        return fail(PAMX_ERR_ARG, "unknown dtype %d", dtype);
    if (opt) {
        if (opt->variant != PAMX_FASTPAM1 && opt->variant != PAMX_FASTPAM2 &&
            opt->variant != PAMX_FASTERPAM)
            return fail(PAMX_ERR_ARG, "unknown variant %d", opt->variant);
        if (opt->window < 0) return fail(PAMX_ERR_ARG, "window must be >= 0");
        if (opt->accum != PAMX_ACC_F64 && opt->accum != PAMX_ACC_F32)
            return fail(PAMX_ERR_ARG, "unknown accum %d", opt->accum);
        if (opt->dist_mode != PAMX_DIST_STORED && opt->dist_mode != PAMX_DIST_BF16)
            return fail(PAMX_ERR_ARG, "unknown dist_mode %d", opt->dist_mode);
        if (opt->accum == PAMX_ACC_F32 && dtype != PAMX_F32)
            return fail(PAMX_ERR_ARG, "accum PAMX_ACC_F32 needs PAMX_F32 data");
        if (opt->accum == PAMX_ACC_F32 && opt->dist_mode != PAMX_DIST_BF16)
            return fail(PAMX_ERR_UNSUPPORTED, "accum PAMX_ACC_F32 is available with PAMX_DIST_BF16 only");
        if (opt->max_iter < 0) return fail(PAMX_ERR_ARG, "max_iter must be >= 0");
        if (opt->trace_cap < 0) return fail(PAMX_ERR_ARG, "trace_cap must be >= 0");
        if (opt->chunk < PAMX_CHUNK_TUNE)
            return fail(PAMX_ERR_ARG, "chunk must be >= 0, or PAMX_CHUNK_TUNE");
        if (opt->build_exclude_self != 0 && opt->build_exclude_self != 1)
            return fail(PAMX_ERR_ARG, "build_exclude_self must be 0 or 1");
        if (opt->dist_mode != PAMX_DIST_STORED && opt->dist_mode != PAMX_DIST_BF16)
            return fail(PAMX_ERR_ARG, "unknown dist_mode %d", opt->dist_mode);
    }
    return PAMX_OK;
}

static int check_rc(int32_t input_kind, int32_t dtype, int32_t metric, int32_t dim, int32_t k,
                    const pamx_options *opt) {
    if (input_kind != PAMX_INPUT_X || dtype != PAMX_F32 || metric != PAMX_L2)
        return fail(PAMX_ERR_ARG, "PAMX_DIST_BF16 needs float32 points with the L2 metric");
    if (dim > kRcMaxDim) return fail(PAMX_ERR_UNSUPPORTED, "PAMX_DIST_BF16 supports dim <= %d", kRcMaxDim);
    if (k > kRcMaxK) return fail(PAMX_ERR_UNSUPPORTED, "PAMX_DIST_BF16 supports k <= %d", kRcMaxK);
    if (opt && opt->variant != PAMX_FASTPAM1)
        return fail(PAMX_ERR_UNSUPPORTED, "PAMX_DIST_BF16 runs FastPAM1 only");
    return PAMX_OK;
}

static int check_matrix(const void *D, int64_t n, int64_t ld) {
    if (!D) return fail(PAMX_ERR_ARG, "D is NULL");
    if (ld < n) return fail(PAMX_ERR_ARG, "ld (%lld) must be >= n (%lld)", (long long)ld, (long long)n);
    if (ld > (int64_t)1 << 40 || n > ((int64_t)1 << 62) / ld)
        return fail(PAMX_ERR_ARG, "n * ld overflows");
    return PAMX_OK;
}

static int check_ws(void *ws, size_t ws_bytes, const Layout &L, const pamx_options *opt) {
    if (!ws) return fail(PAMX_ERR_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t need = layout_need(L, opt);
    if (ws_bytes < need)
        return fail(PAMX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    return PAMX_OK;
}

extern "C" int pamx_workspace_bytes(int64_t n, int32_t k, int32_t dim, int32_t input_kind,
                                    int32_t dtype, const pamx_options *opt, size_t *bytes) {
    if (!bytes) return fail(PAMX_ERR_ARG, "bytes is NULL");
    int rc = check_common(n, k, dtype, opt);
    if (rc) return rc;
    if (input_kind != PAMX_INPUT_D && input_kind != PAMX_INPUT_X)
        return fail(PAMX_ERR_ARG, "unknown input_kind %d", input_kind);
    if (input_kind == PAMX_INPUT_X && dim < 1) return fail(PAMX_ERR_ARG, "dim must be >= 1");
    if (opt && opt->dist_mode == PAMX_DIST_BF16) {
        rc = check_rc(input_kind, dtype, PAMX_L2, dim, k, opt);
        if (rc) return rc;
        RcLayout R;
        make_rc_layout(n, k, dim, opt, &R);
        *bytes = R.total;
        return PAMX_OK;
    }
    Layout L;
    // the pass tiling depends on ld and on the matrix alignment: take the
    // larger of the 16-byte-load and scalar-load layouts
    make_layout(n, k, dim, input_kind, dtype, (n + 3) & ~int64_t(3), opt, &L, nullptr);
    const size_t b4 = layout_need(L, opt);
    make_layout(n, k, dim, input_kind, dtype, (n % 4) ? n : n + 1, opt, &L, nullptr);
    const size_t b1 = layout_need(L, opt);
    *bytes = b4 > b1 ? b4 : b1;
    return PAMX_OK;
}

// ---------------------------------------------------------------- distances
// Integer points: every L1 distance must be an int32 below INT32_MAX (the
// "no medoid" sentinel), and no distance exceeds the sum over coordinates of
// (max - min).  mm is device scratch of 2 * dim int32; the host waits for the
// per-coordinate ranges and refuses points whose sum exceeds INT32_MAX - 1.
static int check_l1_range(const int32_t *X, int64_t n, int32_t dim, int32_t *mm, hipStream_t s) {
    HIP_TRY(launch_range_i32(X, n, dim, mm, s));
    std::vector<int32_t> h((size_t)2 * dim);
    HIP_TRY(hipMemcpyAsync(h.data(), mm, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t span = 0;
    for (int32_t j = 0; j < dim; ++j) {
        span += (int64_t)h[2 * j + 1] - (int64_t)h[2 * j];
        if (span > (int64_t)INT32_MAX - 1)
            return fail(PAMX_ERR_ARG, "int32 points: the coordinate ranges sum past INT32_MAX - 1 "
                                      "(an L1 distance could overflow int32)");
    }
    return PAMX_OK;
}

// scratch: 4 * dim bytes for float32 points (coordinate means), 8 * dim for
// int32 points (coordinate ranges)
static int dist_impl(const void *X, int32_t dtype, int64_t n, int32_t dim, int32_t metric, void *D,
                     int64_t ld, void *scratch, hipStream_t s) {
    if (dtype == PAMX_I32 && metric == PAMX_L1) {
        const int rc = check_l1_range(static_cast<const int32_t *>(X), n, dim,
                                      static_cast<int32_t *>(scratch), s);
        if (rc) return rc;
        HIP_TRY(launch_dist_l1_i32(static_cast<const int32_t *>(X), n, dim, static_cast<int32_t *>(D),
                                   ld, s));
    } else
        HIP_TRY(launch_dist_l2_f32(static_cast<const float *>(X), n, dim, static_cast<float *>(D), ld,
                                   static_cast<float *>(scratch), s));
    return PAMX_OK;
}

static int check_points(const void *X, int32_t dtype, int64_t n, int32_t dim, int32_t metric) {
    if (!X) return fail(PAMX_ERR_ARG, "X is NULL");
    if (dim < 1) return fail(PAMX_ERR_ARG, "dim must be >= 1 (got %d)", dim);
    if (metric != PAMX_L1 && metric != PAMX_L2) return fail(PAMX_ERR_ARG, "unknown metric %d", metric);
    if (dtype == PAMX_I32 && metric != PAMX_L1)
        return fail(PAMX_ERR_UNSUPPORTED, "int32 points support the L1 metric only");
    if (dtype == PAMX_F32 && metric != PAMX_L2)
        return fail(PAMX_ERR_UNSUPPORTED, "float32 points support the L2 metric only");
    return PAMX_OK;
}

extern "C" int pamx_dist(const void *X, int32_t dtype, int64_t n, int32_t dim, int32_t metric,
                         void *D, int64_t ld, void *ws, size_t ws_bytes, void *stream) {
    if (n < 1) return fail(PAMX_ERR_ARG, "n must be >= 1");
    if (dtype != PAMX_I32 && dtype != PAMX_F32) return fail(PAMX_ERR_ARG, "unknown dtype %d", dtype);
    int rc = check_points(X, dtype, n, dim, metric);
    if (rc) return rc;
    rc = check_matrix(D, n, ld);
    if (rc) return rc;
    if (ld % 4) return fail(PAMX_ERR_ARG, "ld must be a multiple of 4");
    const size_t need = (size_t)dim * (dtype == PAMX_F32 ? 4 : 8);
    if (!ws || ws_bytes < need)
        return fail(PAMX_ERR_WORKSPACE, "the points need a workspace of %zu bytes (got %zu)", need,
                    ws ? ws_bytes : (size_t)0);
    if ((reinterpret_cast<uintptr_t>(ws) & 3) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = dist_impl(X, dtype, n, dim, metric, D, ld, ws, s);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return PAMX_OK;
}

extern "C" int pamx_check_dissimilarity(const void *D, int32_t dtype, int64_t n, int64_t ld,
                                        int32_t *flags, int64_t *count, void *ws,
                                        size_t ws_bytes, void *stream) {
    if (n < 1) return fail(PAMX_ERR_ARG, "n must be >= 1");
    if (dtype != PAMX_I32 && dtype != PAMX_F32) return fail(PAMX_ERR_ARG, "unknown dtype %d", dtype);
    int rc = check_matrix(D, n, ld);
    if (rc) return rc;
    if (!flags) return fail(PAMX_ERR_ARG, "flags is NULL");
    if (n > (int64_t)65535 * 64) return fail(PAMX_ERR_ARG, "n too large for the check grid");
    if (!ws || ws_bytes < 8) return fail(PAMX_ERR_WORKSPACE, "the check needs a workspace of 8 bytes");
    if ((reinterpret_cast<uintptr_t>(ws) & 3) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *dflags = static_cast<int32_t *>(ws);
    HIP_TRY(hipMemsetAsync(dflags, 0, 2 * sizeof(int32_t), s));   // never captured in a graph
    HIP_TRY(launch_check_dis(D, dtype, n, ld, dflags, s));
    int32_t h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h, dflags, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *flags = h[0];
    if (count) *count = h[1];
    return PAMX_OK;
}

extern "C" int pamx_read_probe(const void *D, int64_t n, int64_t ld, int32_t chunk, float *sums,
                               int64_t sums_len, void *stream) {
    if (n < 1) return fail(PAMX_ERR_ARG, "n must be >= 1");
    int rc = check_matrix(D, n, ld);
    if (rc) return rc;
    if (ld % 4 != 0 || (reinterpret_cast<uintptr_t>(D) & 15) != 0)
        return fail(PAMX_ERR_ARG, "the probe needs ld %% 4 == 0 and a 16-byte aligned matrix");
    if (chunk < 1) return fail(PAMX_ERR_ARG, "chunk must be >= 1");
    const int64_t tiles = (n + 1023) / 1024, q = (n + chunk - 1) / chunk;
    if (q > 65535) return fail(PAMX_ERR_ARG, "chunk too small: %lld row chunks", (long long)q);
    if (!sums) return fail(PAMX_ERR_ARG, "sums is NULL");
    if (sums_len < tiles * q)
        return fail(PAMX_ERR_ARG, "sums holds %lld floats, the probe writes %lld",
                    (long long)sums_len, (long long)(tiles * q));
    HIP_TRY(launch_read_probe(static_cast<const float *>(D), n, ld, chunk, sums,
                              static_cast<hipStream_t>(stream)));
    return PAMX_OK;
}

extern "C" int pamx_write_probe(void *D, int64_t n, int64_t ld, float value, void *stream) {
    if (n < 1) return fail(PAMX_ERR_ARG, "n must be >= 1");
    int rc = check_matrix(D, n, ld);
    if (rc) return rc;
    if ((reinterpret_cast<uintptr_t>(D) & 3) != 0) return fail(PAMX_ERR_ARG, "D must be 4-byte aligned");
    if (n > (int64_t)65535 * 64) return fail(PAMX_ERR_ARG, "n too large for the probe grid");
    HIP_TRY(launch_write_probe(static_cast<float *>(D), n, ld, value, static_cast<hipStream_t>(stream)));
    return PAMX_OK;
}

// ---------------------------------------------------------------- BUILD / SWAP
namespace {

struct Timer {
    hipEvent_t e[6] = {};
    bool ok = false;
    // on = false: no events are created and every duration reads 0
    explicit Timer(bool on = true) {
        if (!on) return;
        ok = true;
        for (auto &x : e)
            if (hipEventCreate(&x) != hipSuccess) ok = false;
    }
    ~Timer() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    void rec(int i, hipStream_t s) {
        if (ok) (void)hipEventRecord(e[i], s);
    }
    // 0 if either event was not recorded (an early error return); the
    // failed query's error is cleared so no later launch check reports it
    double ms(int a, int b) {
        float v = 0.f;
        if (!ok) return 0.0;
        if (hipEventElapsedTime(&v, e[a], e[b]) == hipSuccess) return v;
        (void)hipGetLastError();
        return 0.0;
    }
};

// A pool of HIP events bracketing pass kernels (pamx_options.profile).
struct EventPool {
    std::vector<hipEvent_t> ev;
    explicit EventPool(size_t count) : ev(count, nullptr) {
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    }
    ~EventPool() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    bool ok() const {
        for (auto e : ev)
            if (!e) return false;
        return true;
    }
    // summed duration of the first `pairs` (begin, end) pairs
    double sum(int pairs) const { return sum(0, pairs); }
    // summed duration of (begin, end) pairs j0 .. j1-1
    double sum(int j0, int j1) const {
        double t = 0.0;
        for (int j = j0; j < j1; ++j) {
            float v = 0.f;
            if (hipEventElapsedTime(&v, ev[2 * j], ev[2 * j + 1]) == hipSuccess) t += v;
        }
        return t;
    }
};

int read_state(const Layout &L, void *ws, hipStream_t s, DevState *out) {
    const char *w = static_cast<const char *>(ws);
    HIP_TRY(hipMemcpyAsync(out, w + L.state, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PAMX_OK;
}

template <typename T>
int build_impl(const T *D, int64_t ld, const Layout &L, int32_t k, const pamx_options &opt,
               int32_t *medoids, double *td, void *ws, hipStream_t s, pamx_stats *stats) {
    std::unique_ptr<EventPool> pool;
    if (opt.profile) {
        pool.reset(new EventPool(2 * (size_t)k));
        if (!pool->ok()) return fail(PAMX_ERR_HIP, "hipEventCreate failed");
    }
    HIP_TRY(run_build<T>(D, ld, L, k, opt.build_exclude_self, medoids, ws, s,
                         pool ? pool->ev.data() : nullptr));
    DevState st;
    int rc = read_state(L, ws, s, &st);
    if (rc) return rc;
    if (st.bad_medoids) return fail(PAMX_ERR_HIP, "BUILD found no candidate");
    if (td) *td = st.td;
    if (stats) {
        const int full = k < 2 ? k : 2;
        stats->build_rows = st.build_rows;
        stats->build_pairs = (int64_t)full * L.n * L.nc + st.build_rows * L.nc;
        if (pool) {
            stats->ms_build_pass = pool->sum(0, full);
            stats->n_build_pass = full;
            stats->ms_build_delta = pool->sum(full, k);
            stats->n_build_delta = k - full;
        }
    }
    return PAMX_OK;
}

// ---- SWAP searches as a HIP graph.  A library stream per host thread and
// device (default priority, never destroyed) runs the replays; events order
// it after the caller's stream and the caller's stream after it.
static hipStream_t graph_stream() {
    constexpr int kMaxDev = 64;
    thread_local hipStream_t streams[kMaxDev] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// An instantiated search graph bakes in every kernel argument: the matrix,
// the workspace (and the layout in it), the medoid and trace arrays.  Graphs
// are kept per host thread for the last few argument sets, so repeated calls
// on the same buffers replay without capturing again.
// Everything a captured search depends on: the arguments, and the layout's
// counts and offsets (a rectangular matrix moves every region behind its
// transpose, and the candidate count sets the grids).
struct SearchKey {
    int dev;
    const void *D, *ws, *med, *trace;
    int64_t ld, n, nc, ldt;
    int32_t k, dtype, variant, chunk, vec, trace_cap, fw, eg, sbS;
    size_t DT, head, total;
    auto tie() const {
        return std::tie(dev, D, ws, med, trace, ld, n, nc, ldt, k, dtype, variant, chunk, vec,
                        trace_cap, fw, eg, sbS, DT, head, total);
    }
    bool operator==(const SearchKey &o) const { return tie() == o.tie(); }
};

struct SearchGraph {
    SearchKey key{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    SearchGraph() = default;
    SearchGraph(const SearchGraph &) = delete;
    SearchGraph &operator=(const SearchGraph &) = delete;
    ~SearchGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    }
};

// The cached graph for these arguments, captured on xs if not yet there.
template <typename T>
static int search_graph(const T *D, int64_t ld, const Layout &L, int32_t *medoids,
                        const pamx_options &opt, void *ws, hipStream_t xs, SearchGraph **out) {
    constexpr size_t kKeep = 4;
    // held until the process ends (not destroyed at exit, when the HIP
    // runtime may already be gone)
    thread_local auto *cache_p = new std::vector<std::unique_ptr<SearchGraph>>();
    auto &cache = *cache_p;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const SearchKey key{dev,      D,      ws,      medoids, opt.trace, ld,   L.n,
                        L.nc,     L.ldt,  L.k,     L.dtype, opt.variant, L.L, L.vec,
                        opt.trace_cap, L.fw, L.eg, L.sbS, L.DT, L.head, L.total};
    for (auto &g : cache)
        if (g->key == key) { *out = g.get(); return PAMX_OK; }
    std::unique_ptr<SearchGraph> g(new SearchGraph);
    g->key = key;
    HIP_TRY(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g->join, hipEventDisableTiming));
    HIP_TRY(hipStreamBeginCapture(xs, hipStreamCaptureModeThreadLocal));
    const hipError_t ce = enqueue_swap_iteration<T>(D, ld, L, medoids, opt, ws, xs, nullptr, nullptr);
    const hipError_t ee = hipStreamEndCapture(xs, &g->graph);
    if (ce != hipSuccess) return fail(PAMX_ERR_HIP, "capture of a search failed: %s", hipGetErrorString(ce));
    if (ee != hipSuccess) return fail(PAMX_ERR_HIP, "end of capture failed: %s", hipGetErrorString(ee));
    HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    if (cache.size() >= kKeep) cache.erase(cache.begin());
    cache.push_back(std::move(g));
    *out = cache.back().get();
    return PAMX_OK;
}

// ---- chunk tuning: the fastest chunk length per (device, shape), timed
// once per process on the caller's matrix and kept for later calls.
struct TuneKey {
    int dev;
    int64_t n, ld;
    int32_t k, dtype, vec, variant;
    bool operator<(const TuneKey &o) const {
        return std::tie(dev, n, ld, k, dtype, vec, variant) <
               std::tie(o.dev, o.n, o.ld, o.k, o.dtype, o.vec, o.variant);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, int32_t> g_tuned;

template <typename T>
static int tune_chunk(const T *D, int64_t ld, Layout *L, const pamx_options &opt, void *ws,
                      hipStream_t s) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const TuneKey key{dev, L->n, ld, L->k, L->dtype, L->vec, opt.variant};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) { set_chunk(L, it->second); return PAMX_OK; }
    }
    constexpr int kReps = 3;
    EventPool pool(2 * kReps);
    if (!pool.ok()) return fail(PAMX_ERR_HIP, "hipEventCreate failed");
    int32_t best = L->L;
    double best_ms = 1e300;
    for (int32_t Lc : tune_chunks(*L)) {
        Layout Tl = *L;
        set_chunk(&Tl, Lc);
        HIP_TRY(enqueue_tune_passes<T>(D, ld, Tl, opt, ws, s, pool.ev.data(), kReps));
        HIP_TRY(hipStreamSynchronize(s));
        double t = 1e300;
        for (int r = 0; r < kReps; ++r) {
            const double v = pool.sum(r, r + 1);
            if (v < t) t = v;
        }
        if (t < best_ms) { best_ms = t; best = Lc; }
    }
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[key] = best;
    }
    set_chunk(L, best);
    return PAMX_OK;
}

template <typename T>
int swap_impl(const T *D, int64_t ld, const Layout &L_in, int32_t k, const pamx_options &opt,
              int32_t *medoids, int32_t *labels, double *td, pamx_stats *stats, void *ws,
              hipStream_t s, Timer &tm) {
    Layout L = L_in;
    const int64_t n = L.n;
    // FastPAM2: the eager apply runs over the whole chip where the device
    // has cooperative launch (such searches are not captured in a graph)
    if (opt.variant == PAMX_FASTPAM2 && L.egred != SIZE_MAX) L.eg = eager_grid(n, L.dtype);
    HIP_TRY(enqueue_swap_init<T>(D, ld, L, medoids, opt, ws, s));
    DevState st;
    int rc = read_state(L, ws, s, &st);
    if (rc) return rc;
    if (st.bad_medoids)
        return fail(PAMX_ERR_INVALID_MEDOIDS, "medoids must be distinct and in [0, n)");
    const bool searches = k >= 2 && k < L.nc;
    const bool scan = opt.variant == PAMX_FASTERPAM;
    if (scan) set_window(&L);   // the window passes have their own chunking
    if (searches) HIP_TRY(enqueue_swap_caches<T>(D, ld, L, medoids, ws, s));
    if (searches && !scan && opt.chunk == PAMX_CHUNK_TUNE && opt.max_iter > 0) {
        rc = tune_chunk<T>(D, ld, &L, opt, ws, s);
        if (rc) return rc;
    }
    tm.rec(2, s);
    int enq = 0;
    double ms_pass = 0.0;
    int n_pass = 0;
    if (searches) {
        constexpr int kMaxBatch = 32;
        std::unique_ptr<EventPool> pool;
        if (opt.profile) {
            pool.reset(new EventPool(2 * kMaxBatch));
            if (!pool->ok()) return fail(PAMX_ERR_HIP, "hipEventCreate failed");
        }
        SearchGraph *g = nullptr;
        hipStream_t xs = s;   // stream the searches run on
        if (opt.graph && !opt.profile && L.eg == 0) {
            hipStream_t gs = graph_stream();
            if (!gs) return fail(PAMX_ERR_HIP, "could not create the library stream");
            rc = search_graph<T>(D, ld, L, medoids, opt, ws, gs, &g);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(g->fork, s));   // after the caller's work on s
            HIP_TRY(hipStreamWaitEvent(gs, g->fork, 0));
            xs = gs;
        }
        int batch = 4;
        for (;;) {
            int b = batch;
            // a FasterPAM scan takes an unknown number of windows (its
            // cap counts passes and is applied on the device)
            if (!scan && b > opt.max_iter + 1 - enq) b = opt.max_iter + 1 - enq;
            if (b < 1) b = 1;
            const int iter0 = st.iter;
            for (int j = 0; j < b; ++j) {
                if (g)
                    HIP_TRY(hipGraphLaunch(g->exec, xs));
                else
                    HIP_TRY(enqueue_swap_iteration<T>(D, ld, L, medoids, opt, ws, s,
                                                      pool ? pool->ev[2 * j] : nullptr,
                                                      pool ? pool->ev[2 * j + 1] : nullptr));
            }
            enq += b;
            rc = read_state(L, ws, xs, &st);
            if (rc) return rc;
            if (pool) {
                // passes of iterations that ran (later ones returned at once)
                const int ran = st.iter - iter0;
                ms_pass += pool->sum(ran);
                n_pass += ran;
            }
            if (st.done) break;
            if (batch < kMaxBatch) batch *= 2;
        }
        if (g) {   // the caller's stream continues after the replays
            HIP_TRY(hipEventRecord(g->join, xs));
            HIP_TRY(hipStreamWaitEvent(s, g->join, 0));
        }
    }
    tm.rec(3, s);
    HIP_TRY(enqueue_finalize<T>(D, ld, L, medoids, labels, ws, s));
    rc = read_state(L, ws, s, &st);
    if (rc) return rc;
    if (st.sync_err) return fail(PAMX_ERR_HIP, "eager apply: a grid barrier wait expired");
    if (td) *td = st.td;
    if (stats) {
        stats->iterations = st.iter;
        stats->swaps = st.swaps;
        stats->converged = searches ? (st.done && !st.capped) : 1;
        stats->rescored = st.rescored;
        stats->td = st.td;
        stats->pass_pairs = (int64_t)st.iter * n * (L.nc - k);
        stats->ms_swap_pass = ms_pass;
        stats->n_swap_pass = n_pass;
        stats->chunk = L.L;
        if (scan) {
            // passes begun over the candidates; every window pass reads all n
            // objects for its candidates
            stats->iterations = searches ? (int32_t)((st.fp_visited + n - 1) / n) : 0;
            stats->windows = searches ? st.iter : 0;
            stats->window = L.fw;
            stats->scan_positions = searches ? st.fp_visited : 0;
            stats->pass_pairs = searches ? st.fp_cols * n : 0;
        }
    }
    return st.capped ? PAMX_WARN_MAXITER : PAMX_OK;
}

// One FastCLARANS local search (Sec. 3.4) over the caller's draws.
template <typename T>
int clarans_impl(const T *D, int64_t ld, const Layout &L, int32_t k, const int32_t *draws,
                 int64_t len, int64_t maxneighbor, const pamx_options &opt, int32_t *medoids,
                 int32_t *labels, double *td, pamx_stats *stats, void *ws, hipStream_t s,
                 Timer &tm) {
    const int64_t n = L.n;
    HIP_TRY(enqueue_swap_init<T>(D, ld, L, medoids, opt, ws, s));
    DevState st;
    int rc = read_state(L, ws, s, &st);
    if (rc) return rc;
    if (st.bad_medoids)
        return fail(PAMX_ERR_INVALID_MEDOIDS, "medoids must be distinct and in [0, n)");
    const bool searches = k >= 2 && k < n;
    if (searches) {
        // every draw in [0, n) before the search starts
        int32_t *err = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + L.cl_i);
        int32_t e0 = 0;
        HIP_TRY(launch_init_zero(err, s));
        HIP_TRY(launch_check_sidx(draws, len, n, err, s));
        HIP_TRY(hipMemcpyAsync(&e0, err, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (e0) return fail(PAMX_ERR_ARG, "draws holds an index outside [0, n)");
        HIP_TRY(enqueue_swap_caches<T>(D, ld, L, medoids, ws, s));
        HIP_TRY(enqueue_cl_init<T>(L, len, maxneighbor, ws, s));
    }
    tm.rec(2, s);
    if (searches) {
        int batch = 4;
        for (;;) {
            for (int j = 0; j < batch; ++j)
                HIP_TRY(enqueue_cl_step<T>(D, ld, L, draws, medoids, opt, ws, s));
            rc = read_state(L, ws, s, &st);
            if (rc) return rc;
            if (st.done) break;
            if (batch < 32) batch *= 2;
        }
    }
    tm.rec(3, s);
    HIP_TRY(enqueue_finalize<T>(D, ld, L, medoids, labels, ws, s));
    DevState fin;
    rc = read_state(L, ws, s, &fin);
    if (rc) return rc;
    if (td) *td = fin.td;
    if (stats) {
        stats->iterations = searches ? st.iter : 0;
        stats->windows = searches ? st.iter : 0;
        stats->swaps = searches ? st.swaps : 0;
        stats->converged = searches ? (st.done && !st.capped) : 1;
        stats->td = fin.td;
        stats->scan_positions = searches ? st.fp_cols : 0;
        stats->pass_pairs = searches ? st.fp_cols * n : 0;
        stats->window = 1024;
    }
    return (searches && st.capped) ? PAMX_WARN_MAXITER : PAMX_OK;
}

}  // namespace

// The mixed-precision form: BUILD and FastPAM1 on recomputed BF16-Gram
// distances with FP64 re-scoring (precision.hip).
static int fit_rc(const float *X, int64_t n, int32_t dim, int32_t k, const pamx_options &opt,
                  int32_t *medoids, int32_t *labels, double *td, pamx_stats *stats, void *ws,
                  size_t ws_bytes, hipStream_t s) {
    RcLayout R;
    make_rc_layout(n, k, dim, &opt, &R);
    if (!ws) return fail(PAMX_ERR_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < R.total)
        return fail(PAMX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, R.total);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    char *w = static_cast<char *>(ws);
    Timer tm;
    tm.rec(0, s);
    float *mean = reinterpret_cast<float *>(w + R.mean);
    HIP_TRY(launch_mean_f32(X, n, dim, mean, s));
    tm.rec(1, s);
    HIP_TRY(rc_prep_build(X, dim, R, k, opt, medoids, ws, s, mean));
    HIP_TRY(rc_td(R, ws, s));
    DevState st;
    const Layout fake = [&] { Layout L; std::memset(&L, 0, sizeof(L)); L.state = R.state; return L; }();
    int rc = read_state(fake, ws, s, &st);
    if (rc) return rc;
    if (st.bad_medoids) return fail(PAMX_ERR_HIP, "BUILD found no candidate");
    const double td_build = st.td;
    const int build_rescored = st.rescored;
    tm.rec(2, s);
    double ms_pass = 0.0;
    int n_pass = 0;
    HIP_TRY(rc_swap_init(X, dim, R, medoids, opt, ws, s));
    if (k >= 2 && k < n) {
        constexpr int kMaxBatch = 16;
        std::unique_ptr<EventPool> pool;
        if (opt.profile) {
            pool.reset(new EventPool(2 * kMaxBatch));
            if (!pool->ok()) return fail(PAMX_ERR_HIP, "hipEventCreate failed");
        }
        int batch = 2, enq = 0;
        st.iter = 0;
        for (;;) {
            int b = batch;
            if (b > opt.max_iter + 1 - enq) b = opt.max_iter + 1 - enq;
            if (b < 1) b = 1;
            const int iter0 = st.iter;
            for (int j = 0; j < b; ++j)
                HIP_TRY(rc_swap_iteration(X, dim, R, medoids, opt, ws, s,
                                          pool ? pool->ev[2 * j] : nullptr,
                                          pool ? pool->ev[2 * j + 1] : nullptr));
            enq += b;
            rc = read_state(fake, ws, s, &st);
            if (rc) return rc;
            if (pool) {
                const int ran = st.iter - iter0;
                ms_pass += pool->sum(ran);
                n_pass += ran;
            }
            if (st.done) break;
            if (batch < kMaxBatch) batch *= 2;
        }
    } else {
        st.iter = 0; st.swaps = 0; st.capped = 0;
    }
    tm.rec(3, s);
    HIP_TRY(rc_finalize(X, dim, R, medoids, labels, ws, s));
    DevState fin;
    rc = read_state(fake, ws, s, &fin);
    if (rc) return rc;
    tm.rec(4, s);
    HIP_TRY(hipStreamSynchronize(s));
    if (td) *td = fin.td;
    if (stats) {
        stats->iterations = st.iter;
        stats->swaps = st.swaps;
        stats->converged = (k >= 2 && k < n) ? (st.done && !st.capped) : 1;
        stats->rescored = st.rescored + build_rescored;
        stats->td_build = td_build;
        stats->td = fin.td;
        stats->ms_dist = tm.ms(0, 1);
        stats->ms_build = tm.ms(1, 2);
        stats->ms_swap = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 4);
        stats->pass_pairs = (int64_t)st.iter * n * (n - k);
        stats->build_pairs = (int64_t)k * n * n;
        stats->ms_swap_pass = ms_pass;
        stats->n_swap_pass = n_pass;
    }
    return st.capped ? PAMX_WARN_MAXITER : PAMX_OK;
}

static int swap_args(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                     const pamx_options *opt, const int32_t *medoids) {
    int rc = check_common(n, k, dtype, opt);
    if (rc) return rc;
    rc = check_matrix(D, n, ld);
    if (rc) return rc;
    if (!medoids) return fail(PAMX_ERR_ARG, "medoids is NULL");
    if (opt && opt->trace_cap > 0 && !opt->trace)
        return fail(PAMX_ERR_ARG, "trace_cap > 0 needs a trace array");
    return PAMX_OK;
}

extern "C" int pamx_build(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                          const pamx_options *opt_in, int32_t *medoids, double *td, void *ws,
                          size_t ws_bytes, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = swap_args(D, dtype, n, ld, k, &opt, medoids);
    if (rc) return rc;
    Layout L;
    make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D);
    rc = check_ws(ws, ws_bytes, L, &opt);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == PAMX_F32)
        return build_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, td, ws, s,
                                 nullptr);
    return build_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids, td, ws, s,
                               nullptr);
}

extern "C" int pamx_swap(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                         const pamx_options *opt_in, int32_t *medoids, int32_t *labels, double *td,
                         pamx_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = swap_args(D, dtype, n, ld, k, &opt, medoids);
    if (rc) return rc;
    Layout L;
    make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D);
    rc = check_ws(ws, ws_bytes, L, &opt);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Timer tm;
    tm.rec(0, s);
    if (dtype == PAMX_F32)
        rc = swap_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, labels, td,
                              stats, ws, s, tm);
    else
        rc = swap_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids, labels, td,
                                stats, ws, s, tm);
    if (rc < 0) return rc;
    tm.rec(4, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PAMX_ERR_HIP, "stream synchronize failed");
    if (stats) {
        stats->ms_swap = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 4);
    }
    return rc;
}

// ---------------------------------------------------------------- SWAP with no allocation
// pamx_swap for callers that cannot allocate: the workspace is a fixed
// device array of this library instead of a caller's buffer.  Each GPU the
// library runs on holds its own copy until the process ends; every call on
// that GPU reuses it (calls that overlap on one GPU race).  Every region the
// SWAP kernels read is written by the same call first (state, caches,
// segments, partials), so what the previous call left there does not matter.
static __device__ __align__(256) unsigned char scratch[PAMX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevs = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kScratchDevs] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device (with it current) and kept.  Host code uses only this
// address: the array's name on the host is a stand-in, not device memory.
int scratch_on_device(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevs)
        return fail(PAMX_ERR_HIP, "device %d beyond the %d devices with a scratch address", dev,
                    kScratchDevs);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PAMX_ERR_HIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return PAMX_OK;
}
}  // namespace

extern "C" int pamx_swap_noalloc(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                                 const pamx_options *opt_in, int32_t *medoids, int32_t *labels,
                                 double *td, pamx_stats *stats, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = swap_args(D, dtype, n, ld, k, &opt, medoids);
    if (rc) return rc;
    // each of these creates HIP events or graphs
    if (opt.profile) return fail(PAMX_ERR_ARG, "pamx_swap_noalloc: profile must be 0");
    if (opt.graph) return fail(PAMX_ERR_ARG, "pamx_swap_noalloc: graph must be 0");
    if (opt.chunk == PAMX_CHUNK_TUNE)
        return fail(PAMX_ERR_ARG, "pamx_swap_noalloc: no chunk tuning (PAMX_CHUNK_TUNE)");
    Layout L;
    make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D);
    const size_t need = layout_need(L, &opt);
    if (need > (size_t)PAMX_NOALLOC_SCRATCH_BYTES)
        return fail(PAMX_ERR_WORKSPACE,
                    "pamx_swap_noalloc: these arguments need %zu bytes of scratch, more than its "
                    "fixed %zu (use pamx_swap with a workspace)",
                    need, (size_t)PAMX_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    rc = scratch_on_device(&ws);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Timer tm(false);
    if (dtype == PAMX_F32)
        rc = swap_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, labels, td,
                              stats, ws, s, tm);
    else
        rc = swap_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids, labels, td,
                                stats, ws, s, tm);
    if (rc < 0) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PAMX_ERR_HIP, "stream synchronize failed");
    return rc;
}

extern "C" int pamx_clarans(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                            const int32_t *draws, int64_t len, int64_t maxneighbor,
                            const pamx_options *opt_in, int32_t *medoids, int32_t *labels,
                            double *td, pamx_stats *stats, void *ws, size_t ws_bytes,
                            void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = swap_args(D, dtype, n, ld, k, &opt, medoids);
    if (rc) return rc;
    if (len < 0) return fail(PAMX_ERR_ARG, "len must be >= 0");
    if (len > 0 && !draws) return fail(PAMX_ERR_ARG, "draws is NULL");
    if (maxneighbor < 1) return fail(PAMX_ERR_ARG, "maxneighbor must be >= 1");
    if (opt.variant != PAMX_FASTPAM1)
        return fail(PAMX_ERR_ARG, "pamx_clarans takes no SWAP variant (leave PAMX_FASTPAM1)");
    Layout L;
    make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D);
    rc = check_ws(ws, ws_bytes, L, &opt);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Timer tm;
    tm.rec(0, s);
    tm.rec(1, s);
    if (dtype == PAMX_F32)
        rc = clarans_impl<float>(static_cast<const float *>(D), ld, L, k, draws, len, maxneighbor,
                                 opt, medoids, labels, td, stats, ws, s, tm);
    else
        rc = clarans_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, draws, len,
                                   maxneighbor, opt, medoids, labels, td, stats, ws, s, tm);
    if (rc < 0) return rc;
    tm.rec(4, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PAMX_ERR_HIP, "stream synchronize failed");
    if (stats) {
        stats->ms_swap = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 4);
    }
    return rc;
}

// ---------------------------------------------------------------- best of several searches
// Restarts (Sec. 3.3: cheap starts, then SWAP, several times) and FastCLARANS's
// numlocal searches (Sec. 3.4) keep the local optimum of smallest TD.  The
// searches run one after another on the caller's stream, each in the SWAP
// workspace; behind it sit the working medoids (k int32) and labels (n int32)
// of the current search.  The result of the smallest TD is copied out, the
// lowest search index on ties.
static size_t best_of_bytes(const Layout &L, const pamx_options *opt) {
    return up256(layout_need(L, opt)) + up256((size_t)L.k * 4) + up256((size_t)L.n * 4);
}

extern "C" int pamx_best_of_workspace_bytes(int64_t n, int32_t k, int32_t dtype,
                                            const pamx_options *opt, size_t *bytes) {
    if (!bytes) return fail(PAMX_ERR_ARG, "bytes is NULL");
    int rc = check_common(n, k, dtype, opt);
    if (rc) return rc;
    size_t need = 0;
    for (int64_t ld : {(n + 3) & ~int64_t(3), (n % 4) ? n : n + 1}) {
        Layout L;
        make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, opt, &L, nullptr);
        need = std::max(need, best_of_bytes(L, opt));
    }
    *bytes = need;
    return PAMX_OK;
}

// search(r, medoids_work, labels_work, &td, &stats) runs search r in place
template <typename F>
static int best_of(const Layout &L, int32_t R, const int32_t *starts, const pamx_options &opt,
                   int32_t *medoids, int32_t *labels, double *td, pamx_stats *stats,
                   double *each_td, int32_t *best, void *ws, size_t ws_bytes, hipStream_t s,
                   F &&search) {
    const int32_t k = L.k;
    if (!ws) return fail(PAMX_ERR_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t need = best_of_bytes(L, &opt);
    if (ws_bytes < need)
        return fail(PAMX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    char *w = static_cast<char *>(ws);
    int32_t *wmed = reinterpret_cast<int32_t *>(w + up256(layout_need(L, &opt)));
    int32_t *wlab = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(wmed) + up256((size_t)k * 4));
    double best_td = 0.0;
    int32_t best_r = -1, best_rc = PAMX_OK;
    pamx_stats best_st;
    std::memset(&best_st, 0, sizeof(best_st));
    Timer tm;
    tm.rec(0, s);
    for (int32_t r = 0; r < R; ++r) {
        HIP_TRY(hipMemcpyAsync(wmed, starts + (size_t)r * k, (size_t)k * 4, hipMemcpyDeviceToDevice, s));
        double tdr = 0.0;
        pamx_stats st;
        std::memset(&st, 0, sizeof(st));
        const int rc = search(r, wmed, labels ? wlab : nullptr, &tdr, &st);
        if (rc < 0) return rc;
        if (each_td) each_td[r] = tdr;
        if (best_r < 0 || tdr < best_td) {
            best_td = tdr;
            best_r = r;
            best_rc = rc;
            best_st = st;
            HIP_TRY(hipMemcpyAsync(medoids, wmed, (size_t)k * 4, hipMemcpyDeviceToDevice, s));
            if (labels)
                HIP_TRY(hipMemcpyAsync(labels, wlab, (size_t)L.n * 4, hipMemcpyDeviceToDevice, s));
        }
    }
    tm.rec(4, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PAMX_ERR_HIP, "stream synchronize failed");
    if (td) *td = best_td;
    if (best) *best = best_r;
    if (stats) {
        *stats = best_st;
        stats->ms_total = tm.ms(0, 4);
    }
    return best_rc;
}

extern "C" int pamx_swap_restarts(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                                  int32_t restarts, const int32_t *starts,
                                  const pamx_options *opt_in, int32_t *medoids, int32_t *labels,
                                  double *td, pamx_stats *stats, double *restart_td,
                                  int32_t *best, void *ws, size_t ws_bytes, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = swap_args(D, dtype, n, ld, k, &opt, medoids);
    if (rc) return rc;
    if (restarts < 1) return fail(PAMX_ERR_ARG, "restarts must be >= 1");
    if (!starts) return fail(PAMX_ERR_ARG, "starts is NULL");
    Layout L;
    make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto one = [&](int32_t, int32_t *wmed, int32_t *wlab, double *tdr, pamx_stats *st) {
        Timer t;
        t.rec(0, s);
        const int r = dtype == PAMX_F32
                          ? swap_impl<float>(static_cast<const float *>(D), ld, L, k, opt, wmed, wlab,
                                             tdr, st, ws, s, t)
                          : swap_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, wmed,
                                               wlab, tdr, st, ws, s, t);
        if (r >= 0) st->ms_swap = t.ms(2, 3);
        return r;
    };
    return best_of(L, restarts, starts, opt, medoids, labels, td, stats, restart_td, best, ws,
                   ws_bytes, s, one);
}

extern "C" int pamx_clarans_numlocal(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                                     int32_t numlocal, const int32_t *starts, const int32_t *draws,
                                     int64_t len, int64_t maxneighbor, const pamx_options *opt_in,
                                     int32_t *medoids, int32_t *labels, double *td,
                                     pamx_stats *stats, double *search_td, int32_t *best, void *ws,
                                     size_t ws_bytes, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = swap_args(D, dtype, n, ld, k, &opt, medoids);
    if (rc) return rc;
    if (numlocal < 1) return fail(PAMX_ERR_ARG, "numlocal must be >= 1");
    if (!starts) return fail(PAMX_ERR_ARG, "starts is NULL");
    if (len < 0) return fail(PAMX_ERR_ARG, "len must be >= 0");
    if (len > 0 && !draws) return fail(PAMX_ERR_ARG, "draws is NULL");
    if (maxneighbor < 1) return fail(PAMX_ERR_ARG, "maxneighbor must be >= 1");
    if (opt.variant != PAMX_FASTPAM1)
        return fail(PAMX_ERR_ARG, "FastCLARANS takes no SWAP variant (leave PAMX_FASTPAM1)");
    if (opt.trace_cap > 0)
        return fail(PAMX_ERR_ARG, "no swap trace over several searches (trace_cap must be 0)");
    Layout L;
    make_layout(n, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto one = [&](int32_t r, int32_t *wmed, int32_t *wlab, double *tdr, pamx_stats *st) {
        Timer t;
        t.rec(0, s);
        const int32_t *dr = draws ? draws + (size_t)r * len : nullptr;
        const int c = dtype == PAMX_F32
                          ? clarans_impl<float>(static_cast<const float *>(D), ld, L, k, dr, len,
                                                maxneighbor, opt, wmed, wlab, tdr, st, ws, s, t)
                          : clarans_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, dr, len,
                                                  maxneighbor, opt, wmed, wlab, tdr, st, ws, s, t);
        if (c >= 0) st->ms_swap = t.ms(2, 3);
        return c;
    };
    return best_of(L, numlocal, starts, opt, medoids, labels, td, stats, search_td, best, ws,
                   ws_bytes, s, one);
}

// ---------------------------------------------------------------- bichromatic medoids
static int rect_args(const void *D, int32_t dtype, int64_t nco, int64_t nl, int64_t ld, int32_t k,
                     const pamx_options *opt, const int32_t *medoids) {
    if (nco < 1 || nco > (int64_t)INT32_MAX - 1) return fail(PAMX_ERR_ARG, "n_cons out of range");
    if (nl < 1 || nl > (int64_t)INT32_MAX - 1) return fail(PAMX_ERR_ARG, "n_loc out of range");
    int rc = check_common(nl, k, dtype, opt);
    if (rc) return rc;
    rc = check_matrix(D, nl, ld);
    if (rc) return rc;
    if (nco > ((int64_t)1 << 62) / ld) return fail(PAMX_ERR_ARG, "n_cons * ld overflows");
    if (!medoids) return fail(PAMX_ERR_ARG, "medoids is NULL");
    if (opt) {
        if (opt->variant != PAMX_FASTPAM1)
            return fail(PAMX_ERR_UNSUPPORTED, "a consumers x locations matrix runs FastPAM1 only");
        if (opt->dist_mode != PAMX_DIST_STORED || opt->chunk == PAMX_CHUNK_TUNE)
            return fail(PAMX_ERR_UNSUPPORTED, "no BF16 form or chunk tuning for a rectangular matrix");
        if (opt->trace_cap > 0 && !opt->trace) return fail(PAMX_ERR_ARG, "trace_cap > 0 needs a trace array");
    }
    return PAMX_OK;
}

extern "C" int pamx_rect_workspace_bytes(int64_t n_cons, int64_t n_loc, int32_t k, int32_t dtype,
                                         const pamx_options *opt, size_t *bytes) {
    if (!bytes) return fail(PAMX_ERR_ARG, "bytes is NULL");
    int32_t dummy = 0;
    int rc = rect_args(reinterpret_cast<const void *>(256), dtype, n_cons, n_loc, n_loc, k, opt,
                       &dummy);
    if (rc) return rc;
    Layout L;
    make_layout(n_cons, k, 0, PAMX_INPUT_D, dtype, (n_loc + 3) & ~int64_t(3), opt, &L, nullptr,
                n_loc);
    const size_t b4 = layout_need(L, opt);
    make_layout(n_cons, k, 0, PAMX_INPUT_D, dtype, (n_loc % 4) ? n_loc : n_loc + 1, opt, &L,
                nullptr, n_loc);
    const size_t b1 = layout_need(L, opt);
    *bytes = b4 > b1 ? b4 : b1;
    return PAMX_OK;
}

// BUILD (if `build`) and FastPAM1 SWAP on an n_cons x n_loc matrix.
static int rect_impl(const void *D, int32_t dtype, int64_t nco, int64_t nl, int64_t ld, int32_t k,
                     const pamx_options *opt_in, bool build, int32_t *medoids, int32_t *labels,
                     double *td, pamx_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = rect_args(D, dtype, nco, nl, ld, k, &opt, medoids);
    if (rc) return rc;
    opt.build_exclude_self = 0;   // no candidate is an object
    Layout L;
    make_layout(nco, k, 0, PAMX_INPUT_D, dtype, ld, &opt, &L, D, nl);
    rc = check_ws(ws, ws_bytes, L, &opt);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Timer tm;
    tm.rec(0, s);
    // the locations' distances to all consumers, one row per location
    HIP_TRY(launch_transpose(D, ld, nco, nl, static_cast<char *>(ws) + L.DT, L.ldt, s));
    tm.rec(1, s);
    double td_build = 0.0;
    pamx_stats bst;
    std::memset(&bst, 0, sizeof(bst));
    if (build) {
        if (dtype == PAMX_F32)
            rc = build_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, &td_build,
                                   ws, s, &bst);
        else
            rc = build_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids,
                                     &td_build, ws, s, &bst);
        if (rc) return rc;
    }
    if (dtype == PAMX_F32)
        rc = swap_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, labels, td,
                              stats, ws, s, tm);
    else
        rc = swap_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids, labels, td,
                                stats, ws, s, tm);
    if (rc < 0) return rc;
    tm.rec(4, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PAMX_ERR_HIP, "stream synchronize failed");
    if (stats) {
        stats->td_build = td_build;
        stats->ms_dist = tm.ms(0, 1);
        stats->ms_build = tm.ms(1, 2);
        stats->ms_swap = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 4);
        stats->build_pairs = bst.build_pairs;
        stats->build_rows = bst.build_rows;
        stats->ms_build_pass = bst.ms_build_pass;
        stats->n_build_pass = bst.n_build_pass;
        stats->ms_build_delta = bst.ms_build_delta;
        stats->n_build_delta = bst.n_build_delta;
    }
    return rc;
}

extern "C" int pamx_fit_rect(const void *D, int32_t dtype, int64_t n_cons, int64_t n_loc,
                             int64_t ld, int32_t k, const pamx_options *opt, int32_t *medoids,
                             int32_t *labels, double *td, pamx_stats *stats, void *ws,
                             size_t ws_bytes, void *stream) {
    return rect_impl(D, dtype, n_cons, n_loc, ld, k, opt, true, medoids, labels, td, stats, ws,
                     ws_bytes, stream);
}

extern "C" int pamx_swap_rect(const void *D, int32_t dtype, int64_t n_cons, int64_t n_loc,
                              int64_t ld, int32_t k, const pamx_options *opt, int32_t *medoids,
                              int32_t *labels, double *td, pamx_stats *stats, void *ws,
                              size_t ws_bytes, void *stream) {
    return rect_impl(D, dtype, n_cons, n_loc, ld, k, opt, false, medoids, labels, td, stats, ws,
                     ws_bytes, stream);
}

// ---------------------------------------------------------------- faster initialisations
extern "C" int pamx_init_workspace_bytes(int64_t n, int32_t m, size_t *bytes) {
    if (!bytes) return fail(PAMX_ERR_ARG, "bytes is NULL");
    if (n < 1 || n > (int64_t)INT32_MAX - 1) return fail(PAMX_ERR_ARG, "n out of range");
    if (m < 0 || m > n) return fail(PAMX_ERR_ARG, "m must be in [0, n]");
    *bytes = make_init_layout(n, m).total;
    return PAMX_OK;
}

static int init_args(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                     const int32_t *medoids, const void *ws, size_t ws_bytes, int32_t m) {
    if (n < 1 || n > (int64_t)INT32_MAX - 1) return fail(PAMX_ERR_ARG, "n out of range");
    if (k < 1 || k > n) return fail(PAMX_ERR_ARG, "k must be in [1, n]");
    if (dtype != PAMX_I32 && dtype != PAMX_F32) return fail(PAMX_ERR_ARG, "unknown dtype %d", dtype);
    int rc = check_matrix(D, n, ld);
    if (rc) return rc;
    if (!medoids) return fail(PAMX_ERR_ARG, "medoids is NULL");
    if (!ws) return fail(PAMX_ERR_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t need = make_init_layout(n, m).total;
    if (ws_bytes < need)
        return fail(PAMX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    return PAMX_OK;
}

extern "C" int pamx_init_dw(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                            const double *u, int32_t *medoids, void *ws, size_t ws_bytes,
                            void *stream) {
    int rc = init_args(D, dtype, n, ld, k, medoids, ws, ws_bytes, 0);
    if (rc) return rc;
    if (!u) return fail(PAMX_ERR_ARG, "u is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == PAMX_F32)
        HIP_TRY(launch_init_dw<float>(static_cast<const float *>(D), ld, n, k, u, medoids, ws, s));
    else
        HIP_TRY(launch_init_dw<int32_t>(static_cast<const int32_t *>(D), ld, n, k, u, medoids, ws, s));
    return PAMX_OK;
}

extern "C" int pamx_init_lab(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t k,
                             const int32_t *samples, int32_t m, int32_t exclude_self,
                             int32_t *medoids, void *ws, size_t ws_bytes, void *stream) {
    if (m < 1 || m > n) return fail(PAMX_ERR_ARG, "m must be in [1, n]");
    int rc = init_args(D, dtype, n, ld, k, medoids, ws, ws_bytes, m);
    if (rc) return rc;
    if (!samples) return fail(PAMX_ERR_ARG, "samples is NULL");
    if (exclude_self != 0 && exclude_self != 1) return fail(PAMX_ERR_ARG, "exclude_self must be 0 or 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every listed index in [0, n) before any step runs
    {
        int32_t *err = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + make_init_layout(n, m).err);
        int32_t e0 = 0;
        HIP_TRY(launch_init_zero(err, s));
        HIP_TRY(launch_check_sidx(samples, (int64_t)k * m, n, err, s));
        HIP_TRY(hipMemcpyAsync(&e0, err, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (e0) return fail(PAMX_ERR_ARG, "samples holds an index outside [0, n)");
    }
    if (dtype == PAMX_F32)
        HIP_TRY(launch_init_lab<float>(static_cast<const float *>(D), ld, n, k, samples, m,
                                       exclude_self, medoids, ws, s));
    else
        HIP_TRY(launch_init_lab<int32_t>(static_cast<const int32_t *>(D), ld, n, k, samples, m,
                                         exclude_self, medoids, ws, s));
    return PAMX_OK;
}

extern "C" int pamx_fit(const void *XorD, int32_t input_kind, int32_t dtype, int64_t n, int32_t dim,
                        int32_t metric, int32_t k, const pamx_options *opt_in, int32_t *medoids,
                        int32_t *labels, double *td, pamx_stats *stats, void *ws, size_t ws_bytes,
                        void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int rc = check_common(n, k, dtype, &opt);
    if (rc) return rc;
    if (input_kind != PAMX_INPUT_D && input_kind != PAMX_INPUT_X)
        return fail(PAMX_ERR_ARG, "unknown input_kind %d", input_kind);
    if (input_kind == PAMX_INPUT_X) {
        rc = check_points(XorD, dtype, n, dim, metric);
        if (rc) return rc;
    } else {
        rc = check_matrix(XorD, n, n);
        if (rc) return rc;
    }
    if (!medoids) return fail(PAMX_ERR_ARG, "medoids is NULL");
    if (opt.trace_cap > 0 && !opt.trace) return fail(PAMX_ERR_ARG, "trace_cap > 0 needs a trace array");
    if (opt.dist_mode == PAMX_DIST_BF16) {
        rc = check_rc(input_kind, dtype, metric, dim, k, &opt);
        if (rc) return rc;
        return fit_rc(static_cast<const float *>(XorD), n, dim, k, opt, medoids, labels, td, stats, ws,
                      ws_bytes, static_cast<hipStream_t>(stream));
    }
    Layout L;
    make_layout(n, k, dim, input_kind, dtype, n, &opt, &L,
                input_kind == PAMX_INPUT_D ? XorD : nullptr);
    rc = check_ws(ws, ws_bytes, L, &opt);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Timer tm;
    tm.rec(0, s);
    const void *D = XorD;
    int64_t ld = n;
    if (input_kind == PAMX_INPUT_X) {
        char *w = static_cast<char *>(ws);
        void *Dw = w + L.D;
        ld = L.ld_fit;
        rc = dist_impl(XorD, dtype, n, dim, metric, Dw, ld, w + L.mean, s);
        if (rc) return rc;
        D = Dw;
    }
    tm.rec(1, s);
    double td_build = 0.0;
    pamx_stats bst;
    std::memset(&bst, 0, sizeof(bst));
    if (dtype == PAMX_F32)
        rc = build_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, &td_build, ws, s,
                               &bst);
    else
        rc = build_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids, &td_build,
                                 ws, s, &bst);
    if (rc) return rc;
    if (dtype == PAMX_F32)
        rc = swap_impl<float>(static_cast<const float *>(D), ld, L, k, opt, medoids, labels, td, stats,
                              ws, s, tm);
    else
        rc = swap_impl<int32_t>(static_cast<const int32_t *>(D), ld, L, k, opt, medoids, labels, td,
                                stats, ws, s, tm);
    if (rc < 0) return rc;
    tm.rec(4, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PAMX_ERR_HIP, "stream synchronize failed");
    if (stats) {
        stats->td_build = td_build;
        stats->ms_dist = tm.ms(0, 1);
        stats->ms_build = tm.ms(1, 2);
        stats->ms_swap = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 4);
        stats->build_pairs = bst.build_pairs;
        stats->build_rows = bst.build_rows;
        stats->ms_build_pass = bst.ms_build_pass;
        stats->n_build_pass = bst.n_build_pass;
        stats->ms_build_delta = bst.ms_build_delta;
        stats->n_build_delta = bst.n_build_delta;
    }
    return rc;
}

// ---------------------------------------------------------------- batched CLARA
namespace {
constexpr int kFullBlocks = 256;   // blocks per instance in the full-data TD
// team scales (percent of the cost-balanced team sizes; 0 = no teams) timed
// by the batched form's tuning
constexpr int kTeamScales[] = {100, 0, 50, 200};
struct BatchTuneKey {
    int dev;
    int32_t n_inst, dim, dtype, max_iter, excl;
    int64_t N;
    uint64_t shape;
    bool operator<(const BatchTuneKey &o) const {
        return std::tie(dev, n_inst, dim, dtype, max_iter, excl, N, shape) <
               std::tie(o.dev, o.n_inst, o.dim, o.dtype, o.max_iter, o.excl, o.N, o.shape);
    }
};
std::mutex g_btune_mu;
std::map<BatchTuneKey, int> g_btuned;

struct BatchLayout {
    size_t soff, kin, moff, tk_inst, tk_mem, tsz, bar, xch, td, tdb, it, sw, rows, ctr, part, tdf,
        range, total;
};

BatchLayout batch_layout(int32_t n_inst) {
    BatchLayout b;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = up256(off + (bytes ? bytes : 1)); return o; };
    b.soff = take((size_t)(n_inst + 1) * 8);
    b.kin = take((size_t)n_inst * 4);
    b.moff = take((size_t)(n_inst + 1) * 8);
    b.tk_inst = take((size_t)n_inst * kBTeamMax * 4);
    b.tk_mem = take((size_t)n_inst * kBTeamMax * 4);
    b.tsz = take((size_t)n_inst * 4);
    b.bar = take((size_t)n_inst * 4);
    b.xch = take((size_t)n_inst * kBTeamSlots * 8);
    b.td = take((size_t)n_inst * 8);
    b.tdb = take((size_t)n_inst * 8);
    b.it = take((size_t)n_inst * 4);
    b.sw = take((size_t)n_inst * 4);
    b.rows = take((size_t)n_inst * 4);
    b.ctr = take(2 * 4);
    b.part = take((size_t)n_inst * kFullBlocks * 8);
    b.tdf = take((size_t)n_inst * 8);
    b.range = take((size_t)2 * kBMaxDim * 4);   // int32 points: coordinate ranges
    b.total = off;
    return b;
}
}  // namespace

extern "C" int pamx_batched_workspace_bytes(int32_t n_inst, int64_t N, size_t *bytes) {
    if (!bytes) return fail(PAMX_ERR_ARG, "bytes is NULL");
    if (n_inst < 1) return fail(PAMX_ERR_ARG, "n_inst must be >= 1");
    if (N < 1) return fail(PAMX_ERR_ARG, "N must be >= 1");
    *bytes = batch_layout(n_inst).total;
    return PAMX_OK;
}

namespace pamx {
template <typename X>
__global__ void k_fill_batch(X *p, int64_t cnt, X v) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < cnt) p[t] = v;
}
}  // namespace pamx

extern "C" int pamx_fit_batched(const void *X, int32_t dtype, int64_t N, int32_t dim, int32_t metric,
                                int32_t n_inst, const int64_t *sample_off, const int32_t *sample_idx,
                                const int32_t *k_inst, const pamx_options *opt_in, int32_t *medoids,
                                double *td_sample, double *td_full, pamx_batch_stats *stats,
                                void *ws, size_t ws_bytes, void *stream) {
    pamx_options opt;
    pamx_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (dtype != PAMX_I32 && dtype != PAMX_F32) return fail(PAMX_ERR_ARG, "unknown dtype %d", dtype);
    if (N < 1 || N > (int64_t)INT32_MAX - 1) return fail(PAMX_ERR_ARG, "N out of range");
    int rc = check_points(X, dtype, N, dim, metric);
    if (rc) return rc;
    if (dim > kBMaxDim) return fail(PAMX_ERR_UNSUPPORTED, "batched instances support dim <= %d", kBMaxDim);
    if (n_inst < 1) return fail(PAMX_ERR_ARG, "n_inst must be >= 1");
    if (!sample_off || !sample_idx || !k_inst || !medoids || !td_sample)
        return fail(PAMX_ERR_ARG, "NULL argument");
    if (opt.max_iter < 0) return fail(PAMX_ERR_ARG, "max_iter must be >= 0");
    if (opt.build_exclude_self != 0 && opt.build_exclude_self != 1)
        return fail(PAMX_ERR_ARG, "build_exclude_self must be 0 or 1");
    if (sample_off[0] != 0) return fail(PAMX_ERR_ARG, "sample_off[0] must be 0");
    int n_max = 0, k_max = 0;
    std::vector<int64_t> moff(n_inst + 1, 0);
    std::vector<std::pair<double, int32_t>> cost(n_inst);
    for (int32_t j = 0; j < n_inst; ++j) {
        const int64_t nj = sample_off[j + 1] - sample_off[j];
        const int32_t kj = k_inst[j];
        if (nj < 1) return fail(PAMX_ERR_ARG, "instance %d has an empty sample", j);
        if (nj > kBMaxN) return fail(PAMX_ERR_UNSUPPORTED, "instance %d: sample of %lld > %d points", j,
                                     (long long)nj, kBMaxN);
        if (kj < 1 || kj > nj) return fail(PAMX_ERR_ARG, "instance %d: k must be in [1, n']", j);
        if (kj > kBMaxK) return fail(PAMX_ERR_UNSUPPORTED, "instance %d: k > %d", j, kBMaxK);
        n_max = nj > n_max ? (int)nj : n_max;
        k_max = kj > k_max ? kj : k_max;
        moff[j + 1] = moff[j] + kj;
        cost[j] = {-(double)(kj + 8) * (double)nj * (double)nj, j};   // BUILD + ~8 SWAP passes
    }
    const size_t lds = batched_lds_bytes_host(n_max, k_max, dim, 4);
    if (lds > 150 * 1024)
        return fail(PAMX_ERR_UNSUPPORTED, "instance too large for one work-group's LDS (%zu B)", lds);
    std::sort(cost.begin(), cost.end());
    const BatchLayout B = batch_layout(n_inst);
    if (!ws) return fail(PAMX_ERR_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(PAMX_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < B.total) return fail(PAMX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes",
                                        ws_bytes, B.total);
    if (dtype == PAMX_I32) {   // the pool's ranges bound every sample's distances
        rc = check_l1_range(static_cast<const int32_t *>(X), N, dim,
                            reinterpret_cast<int32_t *>(static_cast<char *>(ws) + B.range),
                            static_cast<hipStream_t>(stream));
        if (rc) return rc;
    }
    // Teams: with cooperative launch, an instance whose estimated cost is a
    // multiple of the balanced share (total / resident work-groups) gets that
    // many work-groups (at most kBTeamMax, and at least 256 candidates each),
    // so the largest instances do not set the length of the launch.  `scale`
    // (percent) multiplies the team sizes; 0 turns teams off.  The results do
    // not depend on it: a team splits an instance's candidates, every
    // candidate's sums are formed by one lane in a fixed order, and the team
    // takes the same lexicographic minimum.
    int coop = 0;
    const int resident = batched_resident(dim, lds, dtype, &coop);
    if (resident < 1) return fail(PAMX_ERR_UNSUPPORTED, "the batched kernel does not fit a compute unit");
    double total_cost = 0.0;
    for (const auto &cj : cost) total_cost += -cj.first;

    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipMemcpyAsync(w + B.soff, sample_off, (size_t)(n_inst + 1) * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + B.kin, k_inst, (size_t)n_inst * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + B.moff, moff.data(), (size_t)(n_inst + 1) * 8, hipMemcpyHostToDevice, s));
    int32_t *ctr = reinterpret_cast<int32_t *>(w + B.ctr);

    BatchArgs a;
    a.soff = reinterpret_cast<const int64_t *>(w + B.soff);
    a.sidx = sample_idx;
    a.kin = reinterpret_cast<const int32_t *>(w + B.kin);
    a.moff = reinterpret_cast<const int64_t *>(w + B.moff);
    a.tk_inst = reinterpret_cast<const int32_t *>(w + B.tk_inst);
    a.tk_mem = reinterpret_cast<const int32_t *>(w + B.tk_mem);
    a.tsz = reinterpret_cast<const int32_t *>(w + B.tsz);
    a.bar = reinterpret_cast<int32_t *>(w + B.bar);
    a.xch = reinterpret_cast<unsigned long long *>(w + B.xch);
    a.n_inst = n_inst;
    a.max_iter = opt.max_iter;
    a.excl = opt.build_exclude_self;
    a.n_max = n_max;
    a.k_max = k_max;
    a.nblk = kFullBlocks;
    a.med_out = medoids;
    a.td_out = reinterpret_cast<double *>(w + B.td);
    a.tdb_out = reinterpret_cast<double *>(w + B.tdb);
    a.part = reinterpret_cast<double *>(w + B.part);
    a.td_full = reinterpret_cast<double *>(w + B.tdf);
    a.it_out = reinterpret_cast<int32_t *>(w + B.it);
    a.sw_out = reinterpret_cast<int32_t *>(w + B.sw);
    a.rows_out = reinterpret_cast<int32_t *>(w + B.rows);
    a.queue = ctr;
    a.err = ctr + 1;
    // tickets (largest estimated cost first), counters and the PAM launch
    // for one team scale
    std::vector<int32_t> tsz(n_inst), tk_inst, tk_mem;
    auto launch_pam = [&](int scale) -> hipError_t {
        std::fill(tsz.begin(), tsz.end(), 1);
        if (scale > 0 && coop && resident >= 2) {
            const double share = total_cost / resident;
            for (const auto &cj : cost) {
                const int32_t j = cj.second;
                const int64_t nj = sample_off[j + 1] - sample_off[j];
                int lim = (int)std::min<int64_t>(kBTeamMax, std::max<int64_t>(1, nj / 256));
                if (lim > resident) lim = resident;
                const int t = (int)std::llround(-cj.first / share * scale / 100.0);
                tsz[j] = t < 1 ? 1 : (t > lim ? lim : t);
            }
        }
        tk_inst.clear();
        tk_mem.clear();
        int32_t max_team = 1;
        for (const auto &cj : cost) {
            const int32_t j = cj.second;
            for (int32_t m = 0; m < tsz[j]; ++m) { tk_inst.push_back(j); tk_mem.push_back(m); }
            max_team = tsz[j] > max_team ? tsz[j] : max_team;
        }
        a.n_tick = (int32_t)tk_inst.size();
        a.coop = max_team > 1 ? 1 : 0;
        if (a.coop) a.grid = resident < a.n_tick ? resident : a.n_tick;   // all resident at once
        else a.grid = cus < n_inst ? cus : n_inst;
        hipError_t e;
        if ((e = hipMemcpyAsync(w + B.tk_inst, tk_inst.data(), (size_t)a.n_tick * 4,
                                hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(w + B.tk_mem, tk_mem.data(), (size_t)a.n_tick * 4,
                                hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(w + B.tsz, tsz.data(), (size_t)n_inst * 4, hipMemcpyHostToDevice,
                                s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fill_batch<int32_t>, dim3(1), dim3(1), 0, s, ctr, (int64_t)1, 0);   // queue
        hipLaunchKernelGGL(k_fill_batch<int32_t>, dim3((n_inst + 255) / 256), dim3(256), 0, s,
                           reinterpret_cast<int32_t *>(w + B.bar), (int64_t)n_inst, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return dtype == PAMX_F32 ? launch_clara<float>(static_cast<const float *>(X), N, dim, a, s)
                                 : launch_clara<int32_t>(static_cast<const int32_t *>(X), N, dim, a, s);
    };
    hipLaunchKernelGGL(k_fill_batch<int32_t>, dim3(1), dim3(256), 0, s, ctr, (int64_t)2, 0);
    HIP_TRY(hipGetLastError());

    // every sample index in [0, N) before any instance runs
    {
        int32_t e0 = 0;
        HIP_TRY(launch_check_sidx(sample_idx, sample_off[n_inst], N, ctr + 1, s));
        HIP_TRY(hipMemcpyAsync(&e0, ctr + 1, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (e0) return fail(PAMX_ERR_ARG, "sample_idx holds an index outside [0, N)");
    }
    // team scale: the default, or timed once per argument shape (chunk =
    // PAMX_CHUNK_TUNE) over kTeamScales and kept for the process
    int scale = 100;
    if (opt.chunk == PAMX_CHUNK_TUNE && coop && resident >= 2) {
        uint64_t hsh = 1469598103934665603ull;   // FNV-1a over the instance shapes
        auto mix = [&](uint64_t v) { hsh = (hsh ^ v) * 1099511628211ull; };
        for (int32_t j = 0; j <= n_inst; ++j) mix((uint64_t)sample_off[j]);
        for (int32_t j = 0; j < n_inst; ++j) mix((uint64_t)(uint32_t)k_inst[j]);
        const BatchTuneKey key{dev, n_inst, dim, dtype, opt.max_iter, opt.build_exclude_self, N, hsh};
        bool found = false;
        {
            std::lock_guard<std::mutex> g(g_btune_mu);
            auto it = g_btuned.find(key);
            if (it != g_btuned.end()) { scale = it->second; found = true; }
        }
        if (!found) {
            // one untimed launch first: the first launch of a process runs
            // cold (measured 20 ms against 16 for the same work)
            HIP_TRY(launch_pam(kTeamScales[0]));
            Timer tt;
            double best = 0.0;
            for (int sc : kTeamScales) {
                tt.rec(0, s);
                HIP_TRY(launch_pam(sc));
                tt.rec(1, s);
                int32_t e1 = 0;
                HIP_TRY(hipMemcpyAsync(&e1, ctr + 1, 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                if (e1 & 4) return fail(PAMX_ERR_HIP, "a team of the batched kernel did not meet (wait bound reached)");
                if (e1 & 8) return fail(PAMX_ERR_ARG, "an instance's BUILD found no finite distance sum "
                                                      "(non-finite point coordinates)");
                const double ms = tt.ms(0, 1);
                if (sc == kTeamScales[0] || ms < best) { best = ms; scale = sc; }
            }
            std::lock_guard<std::mutex> g(g_btune_mu);
            g_btuned[key] = scale;
        }
    }
    Timer tm;
    tm.rec(0, s);
    HIP_TRY(launch_pam(scale));
    tm.rec(1, s);
    if (td_full) {
        if (dtype == PAMX_F32) HIP_TRY(launch_full_assign<float>(static_cast<const float *>(X), N, dim, a, s));
        else HIP_TRY(launch_full_assign<int32_t>(static_cast<const int32_t *>(X), N, dim, a, s));
    }
    tm.rec(2, s);
    int32_t err = 0;
    std::vector<int32_t> it(n_inst), sw(n_inst), rows(n_inst);
    HIP_TRY(hipMemcpyAsync(&err, ctr + 1, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(td_sample, a.td_out, (size_t)n_inst * 8, hipMemcpyDeviceToHost, s));
    if (td_full) HIP_TRY(hipMemcpyAsync(td_full, a.td_full, (size_t)n_inst * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(it.data(), a.it_out, (size_t)n_inst * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sw.data(), a.sw_out, (size_t)n_inst * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rows.data(), a.rows_out, (size_t)n_inst * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & 4) return fail(PAMX_ERR_HIP, "a team of the batched kernel did not meet (wait bound reached)");
    if (err & 8) return fail(PAMX_ERR_ARG, "an instance's BUILD found no finite distance sum "
                                           "(non-finite point coordinates)");
    if (err) return fail(PAMX_ERR_HIP, "a medoid index outside [0, N) reached the full-data TD");
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        int64_t pairs = 0;
        for (int32_t j = 0; j < n_inst; ++j) {
            stats->iterations += it[j];
            stats->swaps += sw[j];
            const int64_t nj = sample_off[j + 1] - sample_off[j];
            const int64_t kj = k_inst[j];
            // BUILD: two full steps, then the rows of the changed objects;
            // SWAP: every non-medoid candidate against every object
            pairs += (kj < 2 ? kj : 2) * nj * nj + (int64_t)rows[j] * nj + it[j] * nj * (nj - kj);
        }
        stats->pairs = pairs;
        stats->best_inst = -1;
        if (td_full) {
            int32_t b = 0;
            for (int32_t j = 1; j < n_inst; ++j)
                if (td_full[j] < td_full[b]) b = j;
            stats->best_inst = b;
        }
        stats->team_scale = (coop && resident >= 2) ? scale : 0;
        stats->ms_pam = tm.ms(0, 1);
        stats->ms_assign = tm.ms(1, 2);
        stats->ms_total = tm.ms(0, 2);
    }
    for (int32_t j = 0; j < n_inst; ++j)
        if (it[j] > opt.max_iter - 1 && opt.max_iter > 0 && sw[j] >= it[j]) return PAMX_WARN_MAXITER;
    return PAMX_OK;
}
