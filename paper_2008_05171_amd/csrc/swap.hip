// swap.hip -- BUILD and SWAP kernels for gfx950.
//
// Paper: Schubert & Rousseeuw, "Fast and Eager k-Medoids Clustering",
// arXiv 2008.05171.  Notation: nearest(o), dn(o), ds(o) are the slot of and
// the distances to o's nearest and second-nearest medoid (Sec. 2).
//
// Loss change of swapping slot i with candidate c (Eq. better-change3):
//     Delta(i, c) = R_i + B(c) + S_i(c)
//     R_i  = sum_{nearest(o)=i} (ds - dn)                   removal loss
//     B(c) = sum_o min(d(o,c) - dn, 0)                      shared term
//     S_i  = sum_{nearest(o)=i} (med3(d(o,c), dn, ds) - ds) per-medoid term
// (med3(d, dn, ds) - ds is the three-way case of the paper's last sum, as
// dn <= ds).  For exact sums it is regrouped here into sums of non-negative
// terms that need no subtraction per pair:
//     B(c)            = A(c) - TD,        A(c)   = sum_o min(d(o,c), dn(o))
//     R_i + S_i(c)    = M_i(c) - DN_i,    M_i(c) = sum_{nearest(o)=i} med3(d, dn, ds)
//                                          DN_i   = sum_{nearest(o)=i} dn(o)
// so one pair costs min, med3 and two adds.
//
// Layout of the hot pass: objects are sorted by nearest slot (a stable
// counting sort), so the per-medoid sums M_i are segment sums over
// consecutive objects.  A work-group owns a tile of candidates (4 per lane,
// one 16-byte load of D per object) and a chunk of sorted objects; for each
// object it reads the contiguous candidate slice of row o of D (D symmetric,
// so row o holds d(o, c) for all c).  Per-object cache values are wave
// uniform.  Segments cut by a chunk edge leave partial sums ("carries") that
// a merge kernel adds in chunk order: every sum is formed in a fixed order,
// so results are deterministic.
#include <hip/hip_cooperative_groups.h>

#include "pamx_internal.h"

#ifndef PAMX_PSTAGE
#define PAMX_PSTAGE 8
#endif
#ifndef PAMX_PASS_WPE
#define PAMX_PASS_WPE 0
#endif
#if PAMX_PASS_WPE > 0
#define PAMX_PASS_ATTR __attribute__((amdgpu_waves_per_eu(PAMX_PASS_WPE)))
#else
#define PAMX_PASS_ATTR
#endif

namespace pamx {


// ---------------------------------------------------------------- helpers
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = f32x4; };
template <> struct Vec4<int32_t> { using type = i32x4; };

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T (&v)[VEC]) {
    if constexpr (VEC == 4) {
        const auto q = __builtin_nontemporal_load(reinterpret_cast<const typename Vec4<T>::type *>(p));
        v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
    } else {
        v[0] = __builtin_nontemporal_load(p);
    }
}

// ---------------------------------------------------------------- fills
template <typename X>
__global__ __launch_bounds__(256) void k_fill(X *__restrict__ p, int64_t cnt, X v) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < cnt) p[t] = v;
}
template <typename X>
static void fill(X *p, int64_t cnt, X v, hipStream_t s) {
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_fill<X>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, cnt, v);
}

template <typename X>
__global__ __launch_bounds__(256) void k_copy(const X *__restrict__ src, X *__restrict__ dst,
                                              int64_t cnt) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < cnt) dst[t] = src[t];
}

__global__ void k_state_init(DevState *st, int32_t max_iter, int32_t trace_cap) {
    if (threadIdx.x == 0) {
        DevState z{};
        z.max_iter = max_iter;
        z.trace_cap = trace_cap;
        z.best_i = -1;
        z.best_c = -1;
        *st = z;
    }
}

// ================================================================ BUILD (Alg. 1)
// A(c) = sum_o min(D[o][c], dn(o)) for every candidate c, one partial per
// object chunk.  Step 0 runs with dn = +inf, giving the column sums.  The
// candidate's own row contributes min(0, dn(c)) = 0, so A(c) - TD is the full
// TD change of adding c (self-term included); medoids have dn = 0 and add 0.
template <typename T, int VEC>
__global__ __launch_bounds__(kWG) void k_build_pass(const T *__restrict__ D, int64_t ld, int64_t n,
                                                    int64_t nc, const T *__restrict__ dn, int32_t L,
                                                    int64_t ncp, AccT<T> *__restrict__ part) {
    using A = AccT<T>;
    constexpr int U = 8;
    const int64_t a = (int64_t)blockIdx.y * L;
    const int64_t b = min(a + (int64_t)L, n);
    const int64_t c0 = ((int64_t)blockIdx.x * kWG + threadIdx.x) * VEC;
    A acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0;
    if (c0 < nc) {
        int64_t o = a;
        for (; o + U <= b; o += U) {
            T v[U][VEC];
            T m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                load_vec<T, VEC>(D + (o + u) * ld + c0, v[u]);
                m[u] = dn[o + u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] += (A)vmin(v[u][e], m[u]);
        }
        for (; o < b; ++o) {
            T v[VEC];
            load_vec<T, VEC>(D + o * ld + c0, v);
            const T m = dn[o];
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += (A)vmin(v[e], m);
        }
    }
    A *dst = part + (int64_t)blockIdx.y * ncp + c0;
#pragma unroll
    for (int e = 0; e < VEC; ++e) dst[e] = acc[e];
}

// ---- incremental BUILD.  Adding m_t lowers dn only for the objects closer
// to m_t than to every earlier medoid, and
//   A_t(c) - A_{t-1}(c) = sum over those objects of min(d, dn_new) - min(d, dn_old),
// so after the first two steps each step reads only the rows of the objects
// whose dn dropped (about n / t of them) instead of the whole matrix.  The
// sums are exact for int32 matrices; for FP32 the per-object differences are
// exact in FP64 and only their sum rounds.

// The step's medoid (every block reduces the merge partials itself: the
// smallest change, smallest index on ties; block 0 records it), then
// dn2 = min(dn, row m_t of Dl) and, per block of kObjBlk objects, how many
// dropped.  Dl holds a candidate's distances to all objects in a row: D
// itself when D is symmetric, else its transpose.
// FIRST: step 0, dn2 = row m_t (dn is +inf), no counts needed.
template <typename T, bool FIRST>
__global__ __launch_bounds__(kObjBlk) void k_build_select_update(
    const AccT<T> *__restrict__ wg_v, const int32_t *__restrict__ wg_c, int32_t nwg, int32_t t,
    int32_t *__restrict__ medoids, uint8_t *__restrict__ is_med, const T *__restrict__ Dl,
    int64_t ldl, int64_t n, const T *__restrict__ dn, T *__restrict__ dn2,
    DevState *__restrict__ st, int32_t *__restrict__ blkcnt) {
    using A = AccT<T>;
    A v = VT<T>::acc_inf();
    int c = INT_MAX, dummy = 0;
    for (int w = threadIdx.x; w < nwg; w += kObjBlk)
        if (lex_less(wg_v[w], 0, wg_c[w], v, 0, c)) { v = wg_v[w]; c = wg_c[w]; }
    block_argmin3<A, kObjBlk>(v, dummy, c);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->best_c = c;
        if (c != INT_MAX) {
            medoids[t] = c;
            is_med[c] = 1;
        } else {
            st->bad_medoids = 1;  // no candidate left (cannot happen for k <= n)
        }
    }
    const int64_t o = (int64_t)blockIdx.x * kObjBlk + threadIdx.x;
    int chg = 0;
    if (o < n) {
        const T old = dn[o];
        T nw = old;
        if (c != INT_MAX) {
            const T d = Dl[(int64_t)c * ldl + o];
            nw = FIRST ? d : vmin(old, d);
        }
        dn2[o] = nw;
        chg = nw < old;
    }
    if constexpr (!FIRST) {
        const int cnt = __syncthreads_count(chg);
        if (threadIdx.x == 0) blkcnt[blockIdx.x] = cnt;
    }
}

// Stable list of the objects whose dn dropped (ascending object order), with
// their old and new dn; the total goes to the device state.
template <typename T>
__global__ __launch_bounds__(kObjBlk) void k_build_compact(const T *__restrict__ dn,
                                                           const T *__restrict__ dn2, int64_t n,
                                                           const int32_t *__restrict__ blkcnt,
                                                           int32_t nblk, int32_t *__restrict__ chg_o,
                                                           T *__restrict__ chg_old,
                                                           T *__restrict__ chg_new,
                                                           DevState *__restrict__ st) {
    __shared__ int wcnt[kObjBlk / 64];
    int pre = 0, tot = 0;
    for (int b = threadIdx.x; b < nblk; b += kObjBlk) {
        const int v = blkcnt[b];
        tot += v;
        if (b < (int)blockIdx.x) pre += v;
    }
    pre = block_sum<int, kObjBlk>(pre);
    tot = block_sum<int, kObjBlk>(tot);
    const int64_t o = (int64_t)blockIdx.x * kObjBlk + threadIdx.x;
    T old = 0, nw = 0;
    bool chg = false;
    if (o < n) {
        old = dn[o];
        nw = dn2[o];
        chg = nw < old;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long m = __ballot(chg);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int rank = __popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wv; ++w) rank += wcnt[w];
    if (chg) {
        const int pos = pre + rank;
        chg_o[pos] = (int32_t)o;
        chg_old[pos] = old;
        chg_new[pos] = nw;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_chg = tot;
        st->build_rows += tot;
    }
}

// Per candidate and chunk of the list: sum of min(d, new) - min(d, old).
template <typename T, int VEC>
__global__ __launch_bounds__(kWG) void k_build_delta(const T *__restrict__ D, int64_t ld, int64_t nc,
                                                     const int32_t *__restrict__ chg_o,
                                                     const T *__restrict__ chg_old,
                                                     const T *__restrict__ chg_new,
                                                     const DevState *__restrict__ st, int64_t ncp,
                                                     AccT<T> *__restrict__ part) {
    using A = AccT<T>;
    constexpr int U = 4;
    const int64_t m = st->n_chg;
    const int Qd = gridDim.y, q = blockIdx.y;
    const int64_t Ld = (m + Qd - 1) / Qd;
    const int64_t a = min((int64_t)q * Ld, m), b = min(a + Ld, m);
    const int64_t c0 = ((int64_t)blockIdx.x * kWG + threadIdx.x) * VEC;
    A acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0;
    if (c0 < nc) {
        int64_t j = a;
        for (; j + U <= b; j += U) {
            T v[U][VEC];
            T lo[U], hi[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                load_vec<T, VEC>(D + (int64_t)chg_o[j + u] * ld + c0, v[u]);
                lo[u] = chg_old[j + u];
                hi[u] = chg_new[j + u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    acc[e] += (A)vmin(v[u][e], hi[u]) - (A)vmin(v[u][e], lo[u]);
        }
        for (; j < b; ++j) {
            T v[VEC];
            load_vec<T, VEC>(D + (int64_t)chg_o[j] * ld + c0, v);
            const T lo = chg_old[j], hi = chg_new[j];
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += (A)vmin(v[e], hi) - (A)vmin(v[e], lo);
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) part[(int64_t)q * ncp + c0 + e] = acc[e];
}

// A(c) <- A(c) + sum of the chunk deltas (chunk order), then the work-group's
// best (value, candidate) among non-medoids.
template <typename T>
__global__ __launch_bounds__(kWG) void k_build_dmerge(const AccT<T> *__restrict__ part, int32_t Q,
                                                      int64_t ncp, int64_t nc, AccT<T> *__restrict__ acur,
                                                      const T *__restrict__ dn,
                                                      const uint8_t *__restrict__ is_med,
                                                      int32_t add_self, AccT<T> *__restrict__ wg_v,
                                                      int32_t *__restrict__ wg_c) {
    using A = AccT<T>;
    const int64_t c = (int64_t)blockIdx.x * kWG + threadIdx.x;
    A v = VT<T>::acc_inf();
    int ci = INT_MAX;
    if (c < nc) {
        A s = 0;
        const A *pc = part + c;
        int q = 0;
        for (; q + 8 <= Q; q += 8) {
            A x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = pc[(int64_t)(q + u) * ncp];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; q < Q; ++q) s += pc[(int64_t)q * ncp];
        const A a = acur[c] + s;
        acur[c] = a;
        if (!is_med[c]) {
            v = add_self ? a + (A)dn[c] : a;
            ci = (int)c;
        }
    }
    int dummy = 0;
    block_argmin3<A, kWG>(v, dummy, ci);
    if (threadIdx.x == 0) {
        wg_v[blockIdx.x] = v;
        wg_c[blockIdx.x] = ci;
    }
}

// TD = sum_o dn(o) in a fixed order (single work-group).
template <typename T>
__global__ __launch_bounds__(1024) void k_td_sum(const T *__restrict__ dn, int64_t n,
                                                 DevState *__restrict__ st) {
    using A = AccT<T>;
    A s = 0;
    for (int64_t o = threadIdx.x; o < n; o += 1024) s += (A)dn[o];
    s = block_sum<A, 1024>(s);
    if (threadIdx.x == 0) {
        if constexpr (sizeof(T) == 4 && std::is_same<T, float>::value) st->td = s;
        else { st->td_i = s; st->td = (double)s; }
    }
}

// Rows of the candidates' distances to all objects: the transposed copy in
// the workspace for a rectangular (bichromatic) matrix, else D (symmetric).
template <typename T>
static const T *loc_rows(const T *D, int64_t ld, const Layout &L, void *ws, int64_t *ldl) {
    if (L.DT == SIZE_MAX) { *ldl = ld; return D; }
    *ldl = L.ldt;
    return reinterpret_cast<const T *>(static_cast<char *>(ws) + L.DT);
}

// BUILD: the first two steps read the whole matrix (column sums, then A for
// the first medoid's dn); every later step is incremental.  The SWAP-only
// buffers of the workspace serve as scratch: ds is the second dn buffer,
// srow/sdn/sds the list of changed objects, cand_a the running A(c).
template <typename T>
hipError_t run_build(const T *D, int64_t ld, const Layout &L, int32_t k, int32_t exclude_self,
                     int32_t *medoids, void *ws, hipStream_t s, hipEvent_t *ev) {
    using A = AccT<T>;
    char *w = static_cast<char *>(ws);
    const int64_t n = L.n, nc = L.nc;
    int64_t ldl;
    const T *Dl = loc_rows<T>(D, ld, L, ws, &ldl);
    T *dnb[2] = {reinterpret_cast<T *>(w + L.dn), reinterpret_cast<T *>(w + L.ds)};
    uint8_t *is_med = reinterpret_cast<uint8_t *>(w + L.is_med);
    A *part = reinterpret_cast<A *>(w + L.part);
    A *acur = reinterpret_cast<A *>(w + L.cand_a);
    A *wg_v = reinterpret_cast<A *>(w + L.wg_v);
    int32_t *wg_c = reinterpret_cast<int32_t *>(w + L.wg_c);
    int32_t *blkcnt = reinterpret_cast<int32_t *>(w + L.blkcnt);
    int32_t *chg_o = reinterpret_cast<int32_t *>(w + L.srow);
    T *chg_old = reinterpret_cast<T *>(w + L.sdn);
    T *chg_new = reinterpret_cast<T *>(w + L.sds);
    DevState *st = reinterpret_cast<DevState *>(w + L.state);
    const unsigned nblk = (unsigned)L.n_oblk;

    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, 0, 0);
    fill<uint8_t>(is_med, nc, 0, s);
    fill<T>(dnb[0], n, VT<T>::inf(), s);
    const dim3 pgrid(L.n_ctiles, L.Q);
    int cur = 0;   // dnb[cur] holds dn for the medoids chosen so far
    for (int32_t t = 0; t < k; ++t) {
        const T *dn = dnb[cur];
        if (t < 2) {
            if (ev) (void)hipEventRecord(ev[2 * t], s);
            if (L.vec == 4)
                hipLaunchKernelGGL((k_build_pass<T, 4>), pgrid, dim3(kWG), 0, s, D, ld, n, nc, dn,
                                   L.L, L.ncp, part);
            else
                hipLaunchKernelGGL((k_build_pass<T, 1>), pgrid, dim3(kWG), 0, s, D, ld, n, nc, dn,
                                   L.L, L.ncp, part);
            if (ev) (void)hipEventRecord(ev[2 * t + 1], s);
            // a zeroed running sum turns the delta merge into a plain merge
            fill<A>(acur, nc, (A)0, s);
        } else {
            hipLaunchKernelGGL(k_build_compact<T>, dim3(nblk), dim3(kObjBlk), 0, s,
                               (const T *)dnb[cur ^ 1], dn, n, (const int32_t *)blkcnt,
                               (int32_t)nblk, chg_o, chg_old, chg_new, st);
            if (ev) (void)hipEventRecord(ev[2 * t], s);
            if (L.vec == 4)
                hipLaunchKernelGGL((k_build_delta<T, 4>), pgrid, dim3(kWG), 0, s, D, ld, nc,
                                   (const int32_t *)chg_o, (const T *)chg_old, (const T *)chg_new,
                                   (const DevState *)st, L.ncp, part);
            else
                hipLaunchKernelGGL((k_build_delta<T, 1>), pgrid, dim3(kWG), 0, s, D, ld, nc,
                                   (const int32_t *)chg_o, (const T *)chg_old, (const T *)chg_new,
                                   (const DevState *)st, L.ncp, part);
            if (ev) (void)hipEventRecord(ev[2 * t + 1], s);
        }
        hipLaunchKernelGGL(k_build_dmerge<T>, dim3(L.n_mwg), dim3(kWG), 0, s, (const A *)part,
                           L.Q, L.ncp, nc, acur, dn, (const uint8_t *)is_med,
                           (int32_t)(exclude_self && t > 0 && L.DT == SIZE_MAX), wg_v, wg_c);
        if (t == 0)   // dn is +inf: the new dn is the medoid's row
            hipLaunchKernelGGL((k_build_select_update<T, true>), dim3(nblk), dim3(kObjBlk), 0, s,
                               (const A *)wg_v, (const int32_t *)wg_c, L.n_mwg, t, medoids, is_med,
                               Dl, ldl, n, dn, dnb[cur ^ 1], st, blkcnt);
        else
            hipLaunchKernelGGL((k_build_select_update<T, false>), dim3(nblk), dim3(kObjBlk), 0, s,
                               (const A *)wg_v, (const int32_t *)wg_c, L.n_mwg, t, medoids, is_med,
                               Dl, ldl, n, dn, dnb[cur ^ 1], st, blkcnt);
        cur ^= 1;
    }
    if (cur == 1)   // leave the final dn where the caches expect it
        hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const T *)dnb[1], dnb[0], n);
    hipLaunchKernelGGL(k_td_sum<T>, dim3(1), dim3(1024), 0, s, (const T *)dnb[0], n, st);
    return hipGetLastError();
}

// ================================================================ SWAP (Alg. 3)
// ---- nearest / second nearest of every object (O(nk), rows of the medoids)
// Order on (distance, slot) is lexicographic: nearest is the smallest slot at
// the minimum distance and ds the minimum over the other slots.
template <typename T> struct Top2 {
    T d1, d2;
    int32_t j1, j2;   // INT_MAX = none
};

template <typename T>
__device__ __forceinline__ void top2_insert(Top2<T> &t, T d, int32_t j) {
    if (lt2(d, j, t.d1, t.j1)) {
        t.d2 = t.d1; t.j2 = t.j1;
        t.d1 = d; t.j1 = j;
    } else if (lt2(d, j, t.d2, t.j2)) {
        t.d2 = d; t.j2 = j;
    }
}

// Fresh scan for one object (lanes = objects): rows of the medoids are read
// at column o, coalesced across the wave, 8 loads in flight.
template <typename T>
__device__ __forceinline__ Top2<T> scan_medoids(const T *__restrict__ D, int64_t ld, int k,
                                                const int32_t *__restrict__ med, int64_t o) {
    Top2<T> t{VT<T>::inf(), VT<T>::inf(), INT_MAX, INT_MAX};
    int j = 0;
    for (; j + 8 <= k; j += 8) {
        T d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = D[(int64_t)med[j + u] * ld + o];
#pragma unroll
        for (int u = 0; u < 8; ++u) top2_insert(t, d[u], j + u);
    }
    for (; j < k; ++j) top2_insert(t, D[(int64_t)med[j] * ld + o], j);
    return t;
}

// Rescan of one object by a whole wave: lanes take slots lane, lane+64, ...
// (row o of D at the medoid columns), then a butterfly merges the per-lane
// top-2 lists.  Every lane returns the same result.
template <typename T>
__device__ __forceinline__ Top2<T> wave_scan_medoids(const T *__restrict__ D, int64_t ld, int k,
                                                     const int32_t *__restrict__ med, int64_t o,
                                                     int lane) {
    Top2<T> t{VT<T>::inf(), VT<T>::inf(), INT_MAX, INT_MAX};
    const T *row = D + o * ld;
    int j = lane;
    for (; j + 192 < k; j += 256) {   // four loads in flight per lane
        T d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = row[med[j + 64 * u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) top2_insert(t, d[u], j + 64 * u);
    }
    for (; j < k; j += 64) top2_insert(t, row[med[j]], j);
    for (int w = 32; w >= 1; w >>= 1) {
        const T e1 = __shfl_xor(t.d1, w), e2 = __shfl_xor(t.d2, w);
        const int32_t f1 = __shfl_xor(t.j1, w), f2 = __shfl_xor(t.j2, w);
        if (lt2(e1, f1, t.d1, t.j1)) {
            if (lt2(e2, f2, t.d1, t.j1)) { t.d2 = e2; t.j2 = f2; }
            else { t.d2 = t.d1; t.j2 = t.j1; }
            t.d1 = e1; t.j1 = f1;
        } else if (lt2(e1, f1, t.d2, t.j2)) {
            t.d2 = e1; t.j2 = f1;
        }
    }
    return t;
}

template <typename T>
__device__ __forceinline__ void store_top2(const Top2<T> &t, int64_t o, int32_t *__restrict__ near,
                                           int32_t *__restrict__ sec, T *__restrict__ dn,
                                           T *__restrict__ ds) {
    // j1 is a real slot for every finite or infinite distance; only NaN
    // entries (a matrix outside the contract) leave it unset, and slot 0
    // keeps the segment arrays in range then
    near[o] = (t.j1 == INT_MAX) ? 0 : t.j1;
    sec[o] = (t.j2 == INT_MAX) ? -1 : t.j2;
    dn[o] = t.d1;
    ds[o] = t.d2;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cache_init(const T *__restrict__ D, int64_t ld, int64_t n,
                                                    int32_t k, const int32_t *__restrict__ med,
                                                    int32_t *__restrict__ near,
                                                    int32_t *__restrict__ sec, T *__restrict__ dn,
                                                    T *__restrict__ ds, int32_t *__restrict__ labels) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    const Top2<T> t = scan_medoids<T>(D, ld, k, med, o);
    store_top2<T>(t, o, near, sec, dn, ds);
    if (labels) labels[o] = (t.j1 == INT_MAX) ? 0 : t.j1;
}

// Input check: medoids distinct and in range (uses `mark` zeroed beforehand).
__global__ __launch_bounds__(256) void k_check_medoids(const int32_t *__restrict__ med, int32_t k,
                                                       int64_t n, int32_t *__restrict__ mark,
                                                       uint8_t *__restrict__ is_med,
                                                       DevState *__restrict__ st) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= k) return;
    const int32_t m = med[j];
    if (m < 0 || (int64_t)m >= n) { atomicOr(&st->bad_medoids, 1); return; }
    if (atomicAdd(&mark[m], 1) != 0) atomicOr(&st->bad_medoids, 1);
    is_med[m] = 1;
}

// ---- per-object cache update after slot `slot` received a new medoid.
// An object that keeps both its nearest and its second medoid only compares
// against the new one (O(1)); an object that lost one of them needs all k
// medoids again and is returned as "rescan" (done by wave_scan_medoids).
// Written as selects: conditional stores through the references made the
// compiler keep the four values in scratch memory (a store and a reload on
// every update) and, for caches held in register arrays, the whole arrays.
template <typename T>
__device__ __forceinline__ bool cache_update_o1(int slot, T dnew, int32_t &nr, int32_t &sc, T &dn,
                                                T &ds) {
    const bool rescan = nr == slot || sc == slot;
    const bool first = !rescan && lt2(dnew, slot, dn, nr);
    const bool second = !rescan && !first && lt2(dnew, slot, ds, sc < 0 ? INT_MAX : sc);
    const int32_t nr1 = first ? slot : nr;
    const int32_t sc1 = first ? nr : (second ? slot : sc);
    const T dn1 = first ? dnew : dn;
    const T ds1 = first ? dn : (second ? dnew : ds);
    nr = nr1; sc = sc1; dn = dn1; ds = ds1;
    return rescan;
}

// One wave per listed object (the list order varies, each result does not).
// Up to kRsMed medoids, the list of medoids is staged in LDS first, so each
// step of a rescan waits on one global load (the row entry), not two.
constexpr int kRsMed = 4096;
template <typename T>
__global__ __launch_bounds__(256) void k_cache_rescan(const T *__restrict__ D, int64_t ld, int32_t k,
                                                      const int32_t *__restrict__ med,
                                                      int32_t *__restrict__ near,
                                                      int32_t *__restrict__ sec, T *__restrict__ dn,
                                                      T *__restrict__ ds,
                                                      const int32_t *__restrict__ rlist,
                                                      const DevState *__restrict__ st) {
    if (st->done || !st->swapped) return;
    __shared__ int32_t smed[kRsMed];
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * 4;
    const int m = st->n_list;
    if (blockIdx.x * 4 >= m) return;   // no listed object for this work-group
    if (k <= kRsMed) {
        for (int j = threadIdx.x; j < k; j += 256) smed[j] = med[j];
        __syncthreads();
        for (int idx = blockIdx.x * 4 + (threadIdx.x >> 6); idx < m; idx += nw) {
            const int64_t o = rlist[idx];
            const Top2<T> t = wave_scan_medoids<T>(D, ld, k, smed, o, lane);
            if (lane == 0) store_top2<T>(t, o, near, sec, dn, ds);
        }
    } else {
        for (int idx = blockIdx.x * 4 + (threadIdx.x >> 6); idx < m; idx += nw) {
            const int64_t o = rlist[idx];
            const Top2<T> t = wave_scan_medoids<T>(D, ld, k, med, o, lane);
            if (lane == 0) store_top2<T>(t, o, near, sec, dn, ds);
        }
    }
}

// ---- iteration start (folded into the first block of k_seg_count): the
// iteration cap, and the per-iteration flags.
__device__ __forceinline__ void iter_begin(DevState *st) {
    st->swapped = 0;
    st->n_list = 0;
    if (!st->fp && st->iter >= st->max_iter) {
        st->done = 1;
        st->capped = 1;
    }
}

// ---- stable counting sort of objects by nearest slot.  Each block also
// sums its objects' dn and ds (TD and the rounding bound's sum of ds), in a
// fixed order: wave butterflies, then the four waves in order.
template <typename T>
__global__ __launch_bounds__(kObjBlk) void k_seg_count(const int32_t *__restrict__ near,
                                                       const T *__restrict__ dn,
                                                       const T *__restrict__ ds, int64_t n,
                                                       int32_t k, int32_t *__restrict__ blkcnt,
                                                       AccT<T> *__restrict__ tdp,
                                                       DevState *__restrict__ st) {
    using A = AccT<T>;
    if (st->done) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) iter_begin(st);
    if (st->seg_skip) return;
    extern __shared__ int32_t hist[];
    __shared__ A w1[kObjBlk / 64], w2[kObjBlk / 64];
    for (int i = threadIdx.x; i < k; i += kObjBlk) hist[i] = 0;
    __syncthreads();
    const int64_t o = (int64_t)blockIdx.x * kObjBlk + threadIdx.x;
    A s1 = 0, s2 = 0;
    if (o < n) {
        atomicAdd(&hist[near[o]], 1);
        s1 = (A)dn[o];
        s2 = (A)ds[o];
    }
    s1 = wave_sum<A>(s1);
    s2 = wave_sum<A>(s2);
    if ((threadIdx.x & 63) == 0) { w1[threadIdx.x >> 6] = s1; w2[threadIdx.x >> 6] = s2; }
    __syncthreads();
    int32_t *dst = blkcnt + (int64_t)blockIdx.x * k;
    for (int i = threadIdx.x; i < k; i += kObjBlk) dst[i] = hist[i];
    if (threadIdx.x == 0) {
        A t1 = 0, t2 = 0;
        for (int u = 0; u < kObjBlk / 64; ++u) { t1 += w1[u]; t2 += w2[u]; }
        tdp[2 * blockIdx.x] = t1;
        tdp[2 * blockIdx.x + 1] = t2;
    }
}

// Exclusive prefix over blocks of each slot's counts (in place), one wave per
// slot; seg_size[i] = the slot's total.
__global__ __launch_bounds__(256) void k_seg_colscan(int32_t *__restrict__ blkcnt, int32_t nblk,
                                                     int32_t k, int32_t *__restrict__ seg_size,
                                                     const DevState *__restrict__ st) {
    if (st->done || st->seg_skip) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= k) return;
    int32_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 64) {
        const int b = b0 + lane;
        const int32_t c = (b < nblk) ? blkcnt[(int64_t)b * k + i] : 0;
        int32_t x = c;   // inclusive wave scan
        for (int w = 1; w < 64; w <<= 1) {
            const int32_t y = __shfl_up(x, w);
            if (lane >= w) x += y;
        }
        if (b < nblk) blkcnt[(int64_t)b * k + i] = carry + x - c;
        carry += __shfl(x, 63);
    }
    if (lane == 0) seg_size[i] = carry;
}

struct ChunkInfo {
    int32_t sa, sb, flags;  // segment of the first / last object, carry flags
    int32_t se0;            // end of segment sa (seg_off[sa + 1])
};
constexpr int kHead = 1, kTail = 2;

// Segment offsets and the stable scatter in one launch.  Every block scans
// the k slot totals (seg_tot) into LDS offsets and places its objects at
// segment start + block base + rank among the block's objects of the same
// slot.  Block 0 also publishes seg_off[0..k], the smallest empty slot, TD
// and the sum of ds (for the rounding bound) from the nblk block sums of
// k_seg_count, and the carry map of every chunk.
template <typename T>
__global__ __launch_bounds__(kObjBlk) void k_seg_scatter(
    const int32_t *__restrict__ near, const T *__restrict__ dn, const T *__restrict__ ds, int64_t n,
    int32_t k, const int32_t *__restrict__ blkbase, const int32_t *__restrict__ seg_tot,
    int32_t *__restrict__ seg_off, const AccT<T> *__restrict__ tdp, int32_t nblk, int32_t L,
    int32_t Q, ChunkInfo *__restrict__ cinfo, int32_t *__restrict__ srow, T *__restrict__ sdn,
    T *__restrict__ sds, DevState *__restrict__ st) {
    using A = AccT<T>;
    if (st->done || st->seg_skip) return;
    extern __shared__ int32_t soff[];   // k + 1 offsets
    __shared__ int32_t ln[kObjBlk];
    __shared__ int32_t wsum[kObjBlk / 64];
    __shared__ A ws1[kObjBlk / 64], ws2[kObjBlk / 64];
    __shared__ int32_t empty_min;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const bool lead = blockIdx.x == 0;
    // offsets: each thread takes a run of consecutive slots; a block scan of
    // the run totals gives each run's start
    if (t == 0) empty_min = k;
    const int per = (k + kObjBlk - 1) / kObjBlk;
    const int i0 = min(k, t * per), i1 = min(k, i0 + per);
    int32_t run = 0;
    for (int i = i0; i < i1; ++i) run += seg_tot[i];
    int32_t x = run;   // inclusive wave scan
    for (int w = 1; w < 64; w <<= 1) {
        const int32_t y = __shfl_up(x, w);
        if (lane >= w) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int32_t off = x - run;
    for (int u = 0; u < wv; ++u) off += wsum[u];
    for (int i = i0; i < i1; ++i) {
        const int32_t c = seg_tot[i];
        if (lead && c == 0) atomicMin(&empty_min, i);
        soff[i] = off;
        off += c;
    }
    if (t == 0) soff[k] = (int32_t)n;
    __syncthreads();
    if (lead) {
        for (int i = t; i <= k; i += kObjBlk) seg_off[i] = soff[i];
        // TD and sum of ds over the block sums, fixed order (blocks t, t +
        // kObjBlk, ... per thread, wave butterflies, then the wave sums in order)
        A s1 = 0, s2 = 0;
        for (int bb = t; bb < nblk; bb += kObjBlk) { s1 += tdp[2 * bb]; s2 += tdp[2 * bb + 1]; }
        s1 = wave_sum<A>(s1);
        s2 = wave_sum<A>(s2);
        if (lane == 0) { ws1[wv] = s1; ws2[wv] = s2; }
        // carry map of each chunk (binary searches in LDS)
        for (int q = t; q < Q; q += kObjBlk) {
            const int64_t qa = (int64_t)q * L, qb = min(qa + (int64_t)L, n);
            int lo = 0, hi = k;
            while (hi - lo > 1) { const int m = (lo + hi) >> 1; if (soff[m] <= qa) lo = m; else hi = m; }
            const int sa = lo;
            lo = 0; hi = k;
            while (hi - lo > 1) { const int m = (lo + hi) >> 1; if (soff[m] <= qb - 1) lo = m; else hi = m; }
            const int sb = lo;
            int f = 0;
            if (soff[sa] < qa || soff[sa + 1] > qb) f |= kHead;
            if (sb != sa && soff[sb + 1] > qb) f |= kTail;
            cinfo[q] = ChunkInfo{sa, sb, f, soff[sa + 1]};
        }
        __syncthreads();
        if (t == 0) {
            s1 = 0; s2 = 0;
            for (int u = 0; u < kObjBlk / 64; ++u) { s1 += ws1[u]; s2 += ws2[u]; }
            st->empty_slot = empty_min;
            if constexpr (std::is_same<T, float>::value) {
                st->td = s1;
                // bound on the FP64 rounding of a computed change: every partial
                // sum is <= sum(ds), chains are at most n + Q + 64 additions long
                st->margin = 4.0 * ((double)n + Q + 68) * 0x1p-53 * (double)s2;
            } else {
                st->td_i = s1;
                st->td = (double)s1;
                st->margin = 0.0;
            }
        }
    }
    // the stable scatter
    const int64_t o = (int64_t)blockIdx.x * kObjBlk + t;
    const int32_t sl = (o < n) ? near[o] : -1;
    ln[t] = sl;
    __syncthreads();
    if (o >= n) return;
    int rank = 0;
    for (int u = 0; u < t; ++u) rank += (ln[u] == sl);
    const int32_t pos = soff[sl] + blkbase[(int64_t)blockIdx.x * k + sl] + rank;
    srow[pos] = (int32_t)o;
    sdn[pos] = dn[o];
    sds[pos] = ds[o];
}

// FastPAM2's buffer P of M_i(c) - DN_i, laid out so that one pass
// work-group's values are a single contiguous run: tile-major (TW candidates
// per pass tile), and within a tile one row per (chunk q, segment s) at row
// s + q.  Rows of consecutive chunks never overlap (a chunk's first segment is
// at least the previous chunk's last), so k + Q rows hold them all; a segment
// cut by chunk edges (its sums come from the merge) lives in the row of the
// chunk that holds its first object, seg_off[s] / L.
__device__ __forceinline__ int64_t p_index(int64_t rows, int tw_log2, int64_t row, int64_t c) {
    return ((((c >> tw_log2) * rows) + row) << tw_log2) + (c & ((int64_t(1) << tw_log2) - 1));
}

// DN_i = sum over segment i of dn, one wave per segment, fixed order.
// ---- the hot pass.  See the file header for the arithmetic.
// Output per candidate and chunk: part[q][0] = A partial, [1] head carry,
// [2] tail carry, [3] best value over segments complete in the chunk, and
// part_i = its slot.  P2 (FastPAM2) also stores M_i - DN_i of complete
// segments into P[i][c].  Candidates [cb, ce), partials indexed from cb.
template <typename T, int VEC, bool P2, bool PF = false, int UB = 4>
__device__ __forceinline__ void pass_tile(
    int tile, int q, int64_t cb, int64_t ce, const T *__restrict__ D, int64_t ld, int64_t n,
    const int32_t *__restrict__ srow, const T *__restrict__ sdn, const T *__restrict__ sds,
    const int32_t *__restrict__ seg_off, AccT<T> *__restrict__ cdn,
    const ChunkInfo *__restrict__ cinfo, int32_t L, int64_t ncp, AccT<T> *__restrict__ part,
    int32_t *__restrict__ part_i, AccT<T> *__restrict__ P, int64_t prows) {
    using A = AccT<T>;
    constexpr int kTwLog2 = VEC == 4 ? 10 : 8;   // log2(kWG * VEC)
    static_assert(kWG * VEC == (1 << kTwLog2), "pass tile width");
    // UB rows per block: four (measured faster than eight or sixteen on a
    // 20000 x 20000 FP32 matrix)
    constexpr int U = UB;
    const int64_t a = (int64_t)q * L;
    const int64_t b = min(a + (int64_t)L, n);
    const int64_t cr = ((int64_t)tile * kWG + threadIdx.x) * VEC;   // partial column
    const int64_t c0 = cb + cr;
    const bool active = c0 < ce;
    const ChunkInfo ci = cinfo[q];

    A accA[VEC], bv[VEC];
    int32_t bi[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) { accA[e] = 0; bv[e] = VT<T>::acc_inf(); bi[e] = INT_MAX; }
    A *pq = part + (int64_t)q * 4 * ncp + cr;
    // the first lane of the first tile (always a real candidate: windows are
    // never empty) records the chunk's part of DN for segments carried
    // across chunks
    const bool rec = tile == 0 && threadIdx.x == 0;
    // FastPAM2: each wave stages the P values of up to kPStage complete
    // segments in LDS and writes them out together, four 512-byte stores per
    // segment.  A store is counted with the loads the wave waits for, so one
    // store per segment close stalled the stream each time (measured 8 %
    // slower at n = 20000).  Waves with inactive lanes store directly.
    constexpr int kPStage = PAMX_PSTAGE;
    __shared__ A pst[4 * (kPStage > 0 ? kPStage : 1) * 256];
    __shared__ int32_t pseg[4 * (kPStage > 0 ? kPStage : 1)];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int64_t wc0 = cb + ((int64_t)tile * kWG + (threadIdx.x & ~63)) * VEC;   // wave's first column
    const bool wfull = kPStage > 0 && VEC == 4 && wc0 + 64 * VEC <= ce;
    int nst = 0;   // staged segments (wave-uniform)
    auto flush_p = [&]() {
        __builtin_amdgcn_wave_barrier();
        for (int t = 0; t < nst; ++t) {
            A *dst = P + p_index(prows, kTwLog2, (int64_t)pseg[wv * kPStage + t] + q, wc0);
            const A *src = pst + (wv * kPStage + t) * 256;
#pragma unroll
            for (int e = 0; e < 4; ++e) __builtin_nontemporal_store(src[64 * e + ln], dst + 64 * e + ln);
        }
        __builtin_amdgcn_wave_barrier();
        nst = 0;
    };

    if (active) {
        // The chunk's rows are one stream of blocks of U rows; a segment edge
        // inside a block closes the segment there (a wave-uniform branch), so
        // loads are never cut short at segment edges.
        int s = ci.sa;                                   // segment of the current row
        int64_t se = min((int64_t)ci.se0, b);            // its end within the chunk
        A M[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) M[e] = 0;
        A dns = 0;   // DN of the segment's rows in this chunk (same in every lane)
        auto close_seg = [&]() {
            if (s == ci.sa && (ci.flags & kHead)) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) pq[1 * ncp + e] = M[e];
                if (rec) cdn[2 * q] = dns;
            } else if (s == ci.sb && (ci.flags & kTail)) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) pq[2 * ncp + e] = M[e];
                if (rec) cdn[2 * q + 1] = dns;
            } else {
                A v[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    v[e] = M[e] - dns;
                    if (v[e] < bv[e]) { bv[e] = v[e]; bi[e] = s; }
                }
                if constexpr (P2) {
                    // streaming stores (P is read once, by the best-candidate
                    // scan); measured faster than cached stores
                    if (wfull) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) pst[(wv * kPStage + nst) * 256 + ln * VEC + e] = v[e];
                        if (ln == 0) pseg[wv * kPStage + nst] = s;
                        if (++nst == kPStage) flush_p();
                    } else {
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            __builtin_nontemporal_store(
                                v[e], &P[p_index(prows, kTwLog2, (int64_t)s + q, c0 + e)]);
                    }
                }
            }
        };
        // row j starts a new segment: close the current one, move to the
        // next non-empty segment
        auto next_seg = [&](int64_t j) {
            close_seg();
            do { ++s; } while (seg_off[s + 1] <= j);
            se = min((int64_t)seg_off[s + 1], b);
#pragma unroll
            for (int e = 0; e < VEC; ++e) M[e] = 0;
            dns = 0;
        };
        auto add_row = [&](const T (&v)[VEC], T lo, T hi) {
            dns += (A)lo;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                accA[e] += (A)vmin(v[e], lo);
                M[e] += (A)vmed3(v[e], lo, hi);
            }
        };
        auto add_block = [&](int64_t j, const T (&v)[U][VEC], const T (&lo)[U], const T (&hi)[U]) {
            if (j + U <= se) {
#pragma unroll
                for (int u = 0; u < U; ++u) add_row(v[u], lo[u], hi[u]);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (j + u == se) next_seg(j + u);
                    add_row(v[u], lo[u], hi[u]);
                }
            }
        };
        auto load_block = [&](int64_t j, T (&v)[U][VEC], T (&lo)[U], T (&hi)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t o = srow[j + u];
                load_vec<T, VEC>(D + o * ld + c0, v[u]);
                lo[u] = sdn[j + u];
                hi[u] = sds[j + u];
            }
        };
        int64_t j = a;
        if constexpr (PF) {
            // long chunks: the next block's rows are issued before the
            // current block is summed (eight rows in flight per lane)
            if (j + U <= b) {
                T v[U][VEC], lo[U], hi[U];
                load_block(j, v, lo, hi);
                for (; j + 2 * U <= b; j += U) {
                    T w[U][VEC], wl[U], wh[U];
                    load_block(j + U, w, wl, wh);
                    add_block(j, v, lo, hi);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) v[u][e] = w[u][e];
                        lo[u] = wl[u];
                        hi[u] = wh[u];
                    }
                }
                add_block(j, v, lo, hi);
                j += U;
            }
        } else {
            for (; j + U <= b; j += U) {
                T v[U][VEC], lo[U], hi[U];
                load_block(j, v, lo, hi);
                add_block(j, v, lo, hi);
            }
        }
        for (; j < b; ++j) {
            if (j == se) next_seg(j);
            const int64_t o = srow[j];
            T v[VEC];
            load_vec<T, VEC>(D + o * ld + c0, v);
            add_row(v, sdn[j], sds[j]);
        }
        close_seg();
        if constexpr (P2) {
            if (nst > 0) flush_p();
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        pq[0 * ncp + e] = accA[e];
        pq[3 * ncp + e] = bv[e];
        part_i[(int64_t)q * ncp + cr + e] = bi[e];
    }
}

// WIN: the FasterPAM window pass over long chunks (one work-group per chunk
// over every tile of the window [fw_base, fw_end), partials indexed from
// fw_base; ncp is then the window width).  Its rows go in blocks of eight,
// the next block issued before the current one is summed: 106 -> 92 us per
// pass at n = 100000 (392-object chunks) against blocks loaded one at a
// time; prefetched blocks of four were slower than either.  Short chunks
// take k_fp_pass instead.
template <typename T, int VEC, bool P2, bool WIN, bool PF = false>
__global__ __launch_bounds__(kWG) PAMX_PASS_ATTR void k_swap_pass(
    const T *__restrict__ D, int64_t ld, int64_t n, int64_t nc, int32_t k,
    const int32_t *__restrict__ srow,
    const T *__restrict__ sdn, const T *__restrict__ sds, const int32_t *__restrict__ seg_off,
    AccT<T> *__restrict__ cdn, const ChunkInfo *__restrict__ cinfo, int32_t L, int64_t ncp,
    AccT<T> *__restrict__ part, int32_t *__restrict__ part_i, AccT<T> *__restrict__ P,
    int64_t prows, const DevState *__restrict__ st) {
    if constexpr (!WIN) {
        // the chunk's map entry and first row are read with the state, so
        // one memory round trip precedes the first rows of D
        const ChunkInfo ci0 = cinfo[blockIdx.y];
        const int32_t r0 = srow[(int64_t)blockIdx.y * L];
        if (st->done || r0 < 0 || ci0.sa < 0) return;   // rows and slots are never negative
        pass_tile<T, VEC, P2, PF>(blockIdx.x, blockIdx.y, 0, nc, D, ld, n, srow, sdn, sds, seg_off,
                                  cdn, cinfo, L, ncp, part, part_i, P, prows);
    } else {
        if (st->done) return;
        const int64_t cb = st->fw_base, ce = st->fw_end;
        const int nt = (int)((ce - cb + kWG * VEC - 1) / (kWG * VEC));
        for (int t = 0; t < nt; ++t)
            pass_tile<T, VEC, false, true, 8>(t, blockIdx.y, cb, ce, D, ld, n, srow, sdn, sds,
                                              seg_off, cdn, cinfo, L, ncp, part, part_i, P, prows);
    }
}

// ---- FasterPAM window pass.  The window [fw_base, fw_end) is short after a
// swap (one tile), so the pass is spread over the objects.  A work-group
// takes G consecutive chunks g * G + u, each with 4 / G of its waves (wave w:
// chunk u = w / (4 / G), column block w % (4 / G)), over the columns
// x * W + [0, W) of every window tile, W = 256 * VEC / G (rows as in
// pass_tile: blocks of eight, the next block issued before the current one
// is summed).  The waves then merge their chunks' summaries in chunk order
// through LDS, so the window merge reads one summary per group of G chunks:
// part[g][0] = A, [1] = M of the group's first segment run, [2] = M of its
// last run, [3] = best value over segments complete inside the group,
// part_i = its slot; ginfo[g] = {first run's slot, last run's slot, kHead if
// there is a first run, kTail if there is a last one} and cdn[2g],
// cdn[2g + 1] their parts of DN.  A run that continues into the next group is
// finished by the merge (k_fp_merge), exactly as for single chunks.  Used
// for short chunks, which are latency-bound (with G = 4 the merge reads a
// quarter of the partials); long chunks take k_swap_pass<..., WIN = true>,
// whose waves share their rows.
constexpr int kFpU = 8;   // rows per block of the window pass
template <typename T, int VEC, int G>
__global__ __launch_bounds__(kWG) PAMX_PASS_ATTR void k_fp_pass(
    const T *__restrict__ D, int64_t ld, int64_t n, const int32_t *__restrict__ srow,
    const T *__restrict__ sdn, const T *__restrict__ sds, const int32_t *__restrict__ seg_off,
    const ChunkInfo *__restrict__ cinfo, int32_t L, int32_t Q, AccT<T> *__restrict__ cdn,
    ChunkInfo *__restrict__ ginfo, AccT<T> *__restrict__ part, int32_t *__restrict__ part_i,
    int64_t ncp, const DevState *__restrict__ st) {
    using A = AccT<T>;
    constexpr int U = kFpU;
    constexpr int CW = kFpGroup / G;     // waves per chunk
    constexpr int W = CW * 64 * VEC;     // columns per work-group and tile
    static_assert((G == 2 || G == 4) && G * CW == kFpGroup && kFpGroup * 64 == kWG,
                  "waves of a work-group");
    if (st->done) return;
    // per wave (chunk): the summary of each of the W columns, the chunk's run
    // map and the DN parts of its first and last runs
    __shared__ A s_a[G][W], s_bv[G][W], s_h[G][W], s_t[G][W];
    __shared__ int32_t s_bi[G][W];
    __shared__ ChunkInfo s_ci[G];
    __shared__ A s_dh[G], s_dt[G];
    const int64_t cb = st->fw_base, ce = st->fw_end;
    const int nt = (int)((ce - cb + kWG * VEC - 1) / (kWG * VEC));   // window tiles
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int uw = wv / CW;                         // this wave's chunk in the group
    const int li = (wv % CW) * 64 + ln;             // and its lane's column block
    const int g = blockIdx.y;
    const int q = g * G + uw;
    const bool has = q < Q;
    const int64_t a = (int64_t)q * L;
    const int64_t b = has ? min(a + (int64_t)L, n) : a;
    const ChunkInfo ci = has ? cinfo[q] : ChunkInfo{0, 0, 0, 0};
    for (int t = 0; t < nt; ++t) {
        const int64_t wcol = (int64_t)t * kWG * VEC + (int64_t)blockIdx.x * W;   // first column
        const int64_t c0 = cb + wcol + li * VEC;
        A accA[VEC], bv[VEC];
        int32_t bi[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) { accA[e] = 0; bv[e] = VT<T>::acc_inf(); bi[e] = INT_MAX; }
        if (has && c0 < ce) {
            int s = ci.sa;
            int64_t se = min((int64_t)ci.se0, b);
            A M[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) M[e] = 0;
            A dns = 0;
            // the chunk's first and last runs go to LDS as they close (the
            // previous tile's merge is behind the barrier that ends it); their
            // DN parts are the same in every lane, the chunk's first lane
            // writes them
            auto close_seg = [&]() {
                if (s == ci.sa && (ci.flags & kHead)) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) s_h[uw][li * VEC + e] = M[e];
                    if (li == 0) s_dh[uw] = dns;
                } else if (s == ci.sb && (ci.flags & kTail)) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) s_t[uw][li * VEC + e] = M[e];
                    if (li == 0) s_dt[uw] = dns;
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const A v = M[e] - dns;
                        if (v < bv[e]) { bv[e] = v; bi[e] = s; }
                    }
                }
            };
            auto next_seg = [&](int64_t j) {
                close_seg();
                do { ++s; } while (seg_off[s + 1] <= j);
                se = min((int64_t)seg_off[s + 1], b);
#pragma unroll
                for (int e = 0; e < VEC; ++e) M[e] = 0;
                dns = 0;
            };
            auto add_row = [&](const T (&v)[VEC], T lo, T hi) {
                dns += (A)lo;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    accA[e] += (A)vmin(v[e], lo);
                    M[e] += (A)vmed3(v[e], lo, hi);
                }
            };
            auto add_block = [&](int64_t j, const T (&v)[U][VEC], const T (&lo)[U], const T (&hi)[U]) {
                if (j + U <= se) {
#pragma unroll
                    for (int u = 0; u < U; ++u) add_row(v[u], lo[u], hi[u]);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (j + u == se) next_seg(j + u);
                        add_row(v[u], lo[u], hi[u]);
                    }
                }
            };
            auto load_block = [&](int64_t j, T (&v)[U][VEC], T (&lo)[U], T (&hi)[U]) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t o = srow[j + u];
                    load_vec<T, VEC>(D + o * ld + c0, v[u]);
                    lo[u] = sdn[j + u];
                    hi[u] = sds[j + u];
                }
            };
            int64_t j = a;
            if (j + U <= b) {
                T v[U][VEC], lo[U], hi[U];
                load_block(j, v, lo, hi);
                for (; j + 2 * U <= b; j += U) {
                    T w[U][VEC], wl[U], wh[U];
                    load_block(j + U, w, wl, wh);
                    add_block(j, v, lo, hi);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) v[u][e] = w[u][e];
                        lo[u] = wl[u];
                        hi[u] = wh[u];
                    }
                }
                add_block(j, v, lo, hi);
                j += U;
            }
            for (; j < b; ++j) {
                if (j == se) next_seg(j);
                const int64_t o = srow[j];
                T v[VEC];
                load_vec<T, VEC>(D + o * ld + c0, v);
                add_row(v, sdn[j], sds[j]);
            }
            close_seg();
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            s_a[uw][li * VEC + e] = accA[e];
            s_bv[uw][li * VEC + e] = bv[e];
            s_bi[uw][li * VEC + e] = bi[e];
        }
        // run values are read only where the run map has the run; a chunk's
        // first lane is active whenever any column of the work-group is (its
        // column is the work-group's first), so columns that are read have them
        if (li == 0) s_ci[uw] = has ? ci : ChunkInfo{0, 0, 0, 0};
        __syncthreads();
        // the group's summary of column wcol + j: the chunks' summaries in
        // chunk order (runs of the same slot joined, runs that end inside
        // the group taken as complete segments)
        for (int jj = threadIdx.x; jj < W; jj += kWG) {
            A sa = 0, rbv = VT<T>::acc_inf(), fm = 0, fdn = 0, lm = 0, ldn = 0;
            int32_t rbi = INT_MAX, nr = 0, fs = 0, ls = 0;
            auto add = [&](int sl, A m, A dn) {
                if (nr == 0) { nr = 1; fs = sl; fm = m; fdn = dn; return; }
                if (nr == 1) {
                    if (sl == fs) { fm += m; fdn += dn; }
                    else { nr = 2; ls = sl; lm = m; ldn = dn; }
                    return;
                }
                if (sl == ls) { lm += m; ldn += dn; return; }
                const A v = lm - ldn;
                if (lt2(v, ls, rbv, rbi)) { rbv = v; rbi = ls; }
                ls = sl; lm = m; ldn = dn;
            };
#pragma unroll
            for (int u = 0; u < G; ++u) {
                sa += s_a[u][jj];
                const int32_t xi = s_bi[u][jj];
                const A xv = s_bv[u][jj];
                if (xi != INT_MAX && lt2(xv, xi, rbv, rbi)) { rbv = xv; rbi = xi; }
                const ChunkInfo cu = s_ci[u];
                if (cu.flags & kHead) add(cu.sa, s_h[u][jj], s_dh[u]);
                if (cu.flags & kTail) add(cu.sb, s_t[u][jj], s_dt[u]);
            }
            const int64_t col = wcol + jj;
            A *pq = part + (int64_t)g * 4 * ncp + col;
            pq[0] = sa;
            pq[1 * ncp] = fm;
            pq[2 * ncp] = lm;
            pq[3 * ncp] = rbv;
            part_i[(int64_t)g * ncp + col] = rbi;
            if (t == 0 && blockIdx.x == 0 && jj == 0) {
                ginfo[g] = ChunkInfo{fs, ls, (nr >= 1 ? kHead : 0) | (nr == 2 ? kTail : 0), 0};
                cdn[2 * g] = fdn;
                cdn[2 * g + 1] = ldn;
            }
        }
        __syncthreads();   // the summaries are rewritten by the next tile
    }
}

// ---- merge chunk partials per candidate (fixed order).
// A work-group takes kSmC candidates; each candidate's chunks are split into
// kSmG consecutive groups, one thread each, which reduce their chunks to a
// run summary (A, the best segment complete in the group, the first and the
// last segment run); the candidate's first thread combines the kSmG
// summaries in chunk order (as the window merge of FasterPAM does).  Writes,
// per candidate, its best change over slots and the work-group's best
// (value, slot, candidate); for FastPAM2 it completes P[i][c] for segments
// carried across chunks and stores B(c) = A(c) - TD.
constexpr int kSmC = 64, kSmG = kWG / kSmC;
template <typename A>
struct RunSum {
    A accA, bv, fm, fdn, lm, ldn;
    int32_t bi, nr, fs, ls;   // nr: runs seen (0, 1, 2 = more than one)
};
template <typename T, bool P2>
__global__ __launch_bounds__(kWG) void k_swap_merge(
    const AccT<T> *__restrict__ part, const int32_t *__restrict__ part_i,
    const ChunkInfo *__restrict__ cinfo, int32_t Q, int64_t nc, int32_t k, int64_t ncp,
    const AccT<T> *__restrict__ cdn, const uint8_t *__restrict__ is_med,
    const DevState *__restrict__ st, AccT<T> *__restrict__ P, AccT<T> *__restrict__ cand_a,
    AccT<T> *__restrict__ wg_v, int32_t *__restrict__ wg_i, int32_t *__restrict__ wg_c,
    const int32_t *__restrict__ seg_off, int32_t Lc, int64_t prows, int32_t tw_log2) {
    using A = AccT<T>;
    if (st->done) return;
    __shared__ RunSum<A> sm[kSmG][kSmC];
    // row of P for a segment carried across chunks: the chunk of its first object
    auto prow = [&](int s) { return (int64_t)s + seg_off[s] / Lc; };
    const int j = threadIdx.x % kSmC, g = threadIdx.x / kSmC;
    const int64_t c = (int64_t)blockIdx.x * kSmC + j;
    const bool live = c < nc;
    RunSum<A> r;
    r.accA = 0; r.bv = VT<T>::acc_inf(); r.bi = INT_MAX; r.nr = 0;
    r.fs = -1; r.fm = 0; r.fdn = 0; r.ls = -1; r.lm = 0; r.ldn = 0;
    if (live) {
        const int per = (Q + kSmG - 1) / kSmG;
        const int q0 = g * per, q1 = min(Q, q0 + per);
        // the open run is (fs, fm, fdn) while nr == 1, else (ls, lm, ldn)
        auto add = [&](int s, A m, A dn) {
            if (r.nr == 0) { r.nr = 1; r.fs = s; r.fm = m; r.fdn = dn; return; }
            if (r.nr == 1) {
                if (s == r.fs) { r.fm += m; r.fdn += dn; }
                else { r.nr = 2; r.ls = s; r.lm = m; r.ldn = dn; }
                return;
            }
            if (s == r.ls) { r.lm += m; r.ldn += dn; return; }
            const A v = r.lm - r.ldn;   // a run between the first and the last: complete
            if (lt2(v, r.ls, r.bv, r.bi)) { r.bv = v; r.bi = r.ls; }
            if constexpr (P2) P[p_index(prows, tw_log2, prow(r.ls), c)] = v;
            r.ls = s; r.lm = m; r.ldn = dn;
        };
        constexpr int UQ = 8;   // chunks whose partials are loaded together
        for (int qa = q0; qa < q1; qa += UQ) {
            A xa[UQ], xh[UQ], xt[UQ], xv[UQ], dh[UQ], dt[UQ];
            int32_t xi[UQ];
            ChunkInfo ci[UQ];
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                const int q = min(qa + u, q1 - 1);   // clamped: every load in bounds
                const A *pq = part + (int64_t)q * 4 * ncp + c;
                xa[u] = pq[0];
                xh[u] = pq[1 * ncp];   // read even when unused (never written then)
                xt[u] = pq[2 * ncp];
                xv[u] = pq[3 * ncp];
                xi[u] = part_i[(int64_t)q * ncp + c];
                ci[u] = cinfo[q];
                dh[u] = cdn[2 * q];
                dt[u] = cdn[2 * q + 1];
            }
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                if (qa + u >= q1) break;
                r.accA += xa[u];
                if (xi[u] != INT_MAX && lt2(xv[u], xi[u], r.bv, r.bi)) { r.bv = xv[u]; r.bi = xi[u]; }
                if (ci[u].flags & kHead) add(ci[u].sa, xh[u], dh[u]);
                if (ci[u].flags & kTail) add(ci[u].sb, xt[u], dt[u]);
            }
        }
    }
    sm[g][j] = r;
    __syncthreads();
    A bestv = VT<T>::acc_inf();
    int besti = INT_MAX, cc = INT_MAX;
    if (g == 0 && live) {
        A accA = 0, bv = VT<T>::acc_inf(), rm = 0, rdn = 0;
        int bi = INT_MAX, rs = -1;
        auto flush = [&](int s, A m, A dn) {
            if (s < 0) return;
            const A v = m - dn;
            if (lt2(v, s, bv, bi)) { bv = v; bi = s; }
            if constexpr (P2) P[p_index(prows, tw_log2, prow(s), c)] = v;
        };
        for (int h = 0; h < kSmG; ++h) {
            const RunSum<A> &x = sm[h][j];
            accA += x.accA;
            if (x.bi != INT_MAX && lt2(x.bv, x.bi, bv, bi)) { bv = x.bv; bi = x.bi; }
            if (x.nr == 0) continue;
            if (x.fs == rs) { rm += x.fm; rdn += x.fdn; }
            else { flush(rs, rm, rdn); rs = x.fs; rm = x.fm; rdn = x.fdn; }
            if (x.nr == 2) {   // the first run ended inside the group
                flush(rs, rm, rdn);
                rs = x.ls; rm = x.lm; rdn = x.ldn;
            }
        }
        flush(rs, rm, rdn);
        const int e = st->empty_slot;   // an empty slot changes by 0 + B(c)
        if (e < k && lt2((A)0, e, bv, bi)) { bv = 0; bi = e; }
        A td;
        if constexpr (std::is_same<T, float>::value) td = st->td; else td = st->td_i;
        const A bsh = accA - td;
        if constexpr (P2) cand_a[c] = bsh;
        if (!is_med[c]) {
            bestv = bv + bsh;
            besti = bi;
            cc = (int)c;
        }
    }
    block_argmin3<A, kWG>(bestv, besti, cc);
    if (threadIdx.x == 0) {
        wg_v[blockIdx.x] = bestv;
        wg_i[blockIdx.x] = besti;
        wg_c[blockIdx.x] = cc;
    }
}

// ---- FastPAM1 select fused with the cache update: every block reduces the
// merge partials to the global best (value, slot, candidate) itself -- the
// same result in every block -- and, when the swap is taken, updates its
// objects' caches by the O(1) rule (objects that lost their nearest or second
// medoid are listed for a rescan).  Block 0 records the swap in the state.
template <typename T>
__global__ __launch_bounds__(256) void k_select_update(
    const AccT<T> *__restrict__ wg_v, const int32_t *__restrict__ wg_i,
    const int32_t *__restrict__ wg_c, int32_t nwg, const T *__restrict__ D, int64_t ld, int64_t n,
    int32_t *__restrict__ med, uint8_t *__restrict__ is_med, int32_t *__restrict__ near,
    int32_t *__restrict__ sec, T *__restrict__ dn, T *__restrict__ ds, int32_t *__restrict__ rlist,
    DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    if (st->done) return;
    A v = VT<T>::acc_inf();
    int i = INT_MAX, c = INT_MAX;
    for (int w = threadIdx.x; w < nwg; w += 256)
        if (lex_less(wg_v[w], wg_i[w], wg_c[w], v, i, c)) { v = wg_v[w]; i = wg_i[w]; c = wg_c[w]; }
    block_argmin3<A, 256>(v, i, c);
    bool apply;
    if constexpr (std::is_same<T, float>::value) apply = (c != INT_MAX) && (v < -st->margin);
    else apply = (c != INT_MAX) && (v < 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter += 1;
        st->best_i = i;
        st->best_c = c;
        if constexpr (std::is_same<T, float>::value) st->best_v = v;
        else { st->best_vi = v; st->best_v = (double)v; }
        if (!apply) {
            st->done = 1;
            st->swapped = 0;
        } else {
            const int old = med[i];
            is_med[old] = 0;
            is_med[c] = 1;
            med[i] = c;
            st->old_med = old;
            st->new_slot = i;
            st->new_med = c;
            st->swapped = 1;
            if constexpr (std::is_same<T, float>::value) st->td += v;
            else { st->td_i += v; st->td = (double)st->td_i; }
            if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, (double)v};
            st->swaps += 1;
        }
    }
    if (!apply) return;
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    const T dnew = D[(int64_t)c * ld + o];
    int32_t nr = near[o], sc = sec[o];
    T a = dn[o], b = ds[o];
    if (cache_update_o1<T>(i, dnew, nr, sc, a, b)) {
        rlist[atomicAdd(&st->n_list, 1)] = (int32_t)o;
    } else {
        near[o] = nr; sec[o] = sc; dn[o] = a; ds[o] = b;
    }
}

// ---- FasterPAM (Alg. 4): candidates are visited one at a time in index
// order, cyclically; each takes its best slot and is swapped in at once when
// that lowers TD.  On the device the scan is evaluated a window at a time:
// every candidate of [fw_base, fw_end) is scored against the current medoids
// in one pass, and the first one at or after the scan position fp_pos with
// an improving swap is exactly the candidate at which the sequential scan
// swaps next (nothing changes between the position and that candidate).  The
// swap is applied and the next window starts right after it; without one the
// scan moves to the window's end.  The scan ends once n consecutive
// positions went by without a swap, or after max_iter passes.

// Next window: starts at the scan position (rounded down to the load width;
// the positions before it are masked), fw_tiles tiles wide, not past n, the
// stop position or the pass cap.  The width adapts to the spacing of the
// swaps: one tile after a swap, doubled (up to the launch grid's max_tiles)
// after each window without one; results do not depend on it.
__device__ __forceinline__ void fp_window(DevState *st, int64_t n, int64_t tile, int32_t vec) {
    const long long pos = st->fp_pos;
    const long long base = pos - pos % vec;
    long long end = base + (long long)st->fw_tiles * tile;
    if (end > n) end = n;
    const long long rest = (long long)n - st->fp_quiet;
    if (end > pos + rest) end = pos + rest;
    const long long left = st->fp_limit - st->fp_visited;
    if (end > pos + left) end = pos + left;
    st->fw_base = base;
    st->fw_end = end;
}

__global__ void k_fp_init(DevState *st, int64_t n, int64_t tile, int32_t vec, long long limit) {
    st->fp = 1;
    st->fw_tiles = 1;
    st->fp_pos = 0;
    st->fp_visited = 0;
    st->fp_quiet = 0;
    st->fp_limit = limit;
    st->seg_skip = 0;
    if (limit <= 0) {
        st->done = 1;
        st->capped = 1;
    } else {
        fp_window(st, n, tile, vec);
    }
}

// Merge of a window pass's partials (one per group of chunks, k_fp_pass).  A
// window has few candidates and many chunk groups, so 16 threads share a
// candidate: each merges a contiguous range of groups into a summary (sum of A, best complete segment, first and
// last segment run, which may continue into the neighbouring groups), and
// the candidate's first thread combines the 16 summaries in chunk order.
// The work-group (16 candidates) reports its first candidate at or after the
// scan position whose best change is below the acceptance threshold.
// candidates per window-merge work-group and the merge grid: 16 candidates
// (64-byte column segments) on 128 work-groups measured faster than 16 on 64,
// 8 on 128 or 256, and 4 on 256
constexpr int kFmCPB = 16;
constexpr int kFmGrid = 128;


template <typename T>
__global__ __launch_bounds__(256) void k_fp_merge(
    const AccT<T> *__restrict__ part, const int32_t *__restrict__ part_i,
    const ChunkInfo *__restrict__ cinfo, int32_t Q, int64_t cols, int32_t k,
    const AccT<T> *__restrict__ cdn, const uint8_t *__restrict__ is_med,
    const DevState *__restrict__ st, AccT<T> *__restrict__ wg_v, int32_t *__restrict__ wg_i,
    int32_t *__restrict__ wg_c) {
    using A = AccT<T>;
    constexpr int CPB = kFmCPB, G = 256 / kFmCPB;
    if (st->done) return;
    __shared__ RunSum<A> sm[G][CPB];
    __shared__ int first;
    __shared__ A resv;
    __shared__ int resi;
    const int j = threadIdx.x % CPB, g = threadIdx.x / CPB;
    const int64_t cb = st->fw_base, ce = st->fw_end;
    const int64_t ngrp = (ce - cb + CPB - 1) / CPB;
    int found = INT_MAX;
    // groups of 16 candidates, in increasing order per work-group: the first
    // improving candidate found ends the work-group's search
    for (int64_t grp = blockIdx.x; grp < ngrp && found == INT_MAX; grp += gridDim.x) {
        const int64_t cr = grp * CPB + j;   // partial column
        const int64_t c = cb + cr;
        const bool live = c < ce;
        RunSum<A> r;
        r.accA = 0; r.bv = VT<T>::acc_inf(); r.bi = INT_MAX; r.nr = 0;
        r.fs = -1; r.fm = 0; r.fdn = 0; r.ls = -1; r.lm = 0; r.ldn = 0;
        if (live) {
            const int per = (Q + G - 1) / G;
            const int q0 = g * per, q1 = min(Q, q0 + per);
            // the open run is (fs, fm, fdn) while nr == 1, else (ls, lm, ldn)
            auto add = [&](int s, A m, A dn) {
                if (r.nr == 0) { r.nr = 1; r.fs = s; r.fm = m; r.fdn = dn; return; }
                if (r.nr == 1) {
                    if (s == r.fs) { r.fm += m; r.fdn += dn; }
                    else { r.nr = 2; r.ls = s; r.lm = m; r.ldn = dn; }
                    return;
                }
                if (s == r.ls) { r.lm += m; r.ldn += dn; return; }
                const A v = r.lm - r.ldn;   // a run between the first and the last: complete
                if (lt2(v, r.ls, r.bv, r.bi)) { r.bv = v; r.bi = r.ls; }
                r.ls = s; r.lm = m; r.ldn = dn;
            };
            constexpr int UQ = 8;   // chunks whose partials are loaded together
            for (int qa = q0; qa < q1; qa += UQ) {
                A xa[UQ], xh[UQ], xt[UQ], xv[UQ], dh[UQ], dt[UQ];
                int32_t xi[UQ];
                ChunkInfo ci[UQ];
#pragma unroll
                for (int u = 0; u < UQ; ++u) {
                    const int q = min(qa + u, q1 - 1);   // clamped: every load in bounds
                    const A *pq = part + (int64_t)q * 4 * cols + cr;
                    xa[u] = pq[0];
                    xh[u] = pq[1 * cols];   // read even when unused (never written then)
                    xt[u] = pq[2 * cols];
                    xv[u] = pq[3 * cols];
                    xi[u] = part_i[(int64_t)q * cols + cr];
                    ci[u] = cinfo[q];
                    dh[u] = cdn[2 * q];
                    dt[u] = cdn[2 * q + 1];
                }
#pragma unroll
                for (int u = 0; u < UQ; ++u) {
                    if (qa + u >= q1) break;
                    r.accA += xa[u];
                    if (xi[u] != INT_MAX && lt2(xv[u], xi[u], r.bv, r.bi)) { r.bv = xv[u]; r.bi = xi[u]; }
                    if (ci[u].flags & kHead) add(ci[u].sa, xh[u], dh[u]);
                    if (ci[u].flags & kTail) add(ci[u].sb, xt[u], dt[u]);
                }
            }
        }
        sm[g][j] = r;
        if (threadIdx.x == 0) first = INT_MAX;
        __syncthreads();
        A bestv = VT<T>::acc_inf();
        int besti = INT_MAX;
        bool neg = false;
        if (g == 0 && live) {
            A accA = 0, bv = VT<T>::acc_inf(), rm = 0, rdn = 0;
            int bi = INT_MAX, rs = -1;
            auto flush = [&](int s, A m, A dn) {
                if (s < 0) return;
                const A v = m - dn;
                if (lt2(v, s, bv, bi)) { bv = v; bi = s; }
            };
            for (int h = 0; h < G; ++h) {
                const RunSum<A> &x = sm[h][j];
                accA += x.accA;
                if (x.bi != INT_MAX && lt2(x.bv, x.bi, bv, bi)) { bv = x.bv; bi = x.bi; }
                if (x.nr == 0) continue;
                if (x.fs == rs) { rm += x.fm; rdn += x.fdn; }
                else { flush(rs, rm, rdn); rs = x.fs; rm = x.fm; rdn = x.fdn; }
                if (x.nr == 2) {   // the first run ended inside the group
                    flush(rs, rm, rdn);
                    rs = x.ls; rm = x.lm; rdn = x.ldn;
                }
            }
            flush(rs, rm, rdn);
            const int e = st->empty_slot;   // an empty slot changes by 0 + B(c)
            if (e < k && lt2((A)0, e, bv, bi)) { bv = 0; bi = e; }
            A td;
            if constexpr (std::is_same<T, float>::value) td = st->td; else td = st->td_i;
            A thr;
            if constexpr (std::is_same<T, float>::value) thr = -st->margin; else thr = 0;
            bestv = bv + (accA - td);
            besti = bi;
            neg = !is_med[c] && c >= st->fp_pos && bestv < thr;
            if (neg) atomicMin(&first, (int)c);
        }
        __syncthreads();
        if (neg && (int)c == first) { resv = bestv; resi = besti; }
        __syncthreads();
        found = first;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        wg_c[blockIdx.x] = found;
        if (found != INT_MAX) { wg_v[blockIdx.x] = resv; wg_i[blockIdx.x] = resi; }
    }
}

// The window's outcome, by one thread: the swap (medoids, TD, trace) or the
// scan's advance, the scan bookkeeping, the stop rule and the next window.
template <typename T>
__device__ __forceinline__ void fp_decide(DevState *st, bool apply, AccT<T> v, int i, int c,
                                          int64_t n, int64_t tile, int32_t max_tiles, int32_t vec,
                                          int32_t *med, uint8_t *is_med,
                                          pamx_swap_record *trace) {
    st->iter += 1;
    const long long pos = st->fp_pos, end = st->fw_end;
    st->fp_cols += end - st->fw_base;
    if (apply) {
        st->best_i = i;
        st->best_c = c;
        const int old = med[i];
        is_med[old] = 0;
        is_med[c] = 1;
        med[i] = c;
        st->old_med = old;
        st->new_slot = i;
        st->new_med = c;
        if constexpr (std::is_same<T, float>::value) { st->best_v = v; st->td += v; }
        else { st->best_vi = v; st->best_v = (double)v; st->td_i += v; st->td = (double)st->td_i; }
        if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, (double)v};
        st->swaps += 1;
        st->fp_visited += (long long)c - pos + 1;
        st->fp_quiet = 0;
        st->fp_pos = (c + 1 == n) ? 0 : c + 1;
    } else {
        st->fp_visited += end - pos;
        st->fp_quiet += end - pos;
        st->fp_pos = (end == n) ? 0 : end;
    }
    st->swapped = apply ? 1 : 0;
    st->seg_skip = apply ? 0 : 1;
    st->fw_tiles = apply ? 1 : min(2 * st->fw_tiles, max_tiles);
    if (st->fp_quiet >= n) {
        st->done = 1;
    } else if (st->fp_visited >= st->fp_limit) {
        st->done = 1;
        st->capped = 1;
    } else {
        fp_window(st, n, tile, vec);
    }
}

// Every block finds the window's first improving candidate (the smallest
// one any merge work-group reported) -- the same in every block -- and,
// when there is one, updates its objects' caches by the O(1) rule (objects
// that need a rescan go to the grid-wide list of k_cache_rescan).  Block 0
// applies the swap or advances the scan, and places the next window.  Used
// above kRsMed medoids; k_fp_apply otherwise.
template <typename T>
__global__ __launch_bounds__(256) void k_fp_select_update(
    const AccT<T> *__restrict__ wg_v, const int32_t *__restrict__ wg_i,
    const int32_t *__restrict__ wg_c, int32_t nwg, const T *__restrict__ D, int64_t ld,
    int64_t n, int64_t tile, int32_t max_tiles, int32_t vec, int32_t *__restrict__ med,
    uint8_t *__restrict__ is_med,
    int32_t *__restrict__ near, int32_t *__restrict__ sec, T *__restrict__ dn, T *__restrict__ ds,
    int32_t *__restrict__ rlist, DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    if (st->done) return;
    __shared__ long long wfirst;   // (candidate << 32) | merge work-group
    if (threadIdx.x == 0) wfirst = LLONG_MAX;
    __syncthreads();
    for (int w = threadIdx.x; w < nwg; w += 256) {
        const int32_t c = wg_c[w];
        if (c != INT_MAX) atomicMin(&wfirst, ((long long)c << 32) | w);
    }
    __syncthreads();
    const bool apply = wfirst != LLONG_MAX;
    const int wb = apply ? (int)(wfirst & 0xffffffffLL) : 0;
    A v = 0;
    int i = 0, c = 0;
    if (apply) { v = wg_v[wb]; i = wg_i[wb]; c = wg_c[wb]; }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        fp_decide<T>(st, apply, v, i, c, n, tile, max_tiles, vec, med, is_med, trace);
    if (!apply) return;
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    const T dnew = D[(int64_t)c * ld + o];
    int32_t nr = near[o], sc = sec[o];
    T a = dn[o], b = ds[o];
    if (cache_update_o1<T>(i, dnew, nr, sc, a, b)) {
        rlist[atomicAdd(&st->n_list, 1)] = (int32_t)o;
    } else {
        near[o] = nr; sec[o] = sc; dn[o] = a; ds[o] = b;
    }
}

// After the decision of a window (slot i receives candidate c): every block
// updates its objects' caches by the O(1) rule, rescans those of its objects
// that need it (one wave per object, the medoids staged in LDS with the new
// one in its slot, so block 0's write of med does not have to be seen) and
// does k_seg_count's work for its objects (their slots counted, their dn and
// ds summed in the same fixed order).  hist: k ints of dynamic LDS.
template <typename T>
__device__ __forceinline__ void apply_update_count(
    int i, int c, const T *__restrict__ D, int64_t ld, int64_t n, int32_t k,
    const int32_t *__restrict__ med, int32_t *__restrict__ near, int32_t *__restrict__ sec,
    T *__restrict__ dn, T *__restrict__ ds, int32_t *__restrict__ blkcnt,
    AccT<T> *__restrict__ tdp, int32_t *__restrict__ hist) {
    using A = AccT<T>;
    static_assert(kObjBlk == 256, "one object per thread");
    constexpr int NW = kObjBlk / 64;
    __shared__ int32_t smed[kRsMed];
    __shared__ int32_t rl[kObjBlk];     // objects to rescan: one list per wave
    __shared__ int32_t wcnt[NW];
    __shared__ int32_t r_nr[kObjBlk];   // their new caches
    __shared__ T r_dn[kObjBlk], r_ds[kObjBlk];
    __shared__ A w1[NW], w2[NW];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t o = (int64_t)blockIdx.x * kObjBlk + t;
    for (int j = t; j < k; j += kObjBlk) { smed[j] = (j == i) ? c : med[j]; hist[j] = 0; }
    int32_t nr = 0, sc = 0;
    T a = 0, b = 0;
    bool resc = false;
    if (o < n) {
        const T dnew = D[(int64_t)c * ld + o];
        nr = near[o]; sc = sec[o]; a = dn[o]; b = ds[o];
        resc = cache_update_o1<T>(i, dnew, nr, sc, a, b);
        if (!resc) { near[o] = nr; sec[o] = sc; dn[o] = a; ds[o] = b; }
    }
    const unsigned long long msk = __ballot(resc);
    if (resc) rl[wv * 64 + __popcll(msk & ((1ull << lane) - 1ull))] = t;
    if (lane == 0) wcnt[wv] = __popcll(msk);
    __syncthreads();
    int m = 0;
    for (int u = 0; u < NW; ++u) m += wcnt[u];
    for (int idx = wv; idx < m; idx += NW) {
        int q = idx, u = 0;   // entry idx of the wave lists taken in order
        while (q >= wcnt[u]) { q -= wcnt[u]; ++u; }
        const int lt = rl[u * 64 + q];
        const int64_t ob = (int64_t)blockIdx.x * kObjBlk + lt;
        const Top2<T> tp = wave_scan_medoids<T>(D, ld, k, smed, ob, lane);
        if (lane == 0) {
            store_top2<T>(tp, ob, near, sec, dn, ds);
            r_nr[lt] = (tp.j1 == INT_MAX) ? 0 : tp.j1;
            r_dn[lt] = tp.d1;
            r_ds[lt] = tp.d2;
        }
    }
    __syncthreads();
    // k_seg_count's sums for this block, in its order
    A s1 = 0, s2 = 0;
    if (o < n) {
        if (resc) { nr = r_nr[t]; a = r_dn[t]; b = r_ds[t]; }
        atomicAdd(&hist[nr], 1);
        s1 = (A)a;
        s2 = (A)b;
    }
    s1 = wave_sum<A>(s1);
    s2 = wave_sum<A>(s2);
    if (lane == 0) { w1[wv] = s1; w2[wv] = s2; }
    __syncthreads();
    int32_t *dst = blkcnt + (int64_t)blockIdx.x * k;
    for (int j = t; j < k; j += kObjBlk) dst[j] = hist[j];
    if (t == 0) {
        A t1 = 0, t2 = 0;
        for (int u = 0; u < NW; ++u) { t1 += w1[u]; t2 += w2[u]; }
        tdp[2 * blockIdx.x] = t1;
        tdp[2 * blockIdx.x + 1] = t2;
    }
}

// FasterPAM's decision, cache update and count in one launch (k <= kRsMed):
// the decision as k_fp_select_update, then apply_update_count, so the rescan
// and count launches of the window step go away.  Objects of a cluster
// stored together would put their rescans on one block; the synthetic
// workloads, like most data, spread them.
template <typename T>
__global__ __launch_bounds__(kObjBlk) void k_fp_apply(
    const AccT<T> *__restrict__ wg_v, const int32_t *__restrict__ wg_i,
    const int32_t *__restrict__ wg_c, int32_t nwg, const T *__restrict__ D, int64_t ld,
    int64_t n, int32_t k, int64_t tile, int32_t max_tiles, int32_t vec, int32_t *__restrict__ med,
    uint8_t *__restrict__ is_med, int32_t *__restrict__ near, int32_t *__restrict__ sec,
    T *__restrict__ dn, T *__restrict__ ds, int32_t *__restrict__ blkcnt,
    AccT<T> *__restrict__ tdp, DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    if (st->done) return;
    extern __shared__ int32_t hist[];   // k counts
    __shared__ long long wfirst;        // (candidate << 32) | merge work-group
    const int t = threadIdx.x;
    if (t == 0) wfirst = LLONG_MAX;
    __syncthreads();
    for (int w = t; w < nwg; w += kObjBlk) {
        const int32_t c = wg_c[w];
        if (c != INT_MAX) atomicMin(&wfirst, ((long long)c << 32) | w);
    }
    __syncthreads();
    const bool apply = wfirst != LLONG_MAX;
    const int wb = apply ? (int)(wfirst & 0xffffffffLL) : 0;
    A v = 0;
    int i = 0, c = 0;
    if (apply) { v = wg_v[wb]; i = wg_i[wb]; c = wg_c[wb]; }
    if (blockIdx.x == 0 && t == 0) fp_decide<T>(st, apply, v, i, c, n, tile, max_tiles, vec, med, is_med, trace);
    if (!apply) return;   // the segments are kept (seg_skip)
    apply_update_count<T>(i, c, D, ld, n, k, med, near, sec, dn, ds, blkcnt, tdp, hist);
}

// ---- FastCLARANS (Sec. 3.4): one local search over a list of random draws.
// A draw that is a medoid is skipped; any other is a candidate as in Alg. 4
// (best slot, smallest on ties, swapped in when the change is below the
// acceptance threshold).  Draws that do not improve count as failures, a swap
// resets the count, and maxneighbor failures in a row end the search; so does
// the end of the list (not converged).  The device scores a window of draws
// against the current medoids at once and takes the first improving one
// unless the failures before it already end the search -- exactly the
// sequential order.  State: fp_pos = list position, fp_quiet = failures,
// fp_limit = list length, fp_cols = draws evaluated; the window [fw_base,
// fw_end) is in list positions, its width kClUnit << (fw_tiles - 1) draws.
constexpr int kClUnit = 64;      // draws in the window after a swap
constexpr int kClMax = 1024;     // widest window (draws)
constexpr int kClGrid = 256;     // work-groups of the scoring kernel
constexpr int kClWaves = 16;     // its waves per work-group (the draw's segments split over them)

__device__ __forceinline__ void cl_window(DevState *st) {
    const long long base = st->fp_pos;
    long long end = base + ((long long)kClUnit << (st->fw_tiles - 1));
    if (end > st->fp_limit) end = st->fp_limit;
    st->fw_base = base;
    st->fw_end = end;
}

__global__ void k_cl_init(DevState *st, long long len, long long maxneighbor) {
    st->fp = 1;
    st->fp_pos = 0;
    st->fp_quiet = 0;
    st->fp_limit = len;
    st->fp_cols = 0;
    st->fp_visited = maxneighbor;   // the failure limit
    st->seg_skip = 0;
    st->fw_tiles = 1;
    if (len <= 0) {
        st->done = 1;
        st->capped = 1;
    } else {
        cl_window(st);
    }
}

// Change of every draw of the window: one work-group per draw; its kClWaves
// waves take the segments in turn (lanes over the segment's objects, reading
// the candidate's row of D at the sorted objects: D symmetric), each segment
// summed by a wave butterfly, so every sum has a fixed order.  A segment
// costs two dependent reads (the sorted objects, then the row at them), so a
// draw is a chain of about k / kClWaves such steps: sixteen waves rather
// than four shorten it.
template <typename T>
__global__ __launch_bounds__(64 * kClWaves) void k_cl_eval(
    const T *__restrict__ D, int64_t ld, int32_t k, const int32_t *__restrict__ draws,
    const int32_t *__restrict__ srow, const T *__restrict__ sdn, const T *__restrict__ sds,
    const int32_t *__restrict__ seg_off, const uint8_t *__restrict__ is_med,
    const DevState *__restrict__ st, AccT<T> *__restrict__ out_v, int32_t *__restrict__ out_i) {
    using A = AccT<T>;
    constexpr int U = 4, NW = kClWaves;
    if (st->done) return;
    __shared__ A wv[NW], wa[NW];
    __shared__ int wi[NW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long base = st->fw_base, end = st->fw_end;
    // this wave's segments are w, w + NW, ...; up to 64 of them their bounds
    // stay in the lanes (read once per launch)
    const int nseg = (w < k) ? (k - w + NW - 1) / NW : 0;
    const bool cached = nseg <= 64;
    int32_t c_so = 0, c_se = 0;
    if (cached && lane < nseg) { c_so = seg_off[w + lane * NW]; c_se = seg_off[w + lane * NW + 1]; }
    auto seg_bounds = [&](int t, int32_t &so, int32_t &se) {
        if (cached) {
            so = __builtin_amdgcn_readlane(c_so, t);
            se = __builtin_amdgcn_readlane(c_se, t);
        } else {
            so = seg_off[w + t * NW];
            se = seg_off[w + t * NW + 1];
        }
    };
    // the first non-empty segment of this wave at or after its t-th
    auto next_seg = [&](int t, int32_t &so, int32_t &se) {
        for (; t < nseg; ++t) {
            seg_bounds(t, so, se);
            if (so < se) break;
        }
        return t;
    };
    // U slots per lane from chunk start cs of a segment [so, se), masked past
    // its end (in bounds; unused when masked)
    auto load_chunk = [&](int32_t cs, int32_t so, int32_t se, int32_t (&ob)[U], T (&lo)[U],
                          T (&hi)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t p = cs + lane + u * 64;
            const int32_t q = p < se ? p : so;
            ob[u] = srow[q];
            lo[u] = sdn[q];
            hi[u] = sds[q];
        }
    };
    for (long long j = base + blockIdx.x; j < end; j += gridDim.x) {
        const int64_t c = draws[j];
        const int64_t r = j - base;
        if (is_med[c]) {
            if (threadIdx.x == 0) { out_v[r] = VT<T>::acc_inf(); out_i[r] = -1; }
            continue;
        }
        const T *row = D + c * ld;
        A accA = 0, bv = VT<T>::acc_inf();
        int bi = INT_MAX;
        // the wave's segments as one stream of chunks of U * 64 objects (each
        // lane adds its objects of a segment in order): the next chunk's
        // sorted objects are read while the row entries of the current one
        // are gathered, so a chunk costs one dependent read, not two
        int32_t so = 0, se = 0;
        int t = next_seg(0, so, se);
        int32_t p0 = so;
        int32_t ob[U] = {}, ob2[U] = {};
        T lo[U] = {}, hi[U] = {}, lo2[U] = {}, hi2[U] = {};
        if (t < nseg) load_chunk(p0, so, se, ob, lo, hi);
        A M = 0, DN = 0;
        while (t < nseg) {
            T d[U];
#pragma unroll
            for (int u = 0; u < U; ++u) d[u] = row[ob[u]];
            int32_t nso = so, nse = se, np0 = p0 + U * 64;
            int nt = t;
            if (np0 >= se) {
                nt = next_seg(t + 1, nso, nse);
                np0 = nso;
            }
            if (nt < nseg) load_chunk(np0, nso, nse, ob2, lo2, hi2);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (p0 + lane + u * 64 < se) {
                    accA += (A)vmin(d[u], lo[u]);
                    M += (A)vmed3(d[u], lo[u], hi[u]);
                    DN += (A)lo[u];
                }
            }
            if (nt != t) {   // segment w + t * NW is complete
                const int sg = w + t * NW;
                const A v = wave_sum<A>(M) - wave_sum<A>(DN);
                if (lt2(v, sg, bv, bi)) { bv = v; bi = sg; }
                M = 0;
                DN = 0;
            }
            t = nt;
            p0 = np0;
            so = nso;
            se = nse;
#pragma unroll
            for (int u = 0; u < U; ++u) { ob[u] = ob2[u]; lo[u] = lo2[u]; hi[u] = hi2[u]; }
        }
        accA = wave_sum<A>(accA);
        if (lane == 0) { wv[w] = bv; wi[w] = bi; wa[w] = accA; }
        __syncthreads();
        if (threadIdx.x == 0) {
            A v = wv[0];
            int i = wi[0];
            A atot = wa[0];
            for (int u = 1; u < NW; ++u) {
                if (lt2(wv[u], wi[u], v, i)) { v = wv[u]; i = wi[u]; }
                atot += wa[u];
            }
            const int e = st->empty_slot;   // an empty slot changes by 0 + B(c)
            if (e < k && lt2((A)0, e, v, i)) { v = 0; i = e; }
            A td;
            if constexpr (std::is_same<T, float>::value) td = st->td; else td = st->td_i;
            out_v[r] = v + (atot - td);
            out_i[r] = i;
        }
        __syncthreads();
    }
}

// Every block finds, in list order, the first improving draw that comes
// before the failure limit (the same in every block), and updates its
// objects' caches when that draw is swapped in.  Block 0 applies the swap or
// ends / advances the search and places the next window.
template <typename T, bool FUSED>
__global__ __launch_bounds__(256) void k_cl_select_update(
    const AccT<T> *__restrict__ out_v, const int32_t *__restrict__ out_i,
    const int32_t *__restrict__ draws, const T *__restrict__ D, int64_t ld, int64_t n,
    int32_t *__restrict__ med, uint8_t *__restrict__ is_med, int32_t *__restrict__ near,
    int32_t *__restrict__ sec, T *__restrict__ dn, T *__restrict__ ds, int32_t *__restrict__ rlist,
    int32_t k, int32_t *__restrict__ blkcnt, AccT<T> *__restrict__ tdp,
    DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    if (st->done) return;
    static_assert(4 * 256 >= kClMax, "four window entries per thread");
    __shared__ int32_t wsum[4];
    __shared__ int first;
    __shared__ A sv;
    __shared__ int32_t si, sc_, sev;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // this thread's object's caches, read with the window's results (they do
    // not depend on the decision)
    const int64_t o = (int64_t)blockIdx.x * 256 + t;
    int32_t nr = 0, sc = 0;
    T a = 0, b = 0;
    if (o < n) { nr = near[o]; sc = sec[o]; a = dn[o]; b = ds[o]; }
    const long long base = st->fw_base, end = st->fw_end;
    const int W = (int)(end - base);
    const long long fails = st->fp_quiet, maxn = st->fp_visited;
    A thr;
    if constexpr (std::is_same<T, float>::value) thr = -st->margin; else thr = 0;
    // this thread's 4 consecutive entries; evaluated draws per thread,
    // exclusive scan
    A ev_v[4];
    int32_t ev_i[4], ev_c[4];
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = 4 * t + u;
        ev_i[u] = -1; ev_v[u] = 0; ev_c[u] = 0;
        if (r < W) { ev_i[u] = out_i[r]; ev_v[u] = out_v[r]; ev_c[u] = draws[base + r]; }
        if (ev_i[u] >= 0) ++cnt;
    }
    int x = cnt;   // inclusive scan over the wave, then the wave totals in order
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    if (t == 0) first = INT_MAX;
    __syncthreads();
    int before = x - cnt, total = 0;
    for (int u = 0; u < 4; ++u) {
        if (u < wv) before += wsum[u];
        total += wsum[u];
    }
    int mine = -1;   // this thread's first improving entry
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (mine >= 0 || ev_i[u] < 0) continue;
        if (fails + before < maxn && ev_v[u] < thr) { mine = u; atomicMin(&first, 4 * t + u); }
        else ++before;
    }
    __syncthreads();
    const bool apply = first != INT_MAX;
    // the entry's thread passes it on, with the draws evaluated up to and
    // including it
    if (apply && mine >= 0 && 4 * t + mine == first) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u == mine) { sv = ev_v[u]; si = ev_i[u]; sc_ = ev_c[u]; }
        sev = before + 1;
    }
    __syncthreads();
    A v = 0;
    int i = 0, c = 0;
    if (apply) { v = sv; i = si; c = sc_; }
    if (blockIdx.x == 0 && t == 0) {
        st->iter += 1;
        if (apply) {
            st->fp_cols += sev;
            st->best_i = i;
            st->best_c = c;
            const int old = med[i];
            is_med[old] = 0;
            is_med[c] = 1;
            med[i] = c;
            st->old_med = old;
            st->new_slot = i;
            st->new_med = c;
            if constexpr (std::is_same<T, float>::value) { st->best_v = v; st->td += v; }
            else { st->best_vi = v; st->best_v = (double)v; st->td_i += v; st->td = (double)st->td_i; }
            if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, (double)v};
            st->swaps += 1;
            st->fp_quiet = 0;
            st->fp_pos = base + first + 1;
            st->fw_tiles = 1;
        } else if (fails + total >= maxn) {
            st->fp_cols += maxn - fails;   // the search ends at the limit
            st->fp_quiet = maxn;
        } else {
            st->fp_cols += total;
            st->fp_quiet = fails + total;
            st->fp_pos = end;
            if ((kClUnit << st->fw_tiles) <= kClMax) st->fw_tiles += 1;
        }
        st->swapped = apply ? 1 : 0;
        st->seg_skip = apply ? 0 : 1;
        if (st->fp_quiet >= maxn) {
            st->done = 1;
        } else if (st->fp_pos >= st->fp_limit) {
            st->done = 1;
            st->capped = 1;
        } else {
            cl_window(st);
        }
    }
    if (!apply) return;
    if constexpr (FUSED) {
        // k <= kRsMed: the update, rescans and counts here (apply_update_count)
        extern __shared__ int32_t hist[];
        apply_update_count<T>(i, c, D, ld, n, k, med, near, sec, dn, ds, blkcnt, tdp, hist);
        return;
    }
    if (o >= n) return;
    const T dnew = D[(int64_t)c * ld + o];
    if (cache_update_o1<T>(i, dnew, nr, sc, a, b)) {
        rlist[atomicAdd(&st->n_list, 1)] = (int32_t)o;
    } else {
        near[o] = nr; sec[o] = sc; dn[o] = a; ds[o] = b;
    }
}

// ---- FastPAM2: best candidate of every slot, (value, candidate) order.
// Work-group (i, j) scans the j-th of S equal candidate ranges of slot i and
// leaves its (value, candidate) minimum in part_v/part_c[i * S + j];
// k_slot_reduce takes the lexicographic minimum of the S parts.
template <typename T>
__global__ __launch_bounds__(256) void k_slot_best(const AccT<T> *__restrict__ P,
                                                   const AccT<T> *__restrict__ cand_a,
                                                   const int32_t *__restrict__ seg_off, int64_t n,
                                                   int32_t Lc, int64_t prows, int32_t tw_log2,
                                                   const uint8_t *__restrict__ is_med,
                                                   AccT<T> *__restrict__ part_v,
                                                   int32_t *__restrict__ part_c, int64_t span,
                                                   const DevState *__restrict__ st) {
    using A = AccT<T>;
    if (st->done) return;
    const int i = blockIdx.x, j = blockIdx.y, S = gridDim.y;
    const bool empty = seg_off[i] == seg_off[i + 1];
    const int64_t x0 = (int64_t)j * span, x1 = min(x0 + span, n);
    const int64_t row = (int64_t)i + (empty ? 0 : seg_off[i] / Lc);
    A v = VT<T>::acc_inf();
    int c = INT_MAX, dummy = 0;
    for (int64_t x = x0 + threadIdx.x; x < x1; x += 256) {
        const A d = (empty ? (A)0 : P[p_index(prows, tw_log2, row, x)]) + cand_a[x];
        if (!is_med[x] && d < v) { v = d; c = (int)x; }   // ascending x: first minimum per thread
    }
    block_argmin3<A, 256>(v, dummy, c);
    if (threadIdx.x == 0) { part_v[(int64_t)i * S + j] = v; part_c[(int64_t)i * S + j] = c; }
}

template <typename T>
__global__ __launch_bounds__(256) void k_slot_reduce(const AccT<T> *__restrict__ part_v,
                                                     const int32_t *__restrict__ part_c, int S,
                                                     int32_t k, AccT<T> *__restrict__ slot_v,
                                                     int32_t *__restrict__ slot_c,
                                                     const DevState *__restrict__ st) {
    using A = AccT<T>;
    if (st->done) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    A v = VT<T>::acc_inf();
    int c = INT_MAX;
    for (int j = 0; j < S; ++j) {
        const A pv = part_v[(int64_t)i * S + j];
        const int pc = part_c[(int64_t)i * S + j];
        if (lt2(pv, pc, v, c)) { v = pv; c = pc; }
    }
    slot_v[i] = v;
    slot_c[i] = c;
}

// ---- FastPAM2 eager application (one work-group).  Slots with a negative
// best change are visited by (change, slot); a visit is skipped if its
// candidate became a medoid meanwhile, otherwise the swap's change is
// computed again against the current caches (sum of Eq. change over all
// objects) and the swap applied when negative.
template <typename T>
__global__ __launch_bounds__(1024) void k_eager_apply(
    const T *__restrict__ D, int64_t ld, int64_t n, int32_t k, int32_t *__restrict__ med,
    uint8_t *__restrict__ is_med, int32_t *__restrict__ near, int32_t *__restrict__ sec,
    T *__restrict__ dn, T *__restrict__ ds, const AccT<T> *__restrict__ slot_v,
    const int32_t *__restrict__ slot_c, int32_t *__restrict__ order, int32_t *__restrict__ rlist,
    DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    if (st->done) return;
    __shared__ int32_t cnt;
    __shared__ int32_t go;
    __shared__ int32_t nres;
    const int t = threadIdx.x;
    const int lane = t & 63;
    A thr;
    if constexpr (std::is_same<T, float>::value) thr = -st->margin; else thr = 0;
    if (t == 0) cnt = 0;
    __syncthreads();
    // rank the negative slots by (value, slot)
    for (int i = t; i < k; i += 1024) {
        const A vi = slot_v[i];
        if (!(slot_c[i] != INT_MAX && vi < thr)) continue;
        int r = 0;
        for (int j = 0; j < k; ++j) {
            const A vj = slot_v[j];
            if (slot_c[j] != INT_MAX && vj < thr && lt2(vj, j, vi, i)) ++r;
        }
        order[r] = i;
        atomicAdd(&cnt, 1);
    }
    __syncthreads();
    const int m = cnt;
    int applied = 0;
    for (int r = 0; r < m; ++r) {
        const int i = order[r];
        const int c = slot_c[i];
        if (is_med[c]) continue;   // uniform: all threads read the same byte
        const T *rowc = D + (int64_t)c * ld;
        A s = 0;
        for (int64_t o = t; o < n; o += 1024) {
            const T d = rowc[o];
            const T a = dn[o];
            if (near[o] == i) s += (A)vmin(d, ds[o]) - (A)a;   // cases (b1), (b2)
            else s += (A)vmin(d, a) - (A)a;                    // cases (a), (c)
        }
        s = block_sum<A, 1024>(s);
        if (t == 0) { go = (s < thr) ? 1 : 0; nres = 0; }
        __syncthreads();
        if (!go) { __syncthreads(); continue; }
        if (t == 0) {
            const int old = med[i];
            is_med[old] = 0;
            is_med[c] = 1;
            med[i] = c;
            if constexpr (std::is_same<T, float>::value) st->td += s; else { st->td_i += s; st->td = (double)st->td_i; }
            if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, (double)s};
            st->swaps += 1;
        }
        __syncthreads();
        for (int64_t o = t; o < n; o += 1024) {
            int32_t nr = near[o], sc = sec[o];
            T a = dn[o], b2 = ds[o];
            if (cache_update_o1<T>(i, rowc[o], nr, sc, a, b2)) {
                rlist[atomicAdd(&nres, 1)] = (int32_t)o;
            } else {
                near[o] = nr; sec[o] = sc; dn[o] = a; ds[o] = b2;
            }
        }
        __syncthreads();
        const int mr = nres;
        for (int idx = t >> 6; idx < mr; idx += 16) {
            const int64_t o = rlist[idx];
            const Top2<T> tt = wave_scan_medoids<T>(D, ld, k, med, o, lane);
            if (lane == 0) store_top2<T>(tt, o, near, sec, dn, ds);
        }
        ++applied;
        __syncthreads();
    }
    if (t == 0) {
        st->iter += 1;
        if (applied == 0) st->done = 1;
    }
}

// ---- FastPAM2 eager application over the whole chip (cooperative launch).
// The same visits, re-scores and decisions as k_eager_apply, with the
// objects spread over the grid: thread (b, t) owns objects b*256 + t +
// j*256*G, so an object's caches are read and written by one thread (its
// rescan by a wave of the same work-group) and need no exchange.  Per visit:
//   1. every work-group sums Eq. change over its objects (fixed tree order)
//      and writes the sum to red[parity][b];
//   2. grid barrier; every work-group adds red[parity][0..G) in one fixed
//      order, so all take the same decision on the same value;
//   3. if the swap is applied, work-group 0 records it (medoids, TD, trace)
//      and every work-group updates its objects (O(1) rule, wave rescans of
//      those that lost their nearest or second medoid).
// Up to kRsMed medoids, every work-group keeps its own copy of the medoids
// in LDS (it answers "is c a medoid now" and serves the rescans), so a visit
// needs one grid barrier; above that, a second barrier publishes work-group
// 0's medoid arrays before the rescans.  The partials alternate between two
// halves of red, so a work-group still reading one visit's sums is never
// overtaken by the next visit's writes (a barrier lies between).  Loops and
// branches are uniform over the grid: every work-group reaches every barrier.
constexpr int kEgT = 256;       // threads (and objects per round) of a work-group
constexpr int kEgMax = 1024;    // largest grid (red holds 2 * kEgMax sums)
constexpr int kEgCap = 128;     // grid used at most (measured, see eager_grid_t)
template <typename T>
__global__ __launch_bounds__(kEgT) void k_eager_grid(
    const T *__restrict__ D, int64_t ld, int64_t n, int32_t k, int32_t *__restrict__ med,
    uint8_t *__restrict__ is_med, int32_t *__restrict__ near, int32_t *__restrict__ sec,
    T *__restrict__ dn, T *__restrict__ ds, const AccT<T> *__restrict__ slot_v,
    const int32_t *__restrict__ slot_c, int32_t *__restrict__ order, AccT<T> *__restrict__ red,
    DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    // read by every work-group before its first barrier; written only after
    // the last one
    if (st->done) return;
    __shared__ int32_t rl[kEgT];
    __shared__ int32_t nres;
    __shared__ A tot_s;
    __shared__ int32_t smed[kRsMed];   // this work-group's copy of the medoids (k <= kRsMed)
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int G = gridDim.x;
    const bool lmed = k <= kRsMed;
    if (lmed)
        for (int j = t; j < k; j += kEgT) smed[j] = med[j];   // published by the barrier below
    A thr;
    if constexpr (std::is_same<T, float>::value) thr = -st->margin; else thr = 0;
    // rank the negative slots by (value, slot), spread over the grid; every
    // work-group counts them itself
    int cnt = 0;
    for (int i = blockIdx.x * kEgT + t; i < k; i += G * kEgT) {
        const A vi = slot_v[i];
        if (!(slot_c[i] != INT_MAX && vi < thr)) continue;
        int r = 0;
        for (int j = 0; j < k; ++j) {
            const A vj = slot_v[j];
            if (slot_c[j] != INT_MAX && vj < thr && lt2(vj, j, vi, i)) ++r;
        }
        order[r] = i;
    }
    for (int i = t; i < k; i += kEgT) cnt += (slot_c[i] != INT_MAX && slot_v[i] < thr) ? 1 : 0;
    const int m = block_sum<int, kEgT>(cnt);
    grid.sync();
    const int64_t stride = (int64_t)G * kEgT;
    const int64_t o0 = (int64_t)blockIdx.x * kEgT + t;
    int applied = 0, par = 0;
    for (int r = 0; r < m; ++r) {
        const int i = order[r];
        const int c = slot_c[i];
        bool taken;   // c is a medoid now: the same answer in every work-group
        if (lmed) {
            int hit = 0;
            for (int jj = t; jj < k; jj += kEgT) hit |= (smed[jj] == c);
            taken = __syncthreads_or(hit) != 0;
        } else {
            taken = is_med[c] != 0;
        }
        if (taken) continue;
        const T *rowc = D + (int64_t)c * ld;
        A s = 0;
        for (int64_t o = o0; o < n; o += stride) {
            const T d = rowc[o];
            const T a = dn[o];
            if (near[o] == i) s += (A)vmin(d, ds[o]) - (A)a;   // cases (b1), (b2)
            else s += (A)vmin(d, a) - (A)a;                    // cases (a), (c)
        }
        s = block_sum<A, kEgT>(s);
        A *rb = red + (int64_t)par * kEgMax;
        par ^= 1;
        if (t == 0) rb[blockIdx.x] = s;
        grid.sync();
        if (wv == 0) {
            A x = 0;
            for (int j = lane; j < G; j += 64) x += rb[j];
            for (int w = 32; w >= 1; w >>= 1) x += __shfl_xor(x, w);   // same sum in every lane
            if (lane == 0) tot_s = x;
        }
        __syncthreads();
        const A tot = tot_s;
        if (!(tot < thr)) continue;
        if (blockIdx.x == 0 && t == 0) {
            const int old = med[i];
            is_med[old] = 0;
            is_med[c] = 1;
            med[i] = c;
            if constexpr (std::is_same<T, float>::value) st->td += tot; else { st->td_i += tot; st->td = (double)st->td_i; }
            if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, (double)tot};
            st->swaps += 1;
        }
        if (lmed) {
            // every work-group updates its own copy of the medoids, so no
            // work-group reads what work-group 0 just wrote: no barrier
            if (t == 0) smed[i] = c;
            __syncthreads();
        } else {
            grid.sync();   // med and is_med from work-group 0 before the rescans
        }
        for (int64_t b0 = (int64_t)blockIdx.x * kEgT; b0 < n; b0 += stride) {
            if (t == 0) nres = 0;
            __syncthreads();
            const int64_t o = b0 + t;
            if (o < n) {
                int32_t nr = near[o], sc = sec[o];
                T a = dn[o], b2 = ds[o];
                if (cache_update_o1<T>(i, rowc[o], nr, sc, a, b2)) {
                    rl[atomicAdd(&nres, 1)] = (int32_t)o;
                } else {
                    near[o] = nr; sec[o] = sc; dn[o] = a; ds[o] = b2;
                }
            }
            __syncthreads();
            const int mr = nres;
            for (int idx = wv; idx < mr; idx += kEgT / 64) {
                const int64_t q = rl[idx];
                const Top2<T> tt = lmed ? wave_scan_medoids<T>(D, ld, k, smed, q, lane)
                                        : wave_scan_medoids<T>(D, ld, k, med, q, lane);
                if (lane == 0) store_top2<T>(tt, q, near, sec, dn, ds);
            }
            __syncthreads();
        }
        ++applied;
    }
    if (blockIdx.x == 0 && t == 0) {
        st->iter += 1;
        if (applied == 0) st->done = 1;
    }
}

// The same visits with each thread's objects held in registers (at most
// R per thread; the host picks R >= n / (grid * kEgT)).  An object's
// caches are read once per search and written back at its end; per visit a
// thread loads only its objects' entries of the candidate's row, all
// together, and the update reuses them.  Rescans still write the caches to
// memory (by a wave of the owner's work-group); the owner reloads those
// objects after the work-group barrier that follows the rescans.  All
// sums keep the order of k_eager_grid: the same decisions, bit for bit.
constexpr int kEgR = 16;   // largest R
constexpr int kEgSpin = 1 << 24;   // polls (about 64 cycles each) before a barrier wait fails
template <typename T, int R>
__global__ __launch_bounds__(kEgT) void k_eager_grid_r(
    const T *__restrict__ D, int64_t ld, int64_t n, int32_t k, int32_t *__restrict__ med,
    uint8_t *__restrict__ is_med, int32_t *__restrict__ near, int32_t *__restrict__ sec,
    T *__restrict__ dn, T *__restrict__ ds, const AccT<T> *__restrict__ slot_v,
    const int32_t *__restrict__ slot_c, int32_t *__restrict__ order, AccT<T> *__restrict__ red,
    DevState *__restrict__ st, pamx_swap_record *__restrict__ trace) {
    using A = AccT<T>;
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    if (st->done) return;
    __shared__ int32_t rl[kEgT * R];
    __shared__ int32_t nres;
    __shared__ A tot_s;
    __shared__ int32_t smed[kRsMed];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int G = gridDim.x;
    const bool lmed = k <= kRsMed;
    if (lmed)
        for (int j = t; j < k; j += kEgT) smed[j] = med[j];
    A thr;
    if constexpr (std::is_same<T, float>::value) thr = -st->margin; else thr = 0;
    int cnt = 0;
    for (int i = blockIdx.x * kEgT + t; i < k; i += G * kEgT) {
        const A vi = slot_v[i];
        if (!(slot_c[i] != INT_MAX && vi < thr)) continue;
        int r = 0;
        for (int j = 0; j < k; ++j) {
            const A vj = slot_v[j];
            if (slot_c[j] != INT_MAX && vj < thr && lt2(vj, j, vi, i)) ++r;
        }
        order[r] = i;
    }
    for (int i = t; i < k; i += kEgT) cnt += (slot_c[i] != INT_MAX && slot_v[i] < thr) ? 1 : 0;
    const int m = block_sum<int, kEgT>(cnt);
    // the visits' barrier: an arrival count after the two halves of red
    int32_t *bar = reinterpret_cast<int32_t *>(red + 2 * kEgMax);
    if (blockIdx.x == 0 && t == 0) __hip_atomic_store(bar, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int nbar = 0;
    const int64_t stride = (int64_t)G * kEgT;
    const int64_t o0 = (int64_t)blockIdx.x * kEgT + t;
    int32_t rn[R], rsc[R];
    T rdn[R], rds[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int64_t o = min(o0 + j * stride, n - 1);   // clamped: entries past n are unused
        rn[j] = near[o]; rsc[j] = sec[o]; rdn[j] = dn[o]; rds[j] = ds[o];
    }
    grid.sync();
    int applied = 0, par = 0;
    for (int r = 0; r < m; ++r) {
        const int i = order[r];
        const int c = slot_c[i];
        bool taken;
        if (lmed) {
            int hit = 0;
            for (int jj = t; jj < k; jj += kEgT) hit |= (smed[jj] == c);
            taken = __syncthreads_or(hit) != 0;
        } else {
            taken = is_med[c] != 0;
        }
        if (taken) continue;
        const T *rowc = D + (int64_t)c * ld;
        T dv[R];
#pragma unroll
        for (int j = 0; j < R; ++j) dv[j] = rowc[min(o0 + j * stride, n - 1)];
        A s = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (o0 + j * stride < n) {
                if (rn[j] == i) s += (A)vmin(dv[j], rds[j]) - (A)rdn[j];   // cases (b1), (b2)
                else s += (A)vmin(dv[j], rdn[j]) - (A)rdn[j];               // cases (a), (c)
            }
        }
        s = block_sum<A, kEgT>(s);
        A *rb = red + (int64_t)par * kEgMax;
        par ^= 1;
        // grid barrier without cache maintenance: the only data that crosses
        // work-groups here, the sums, is written and read with device-scope
        // atomic accesses (coherent at the device level), and the count is
        // incremented after the sum's store has completed
        ++nbar;
        if (t == 0) {
            __hip_atomic_store(&rb[blockIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int target = nbar * G;
            int spin = 0;
            while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spin > kEgSpin) { atomicOr(&st->sync_err, 1); break; }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (wv == 0) {
            A x = 0;
            for (int j = lane; j < G; j += 64)
                x += __hip_atomic_load(&rb[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int w = 32; w >= 1; w >>= 1) x += __shfl_xor(x, w);
            if (lane == 0) tot_s = x;
        }
        __syncthreads();
        const A tot = tot_s;
        if (!(tot < thr)) continue;
        if (blockIdx.x == 0 && t == 0) {
            const int old = med[i];
            is_med[old] = 0;
            is_med[c] = 1;
            med[i] = c;
            if constexpr (std::is_same<T, float>::value) st->td += tot; else { st->td_i += tot; st->td = (double)st->td_i; }
            if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, (double)tot};
            st->swaps += 1;
        }
        if (lmed) {
            if (t == 0) smed[i] = c;
        } else {
            grid.sync();   // med and is_med from work-group 0 before the rescans
        }
        if (t == 0) nres = 0;
        __syncthreads();
        uint32_t resc = 0;   // bit j: object j was listed for a rescan
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t o = o0 + j * stride;
            if (cache_update_o1<T>(i, dv[j], rn[j], rsc[j], rdn[j], rds[j]) && o < n) {
                rl[atomicAdd(&nres, 1)] = (int32_t)o;
                resc |= 1u << j;
            }
        }
        __syncthreads();
        const int mr = nres;
        for (int idx = wv; idx < mr; idx += kEgT / 64) {
            const int64_t q = rl[idx];
            const Top2<T> tt = lmed ? wave_scan_medoids<T>(D, ld, k, smed, q, lane)
                                    : wave_scan_medoids<T>(D, ld, k, med, q, lane);
            if (lane == 0) store_top2<T>(tt, q, near, sec, dn, ds);
        }
        __syncthreads();
        if (resc) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if ((resc >> j) & 1u) {
                    const int64_t o = o0 + j * stride;
                    rn[j] = near[o]; rsc[j] = sec[o]; rdn[j] = dn[o]; rds[j] = ds[o];
                }
            }
        }
        ++applied;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int64_t o = o0 + j * stride;
        if (o < n) { near[o] = rn[j]; sec[o] = rsc[j]; dn[o] = rdn[j]; ds[o] = rds[j]; }
    }
    if (blockIdx.x == 0 && t == 0) {
        st->iter += 1;
        if (applied == 0) st->done = 1;
    }
}

// Grid of k_eager_grid for n objects on the current device: one work-group
// per 256 objects, at most what can be resident at once (a cooperative
// launch requires it) and kEgMax; 0 if the device has no cooperative launch.
template <typename T>
static int32_t eager_grid_t(int64_t n) {
    int dev = 0, coop = 0, cus = 0, per = 0;
    if (!cooperative_allowed()) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_eager_grid<T>, kEgT, 0) != hipSuccess)
        return 0;
    int per_r = 0;   // the register forms' largest LDS use
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_r, k_eager_grid_r<T, kEgR>, kEgT, 0) !=
        hipSuccess)
        return 0;
    if (per_r < per) per = per_r;
    int64_t g = (n + kEgT - 1) / kEgT;
    const int64_t cap = (int64_t)cus * per;
    if (g > cap) g = cap;
    if (g > kEgMax) g = kEgMax;
    // fewer work-groups make the per-visit grid barrier cheaper: on the 1e5-point
    // workload 128 work-groups (about three objects per thread) beat 391 (one
    // each): SWAP phase 139.0 -> 134.8 ms per fit; 64: 136.6, 256: 136.3
    if (g > kEgCap) g = kEgCap;
    // PAMX_EAGER_GRID=g caps the grid further (equal results: the visits and
    // sums do not depend on it; lets small inputs take every register form)
    if (const char *e = std::getenv("PAMX_EAGER_GRID")) {
        const long c = std::strtol(e, nullptr, 10);
        if (c > 0 && g > c) g = c;
    }
    return (int32_t)(g < 1 ? 0 : g);
}
int32_t eager_grid(int64_t n, int32_t dtype) {
    return dtype == PAMX_I32 ? eager_grid_t<int32_t>(n) : eager_grid_t<float>(n);
}

// ================================================================ host side
template <typename T>
struct SwapPtrs {
    int32_t *near, *sec, *srow, *blkcnt, *seg_off, *part_i, *wg_i, *wg_c, *slot_c, *order, *rlist;
    T *dn, *ds, *sdn, *sds;
    uint8_t *is_med;
    AccT<T> *cdn, *part, *wg_v, *P, *cand_a, *slot_v, *tdp;
    int32_t *segtot;
    ChunkInfo *cinfo, *ginfo;
    DevState *st;
};

template <typename T>
static SwapPtrs<T> ptrs(const Layout &L, void *ws) {
    char *w = static_cast<char *>(ws);
    SwapPtrs<T> p;
    p.near = reinterpret_cast<int32_t *>(w + L.near);
    p.sec = reinterpret_cast<int32_t *>(w + L.sec);
    p.dn = reinterpret_cast<T *>(w + L.dn);
    p.ds = reinterpret_cast<T *>(w + L.ds);
    p.is_med = reinterpret_cast<uint8_t *>(w + L.is_med);
    p.srow = reinterpret_cast<int32_t *>(w + L.srow);
    p.sdn = reinterpret_cast<T *>(w + L.sdn);
    p.sds = reinterpret_cast<T *>(w + L.sds);
    p.blkcnt = reinterpret_cast<int32_t *>(w + L.blkcnt);
    p.tdp = reinterpret_cast<AccT<T> *>(w + L.tdp);
    p.segtot = reinterpret_cast<int32_t *>(w + L.segtot);
    p.seg_off = reinterpret_cast<int32_t *>(w + L.seg_off);
    p.cinfo = reinterpret_cast<ChunkInfo *>(w + L.blkbase);
    p.ginfo = (L.ginfo != SIZE_MAX) ? reinterpret_cast<ChunkInfo *>(w + L.ginfo) : nullptr;
    p.cdn = reinterpret_cast<AccT<T> *>(w + L.cdn);
    p.part = reinterpret_cast<AccT<T> *>(w + L.part);
    p.part_i = reinterpret_cast<int32_t *>(w + L.part_i);
    p.cand_a = reinterpret_cast<AccT<T> *>(w + L.cand_a);
    p.wg_v = reinterpret_cast<AccT<T> *>(w + L.wg_v);
    p.wg_i = reinterpret_cast<int32_t *>(w + L.wg_i);
    p.wg_c = reinterpret_cast<int32_t *>(w + L.wg_c);
    p.P = (L.P != SIZE_MAX) ? reinterpret_cast<AccT<T> *>(w + L.P) : nullptr;
    p.slot_v = reinterpret_cast<AccT<T> *>(w + L.slot_v);
    p.slot_c = reinterpret_cast<int32_t *>(w + L.slot_c);
    p.order = reinterpret_cast<int32_t *>(w + L.list);
    p.rlist = reinterpret_cast<int32_t *>(w + L.rlist);
    p.st = reinterpret_cast<DevState *>(w + L.state);
    return p;
}

template <typename T>
hipError_t enqueue_swap_init(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                             const pamx_options &opt, void *ws, hipStream_t s) {
    auto p = ptrs<T>(L, ws);
    const int64_t n = L.n;
    const int32_t k = L.k;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, p.st, opt.max_iter,
                       opt.trace ? opt.trace_cap : 0);
    int32_t *mark = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + L.mark);
    fill<uint8_t>(p.is_med, L.nc, 0, s);
    fill<int32_t>(mark, L.nc, 0, s);
    hipLaunchKernelGGL(k_check_medoids, dim3((k + 255) / 256), dim3(256), 0, s, medoids, k, L.nc,
                       mark, p.is_med, p.st);
    if (opt.variant == PAMX_FASTERPAM)
        hipLaunchKernelGGL(k_fp_init, dim3(1), dim3(1), 0, s, p.st, n, (int64_t)L.tile, L.vec,
                           (long long)opt.max_iter * (long long)n);
    return hipGetLastError();
}

template <typename T>
static hipError_t enqueue_caches(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                                 int32_t *labels, void *ws, hipStream_t s) {
    auto p = ptrs<T>(L, ws);
    const int64_t n = L.n;
    int64_t ldl;
    const T *Dl = loc_rows<T>(D, ld, L, ws, &ldl);
    hipLaunchKernelGGL(k_cache_init<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Dl,
                       ldl, n, L.k, medoids, p.near, p.sec, p.dn, p.ds, labels);
    return hipGetLastError();
}

// FasterPAM with the fused decision, update and count (k_fp_apply)
static bool fp_fused(const Layout &L) { return L.fw > 0 && L.k <= kRsMed; }

template <typename T>
static void enqueue_count(const Layout &L, const SwapPtrs<T> &p, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_count<T>, dim3(L.n_oblk), dim3(kObjBlk), (size_t)L.k * 4, s,
                       (const int32_t *)p.near, (const T *)p.dn, (const T *)p.ds, L.n, L.k,
                       p.blkcnt, p.tdp, p.st);
}

// Objects sorted by nearest slot, segment offsets, chunk map (the chunk
// map depends on the chunk length of L); count = false when the per-block
// counts are already there (k_fp_apply).
template <typename T>
static void enqueue_segments(const Layout &L, const SwapPtrs<T> &p, hipStream_t s,
                             bool count = true) {
    const int64_t n = L.n;
    const int32_t k = L.k;
    if (count) enqueue_count<T>(L, p, s);
    hipLaunchKernelGGL(k_seg_colscan, dim3((k + 3) / 4), dim3(256), 0, s, p.blkcnt, L.n_oblk, k,
                       p.segtot, (const DevState *)p.st);
    hipLaunchKernelGGL(k_seg_scatter<T>, dim3(L.n_oblk), dim3(kObjBlk), (size_t)(k + 1) * 4, s,
                       (const int32_t *)p.near, (const T *)p.dn, (const T *)p.ds, n, k,
                       (const int32_t *)p.blkcnt, (const int32_t *)p.segtot, p.seg_off,
                       (const AccT<T> *)p.tdp, L.n_oblk, L.L, L.Q, p.cinfo, p.srow, p.sdn, p.sds,
                       p.st);
}

// rows of FastPAM2's P per pass tile (k + Q, see p_index) and log2 of the tile width
static int64_t p_rows(const Layout &L) { return (int64_t)L.k + L.Q; }
static int32_t tw_log2(const Layout &L) { return L.vec == 4 ? 10 : 8; }

// win: FasterPAM window pass (L placed by set_window: L.L, L.Q are the
// window chunking, L.Qg its groups, the partials have L.fw columns)
template <typename T>
static void enqueue_pass(const T *D, int64_t ld, const Layout &L, const SwapPtrs<T> &p, bool p2,
                         hipStream_t s, bool win = false) {
    if (win && L.fwG > 1) {
        const dim3 wgrid(L.fwG, L.Qg);   // G column blocks per tile, Qg groups
#define PAMX_FPPASS(VEC, G)                                                                    \
        hipLaunchKernelGGL((k_fp_pass<T, VEC, G>), wgrid, dim3(kWG), 0, s, D, ld, L.n,         \
                           (const int32_t *)p.srow, (const T *)p.sdn, (const T *)p.sds,        \
                           (const int32_t *)p.seg_off, (const ChunkInfo *)p.cinfo, L.L, L.Q,   \
                           p.cdn, p.ginfo, p.part, p.part_i, (int64_t)L.fw,                    \
                           (const DevState *)p.st)
        if (L.vec == 4) {
            if (L.fwG == 4) PAMX_FPPASS(4, 4); else PAMX_FPPASS(4, 2);
        } else {
            if (L.fwG == 4) PAMX_FPPASS(1, 4); else PAMX_FPPASS(1, 2);
        }
#undef PAMX_FPPASS
        return;
    }
    const dim3 pgrid(win ? 1 : L.n_ctiles, L.Q);
    const int64_t cols = win ? L.fw : L.ncp;
#define PAMX_PASS(VEC, P2, WIN, PF)                                                           \
    hipLaunchKernelGGL((k_swap_pass<T, VEC, P2, WIN, PF>), pgrid, dim3(kWG), 0, s, D, ld, L.n, \
                       L.nc, L.k, (const int32_t *)p.srow, (const T *)p.sdn, (const T *)p.sds, \
                       (const int32_t *)p.seg_off, p.cdn,                                     \
                       (const ChunkInfo *)p.cinfo, L.L, cols, p.part, p.part_i, p.P,          \
                       p_rows(L), (const DevState *)p.st)
    // chunks of at least kPfChunk rows: the prefetching row loop
    const bool pf = !win && L.L >= kPfChunk;
    if (win) {
        if (L.vec == 4) PAMX_PASS(4, false, true, false); else PAMX_PASS(1, false, true, false);
    } else if (L.vec == 4) {
        if (pf) {
            if (p2) PAMX_PASS(4, true, false, true); else PAMX_PASS(4, false, false, true);
        } else {
            if (p2) PAMX_PASS(4, true, false, false); else PAMX_PASS(4, false, false, false);
        }
    } else {
        if (p2) PAMX_PASS(1, true, false, false); else PAMX_PASS(1, false, false, false);
    }
#undef PAMX_PASS
}

// Chunk tuning: the segments for L's chunk length, then `reps` SWAP passes,
// each between events ev[2r] and ev[2r+1].  The passes change no state that
// the next search reads (their partials are recomputed by every search).
template <typename T>
hipError_t enqueue_tune_passes(const T *D, int64_t ld, const Layout &L, const pamx_options &opt,
                               void *ws, hipStream_t s, hipEvent_t *ev, int reps) {
    auto p = ptrs<T>(L, ws);
    enqueue_segments<T>(L, p, s);
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(ev[2 * r], s);
        enqueue_pass<T>(D, ld, L, p, opt.variant == PAMX_FASTPAM2, s);
        (void)hipEventRecord(ev[2 * r + 1], s);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t enqueue_swap_iteration(const T *D, int64_t ld, const Layout &L, int32_t *medoids,
                                  const pamx_options &opt, void *ws, hipStream_t s,
                                  hipEvent_t ev0, hipEvent_t ev1) {
    using A = AccT<T>;
    auto p = ptrs<T>(L, ws);
    const int64_t n = L.n;
    const int32_t k = L.k;
    const bool p2 = opt.variant == PAMX_FASTPAM2;
    pamx_swap_record *trace = static_cast<pamx_swap_record *>(opt.trace);
    const unsigned ob = (unsigned)((n + 255) / 256);
    const int32_t smwg = (int32_t)((L.nc + kSmC - 1) / kSmC);   // SWAP merge work-groups

    if (opt.variant == PAMX_FASTERPAM) {
        // one window of the scan (segments are rebuilt only after a swap)
        const int nwg = (L.fw / kFmCPB < kFmGrid) ? L.fw / kFmCPB : kFmGrid;   // merge work-groups
        const bool fused = fp_fused(L);
        enqueue_segments<T>(L, p, s, !fused);
        if (ev0) (void)hipEventRecord(ev0, s);
        enqueue_pass<T>(D, ld, L, p, false, s, true);
        if (ev1) (void)hipEventRecord(ev1, s);
        // the merge reads per-group partials and run maps from k_fp_pass,
        // per-chunk ones from the long-chunk pass (L.Qg = L.Q then)
        hipLaunchKernelGGL(k_fp_merge<T>, dim3(nwg), dim3(256), 0, s, (const A *)p.part,
                           (const int32_t *)p.part_i,
                           (const ChunkInfo *)(L.fwG > 1 ? p.ginfo : p.cinfo), L.Qg,
                           (int64_t)L.fw, k, (const A *)p.cdn, (const uint8_t *)p.is_med,
                           (const DevState *)p.st, p.wg_v, p.wg_i, p.wg_c);
        if (fused) {
            hipLaunchKernelGGL(k_fp_apply<T>, dim3(L.n_oblk), dim3(kObjBlk), (size_t)k * 4, s,
                               (const A *)p.wg_v, (const int32_t *)p.wg_i,
                               (const int32_t *)p.wg_c, nwg, D, ld, n, k, (int64_t)L.tile,
                               L.fw / L.tile, L.vec, medoids, p.is_med, p.near, p.sec, p.dn,
                               p.ds, p.blkcnt, p.tdp, p.st, trace);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_fp_select_update<T>, dim3(ob), dim3(256), 0, s, (const A *)p.wg_v,
                           (const int32_t *)p.wg_i, (const int32_t *)p.wg_c, nwg, D, ld, n,
                           (int64_t)L.tile, L.fw / L.tile, L.vec, medoids, p.is_med, p.near,
                           p.sec, p.dn, p.ds,
                           p.rlist, p.st, trace);
        hipLaunchKernelGGL(k_cache_rescan<T>, dim3(256), dim3(256), 0, s, D, ld, k,
                           (const int32_t *)medoids, p.near, p.sec, p.dn, p.ds,
                           (const int32_t *)p.rlist, (const DevState *)p.st);
        return hipGetLastError();
    }
    enqueue_segments<T>(L, p, s);
    if (ev0) (void)hipEventRecord(ev0, s);
    enqueue_pass<T>(D, ld, L, p, p2, s);
    if (ev1) (void)hipEventRecord(ev1, s);
    if (p2) {
        hipLaunchKernelGGL((k_swap_merge<T, true>), dim3(smwg), dim3(kWG), 0, s,
                           (const A *)p.part, (const int32_t *)p.part_i, (const ChunkInfo *)p.cinfo,
                           L.Q, L.nc, k, L.ncp, (const A *)p.cdn, (const uint8_t *)p.is_med,
                           (const DevState *)p.st, p.P, p.cand_a, p.wg_v, p.wg_i, p.wg_c,
                           (const int32_t *)p.seg_off, L.L, p_rows(L), tw_log2(L));
        {
            A *sb_v = reinterpret_cast<A *>(static_cast<char *>(ws) + L.sb_v);
            int32_t *sb_c = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + L.sb_c);
            const int64_t span = (L.nc + L.sbS - 1) / L.sbS;
            hipLaunchKernelGGL(k_slot_best<T>, dim3(k, L.sbS), dim3(256), 0, s, (const A *)p.P,
                               (const A *)p.cand_a, (const int32_t *)p.seg_off, L.nc, L.L,
                               p_rows(L), tw_log2(L), (const uint8_t *)p.is_med, sb_v, sb_c, span,
                               (const DevState *)p.st);
            hipLaunchKernelGGL(k_slot_reduce<T>, dim3((k + 255) / 256), dim3(256), 0, s,
                               (const A *)sb_v, (const int32_t *)sb_c, L.sbS, k, p.slot_v,
                               p.slot_c, (const DevState *)p.st);
        }
        if (L.eg > 0) {
            const T *a_D = D;
            int64_t a_ld = ld, a_n = n;
            int32_t a_k = k;
            int32_t *a_med = medoids, *a_near = p.near, *a_sec = p.sec, *a_order = p.order;
            uint8_t *a_is_med = p.is_med;
            T *a_dn = p.dn, *a_ds = p.ds;
            const A *a_sv = p.slot_v;
            const int32_t *a_sc = p.slot_c;
            A *a_red = reinterpret_cast<A *>(static_cast<char *>(ws) + L.egred);
            DevState *a_st = p.st;
            pamx_swap_record *a_tr = trace;
            void *args[] = {&a_D, &a_ld, &a_n, &a_k, &a_med, &a_is_med, &a_near, &a_sec,
                            &a_dn, &a_ds, &a_sv, &a_sc, &a_order, &a_red, &a_st, &a_tr};
            // objects held in registers when every thread owns at most kEgR
            const int64_t per_t = (n + (int64_t)L.eg * kEgT - 1) / ((int64_t)L.eg * kEgT);
            const void *kern = reinterpret_cast<const void *>(k_eager_grid<T>);
            if (per_t <= 1) kern = reinterpret_cast<const void *>(k_eager_grid_r<T, 1>);
            else if (per_t <= 2) kern = reinterpret_cast<const void *>(k_eager_grid_r<T, 2>);
            else if (per_t <= 4) kern = reinterpret_cast<const void *>(k_eager_grid_r<T, 4>);
            else if (per_t <= 8) kern = reinterpret_cast<const void *>(k_eager_grid_r<T, 8>);
            else if (per_t <= kEgR) kern = reinterpret_cast<const void *>(k_eager_grid_r<T, kEgR>);
            const hipError_t e = hipLaunchCooperativeKernel(kern, dim3(L.eg), dim3(kEgT), args, 0, s);
            if (e != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL(k_eager_apply<T>, dim3(1), dim3(1024), 0, s, D, ld, n, k, medoids,
                               p.is_med, p.near, p.sec, p.dn, p.ds, (const A *)p.slot_v,
                               (const int32_t *)p.slot_c, p.order, p.rlist, p.st, trace);
        }
    } else {
        hipLaunchKernelGGL((k_swap_merge<T, false>), dim3(smwg), dim3(kWG), 0, s,
                           (const A *)p.part, (const int32_t *)p.part_i, (const ChunkInfo *)p.cinfo,
                           L.Q, L.nc, k, L.ncp, (const A *)p.cdn, (const uint8_t *)p.is_med,
                           (const DevState *)p.st, p.P, p.cand_a, p.wg_v, p.wg_i, p.wg_c,
                           (const int32_t *)p.seg_off, L.L, p_rows(L), tw_log2(L));
        int64_t ldl;
        const T *Dl = loc_rows<T>(D, ld, L, ws, &ldl);
        hipLaunchKernelGGL(k_select_update<T>, dim3(ob), dim3(256), 0, s, (const A *)p.wg_v,
                           (const int32_t *)p.wg_i, (const int32_t *)p.wg_c, smwg, Dl, ldl, n,
                           medoids, p.is_med, p.near, p.sec, p.dn, p.ds, p.rlist, p.st, trace);
        // the rescan reads row o of D at the medoid columns (consumer rows)
        hipLaunchKernelGGL(k_cache_rescan<T>, dim3(256), dim3(256), 0, s, D, ld, k,
                           (const int32_t *)medoids, p.near, p.sec, p.dn, p.ds,
                           (const int32_t *)p.rlist, (const DevState *)p.st);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t enqueue_cl_init(const Layout &L, int64_t len, int64_t maxneighbor, void *ws,
                           hipStream_t s) {
    auto p = ptrs<T>(L, ws);
    hipLaunchKernelGGL(k_cl_init, dim3(1), dim3(1), 0, s, p.st, (long long)len,
                       (long long)maxneighbor);
    // the first window's counts when the decision kernel counts the others
    if (L.k <= kRsMed) enqueue_count<T>(L, p, s);
    return hipGetLastError();
}

// one window of a FastCLARANS search (segments are rebuilt only after a swap)
template <typename T>
hipError_t enqueue_cl_step(const T *D, int64_t ld, const Layout &L, const int32_t *draws,
                           int32_t *medoids, const pamx_options &opt, void *ws, hipStream_t s) {
    using A = AccT<T>;
    auto p = ptrs<T>(L, ws);
    char *w = static_cast<char *>(ws);
    A *clv = reinterpret_cast<A *>(w + L.cl_v);
    int32_t *cli = reinterpret_cast<int32_t *>(w + L.cl_i);
    pamx_swap_record *trace = static_cast<pamx_swap_record *>(opt.trace);
    const unsigned ob = (unsigned)((L.n + 255) / 256);
    // up to kRsMed medoids the decision kernel also updates, rescans and
    // counts (the counts of the first window come from enqueue_cl_init)
    const bool fused = L.k <= kRsMed;
    enqueue_segments<T>(L, p, s, !fused);
    hipLaunchKernelGGL(k_cl_eval<T>, dim3(kClGrid), dim3(64 * kClWaves), 0, s, D, ld, L.k, draws,
                       (const int32_t *)p.srow, (const T *)p.sdn, (const T *)p.sds,
                       (const int32_t *)p.seg_off, (const uint8_t *)p.is_med,
                       (const DevState *)p.st, clv, cli);
    if (fused) {
        hipLaunchKernelGGL((k_cl_select_update<T, true>), dim3(ob), dim3(256), (size_t)L.k * 4, s,
                           (const A *)clv, (const int32_t *)cli, draws, D, ld, L.n, medoids,
                           p.is_med, p.near, p.sec, p.dn, p.ds, p.rlist, L.k, p.blkcnt, p.tdp,
                           p.st, trace);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_cl_select_update<T, false>), dim3(ob), dim3(256), 0, s, (const A *)clv,
                       (const int32_t *)cli, draws, D, ld, L.n, medoids, p.is_med, p.near, p.sec,
                       p.dn, p.ds, p.rlist, L.k, p.blkcnt, p.tdp, p.st, trace);
    hipLaunchKernelGGL(k_cache_rescan<T>, dim3(256), dim3(256), 0, s, D, ld, L.k,
                       (const int32_t *)medoids, p.near, p.sec, p.dn, p.ds,
                       (const int32_t *)p.rlist, (const DevState *)p.st);
    return hipGetLastError();
}

template <typename T>
hipError_t enqueue_finalize(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                            int32_t *labels, void *ws, hipStream_t s) {
    auto p = ptrs<T>(L, ws);
    hipError_t e = enqueue_caches<T>(D, ld, L, medoids, labels, ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_td_sum<T>, dim3(1), dim3(1024), 0, s, (const T *)p.dn, L.n, p.st);
    return hipGetLastError();
}

// caches for the first iteration (after enqueue_swap_init's medoid check)
template <typename T>
hipError_t enqueue_swap_caches(const T *D, int64_t ld, const Layout &L, const int32_t *medoids,
                               void *ws, hipStream_t s) {
    const hipError_t e = enqueue_caches<T>(D, ld, L, medoids, nullptr, ws, s);
    if (e != hipSuccess) return e;
    // FasterPAM with k_fp_apply: the first window's counts (later windows
    // get theirs from k_fp_apply)
    if (fp_fused(L)) enqueue_count<T>(L, ptrs<T>(L, ws), s);
    return hipGetLastError();
}

// The segment kernels on FP32 caches, for the mixed-precision form.
hipError_t launch_segments_f32(const int32_t *near, const float *dn, const float *ds, int64_t n,
                               int32_t k, int32_t n_oblk, int32_t *blkcnt, double *tdp,
                               int32_t *segtot, int32_t *seg_off, int32_t L, int32_t Q, void *cinfo,
                               int32_t *srow, float *sdn, float *sds, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_count<float>, dim3(n_oblk), dim3(kObjBlk), (size_t)k * 4, s, near, dn,
                       ds, n, k, blkcnt, tdp, st);
    hipLaunchKernelGGL(k_seg_colscan, dim3((k + 3) / 4), dim3(256), 0, s, blkcnt, n_oblk, k,
                       segtot, (const DevState *)st);
    hipLaunchKernelGGL(k_seg_scatter<float>, dim3(n_oblk), dim3(kObjBlk), (size_t)(k + 1) * 4, s,
                       near, dn, ds, n, k, (const int32_t *)blkcnt, (const int32_t *)segtot, seg_off,
                       (const double *)tdp, n_oblk, L, Q, static_cast<ChunkInfo *>(cinfo), srow, sdn,
                       sds, st);
    return hipGetLastError();
}

// explicit instantiations
#define PAMX_INST(T)                                                                           \
    template hipError_t run_build<T>(const T *, int64_t, const Layout &, int32_t, int32_t,     \
                                     int32_t *, void *, hipStream_t, hipEvent_t *);            \
    template hipError_t enqueue_swap_init<T>(const T *, int64_t, const Layout &,               \
                                             const int32_t *, const pamx_options &, void *,    \
                                             hipStream_t);                                     \
    template hipError_t enqueue_swap_iteration<T>(const T *, int64_t, const Layout &,          \
                                                  int32_t *, const pamx_options &, void *,     \
                                                  hipStream_t, hipEvent_t, hipEvent_t);        \
    template hipError_t enqueue_tune_passes<T>(const T *, int64_t, const Layout &,             \
                                               const pamx_options &, void *, hipStream_t,       \
                                               hipEvent_t *, int);                             \
    template hipError_t enqueue_finalize<T>(const T *, int64_t, const Layout &,                \
                                            const int32_t *, int32_t *, void *, hipStream_t);  \
    template hipError_t enqueue_swap_caches<T>(const T *, int64_t, const Layout &,             \
                                               const int32_t *, void *, hipStream_t);          \
    template hipError_t enqueue_cl_init<T>(const Layout &, int64_t, int64_t, void *,           \
                                           hipStream_t);                                       \
    template hipError_t enqueue_cl_step<T>(const T *, int64_t, const Layout &, const int32_t *, \
                                           int32_t *, const pamx_options &, void *, hipStream_t);
PAMX_INST(float)
PAMX_INST(int32_t)
#undef PAMX_INST

}  // namespace pamx
