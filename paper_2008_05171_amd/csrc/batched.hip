// batched.hip -- many independent PAM runs (CLARA subsamples) in one launch.
//
// CLARA (Sec. 2.1 of Schubert & Rousseeuw, arXiv 2008.05171) runs PAM on
// subsamples and keeps the run whose medoids give the smallest TD on the
// whole data set; with FastPAM1 inside, each run costs O(k n'^2) for BUILD
// and O(n'^2) per SWAP iteration (Sec. 3.4).
//
// k_clara: a persistent kernel.  Each work-group (1024 lanes, one per CU: its
// LDS holds one instance) takes tickets from an atomic work queue (largest
// estimated cost first) and runs BUILD (Alg. 1) and FastPAM1 SWAP (Alg. 3)
// for the ticket's instance entirely in LDS: the sample's points, the caches
// and the segment-sorted object order.  Distances are recomputed from the
// points in LDS (Euclidean FP32 or Manhattan int32), so nothing of size n'^2
// is stored.  Sums are FP64 (int64 for integer points) in a fixed order.
//
// A large instance is run by a team of T work-groups (T consecutive tickets)
// so that it does not set the length of the whole launch: member m evaluates
// the candidates m*1024 + lane + r*T*1024, every member keeps its own full
// copy of the points and caches (the same values: the same code on the same
// data), and the only exchange is the (value, slot, candidate) minimum of
// each BUILD step and SWAP iteration, through global memory and a team
// barrier.  The minimum of a total order does not depend on how the
// candidates are split, so a team's results equal one work-group's.  Teams
// need every member resident at once: they are formed only under a
// cooperative launch.
//
// k_full_assign + k_full_reduce: TD of every instance's medoids over all N
// points (FP32 distances, FP64 sums in a fixed order).
#include "pamx_internal.h"

namespace pamx {

constexpr int kBT = 1024;      // lanes per instance work-group
constexpr int kBR = 2;         // candidates per lane: n' <= kBT * kBR
constexpr int kBW = kBT / 64;  // waves per work-group

// Point distances (MD = compile-time bound on the dimension; FULL: the
// dimension equals MD, so no coordinate is tested and the loads go out
// together): Euclidean in FP32 for float points, the root by the hardware
// instruction (within 1 ulp; subnormals to 0), exact Manhattan for int32
// points.  The same function serves every distance of an instance, so
// d(o,c) = d(c,o) and d(o,o) = 0 exactly.
template <int MD, bool FULL>
__device__ __forceinline__ float pdist(const float *__restrict__ a, const float (&b)[MD], int dim) {
    float acc = 0.0f;
#pragma unroll
    for (int d = 0; d < MD; ++d) {
        if (FULL || d < dim) {
            const float t = a[d] - b[d];
            acc = fmaf(t, t, acc);
        }
    }
    return __builtin_amdgcn_sqrtf(acc);
}

template <int MD, bool FULL>
__device__ __forceinline__ int32_t pdist(const int32_t *__restrict__ a, const int32_t (&b)[MD],
                                         int dim) {
    int32_t acc = 0;
#pragma unroll
    for (int d = 0; d < MD; ++d)
        if (FULL || d < dim) acc += abs(a[d] - b[d]);
    return acc;
}

template <typename T, int MD, bool FULL>
__device__ __forceinline__ void load_pt(const T *__restrict__ src, int dim, T (&b)[MD]) {
#pragma unroll
    for (int d = 0; d < MD; ++d) b[d] = (FULL || d < dim) ? src[d] : T(0);
}

// Work-group lexicographic argmin over (v, i, c): waves by butterfly, then
// the 16 wave results in a fixed order.  Every lane returns the result.
template <typename A>
__device__ __forceinline__ void wg_argmin3(A &v, int &i, int &c, A *rv, int *ri, int *rc) {
    wave_argmin3(v, i, c);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { rv[w] = v; ri[w] = i; rc[w] = c; }
    __syncthreads();
    v = rv[0]; i = ri[0]; c = rc[0];
    for (int u = 1; u < kBW; ++u)
        if (lex_less(rv[u], ri[u], rc[u], v, i, c)) { v = rv[u]; i = ri[u]; c = rc[u]; }
    __syncthreads();
}

// Team-wide (value, slot, candidate) minimum for instance j: member m posts
// its work-group result in the exchange slots of this step's parity, arrives
// at the team's counter and waits until all T members have arrived at this
// step; every member then takes the minimum over the T posts.  Two parities:
// a member can post step g+1 while a slower one still reads step g, never
// step g+2 (that needs the slower one's arrival at g+1).  The wait is bounded
// (a count no correct run reaches): past it the kernel reports err |= 4 and
// the work-group leaves (returns false).
constexpr long long kSpinMax = 1ll << 24;
template <typename E>
__device__ bool team_argmin3(AccT<E> &v, int &i, int &c, int T, int m, int j, int &gen,
                             int32_t *__restrict__ bar, unsigned long long *__restrict__ xch,
                             int32_t *__restrict__ err, AccT<E> *rv, int *ri, int *rc) {
    using A = AccT<E>;
    if (T == 1) return true;
    __shared__ int ok_s;
    unsigned long long *slot = xch + ((size_t)(2 * j + (gen & 1)) * kBTeamMax) * 2;
    if (threadIdx.x == 0) {
        // the posts and the count are device-scope atomic accesses, coherent
        // at the device level without cache maintenance; the count is raised
        // only after the posts' stores have completed
        __hip_atomic_store(&slot[2 * m], __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&slot[2 * m + 1], ((unsigned long long)(uint32_t)i << 32) | (uint32_t)c,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
        __hip_atomic_fetch_add(&bar[j], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int want = (gen + 1) * T;
        long long spins = 0;
        int ok = 1;
        while (__hip_atomic_load(&bar[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinMax) { ok = 0; break; }
        }
        if (ok) {
            A bv = VT<E>::acc_inf();
            int bi = INT_MAX, bc = INT_MAX;
            for (int u = 0; u < T; ++u) {
                const unsigned long long a0 =
                    __hip_atomic_load(&slot[2 * u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long a1 =
                    __hip_atomic_load(&slot[2 * u + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const A uv = __builtin_bit_cast(A, a0);
                const int ui = (int)(uint32_t)(a1 >> 32), uc = (int)(uint32_t)a1;
                if (lex_less(uv, ui, uc, bv, bi, bc)) { bv = uv; bi = ui; bc = uc; }
            }
            rv[0] = bv; ri[0] = bi; rc[0] = bc;
        } else {
            atomicOr(err, 4);
        }
        ok_s = ok;
    }
    __syncthreads();
    const bool ok = ok_s != 0;
    if (ok) { v = rv[0]; i = ri[0]; c = rc[0]; }
    __syncthreads();
    ++gen;
    return ok;
}

template <typename A>
__device__ __forceinline__ A wg_sum(A x, A *rv) {
    x = wave_sum(x);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) rv[w] = x;
    __syncthreads();
    A s = rv[0];
    for (int u = 1; u < kBW; ++u) s += rv[u];
    __syncthreads();
    return s;
}

// LDS carve-up for one instance of at most n_max points and k_max medoids.
template <typename T>
struct BLds {
    T *P, *dn, *ds, *sdn, *sds;
    int32_t *near, *srow, *pos, *med, *seg, *wcnt;
    AccT<T> *DN;
    uint8_t *is_med;
};

__host__ __device__ inline size_t batched_lds_bytes(int n_max, int k_max, int dim, size_t esz) {
    size_t b = (size_t)n_max * dim * esz;            // P
    b += 4 * (size_t)n_max * esz;                     // dn, ds, sdn, sds
    b += 3 * (size_t)n_max * 4;                       // near, srow, pos
    b += (size_t)k_max * 4 + (size_t)(k_max + 1) * 4; // med, seg
    b += (size_t)kBW * k_max * 4;                     // wave counts
    b = (b + 7) & ~size_t(7);
    b += (size_t)k_max * 8;                           // DN
    b += (size_t)n_max;                               // is_med
    return (b + 15) & ~size_t(15);
}

template <typename T>
__device__ BLds<T> carve(unsigned char *base, int n_max, int k_max, int dim) {
    BLds<T> L;
    T *t = reinterpret_cast<T *>(base);
    L.P = t; t += (size_t)n_max * dim;
    L.dn = t; t += n_max;
    L.ds = t; t += n_max;
    L.sdn = t; t += n_max;
    L.sds = t; t += n_max;
    int32_t *q = reinterpret_cast<int32_t *>(t);
    L.near = q; q += n_max;
    L.srow = q; q += n_max;
    L.pos = q; q += n_max;
    L.med = q; q += k_max;
    L.seg = q; q += k_max + 1;
    L.wcnt = q; q += kBW * k_max;
    uintptr_t a = (reinterpret_cast<uintptr_t>(q) + 7) & ~uintptr_t(7);
    L.DN = reinterpret_cast<AccT<T> *>(a);
    L.is_med = reinterpret_cast<uint8_t *>(L.DN + k_max);
    return L;
}

// Nearest / second nearest of every object over the k medoids (fresh scan).
template <typename T, int MD, bool FULL>
__device__ void b_caches(const BLds<T> &L, int n, int k, int dim) {
    for (int o = threadIdx.x; o < n; o += kBT) {
        T b[MD];
        load_pt<T, MD, FULL>(L.P + (size_t)o * dim, dim, b);
        T d1 = VT<T>::inf(), d2 = VT<T>::inf();
        int j1 = INT_MAX;
        for (int j = 0; j < k; ++j) {
            const T d = pdist<MD, FULL>(L.P + (size_t)L.med[j] * dim, b, dim);
            if (d < d1) { d2 = d1; d1 = d; j1 = j; }
            else if (d < d2) { d2 = d; }
        }
        L.near[o] = (j1 == INT_MAX) ? 0 : j1;   // NaN distances only: keep the slot in range
        L.dn[o] = d1; L.ds[o] = d2;
    }
}

template <typename T, int MD, bool FULL>
__global__ __launch_bounds__(kBT) void k_clara(
    const T *__restrict__ X, int64_t N, int32_t dim, const int64_t *__restrict__ soff,
    const int32_t *__restrict__ sidx, const int32_t *__restrict__ kin,
    const int64_t *__restrict__ moff, const int32_t *__restrict__ tk_inst,
    const int32_t *__restrict__ tk_mem, const int32_t *__restrict__ tsz, int32_t n_tick,
    int32_t max_iter, int32_t excl, int32_t n_max, int32_t k_max, int32_t *__restrict__ med_out,
    double *__restrict__ td_out, double *__restrict__ tdb_out, int32_t *__restrict__ it_out,
    int32_t *__restrict__ sw_out, int32_t *__restrict__ rows_out, int32_t *__restrict__ queue,
    int32_t *__restrict__ bar, unsigned long long *__restrict__ xch, int32_t *__restrict__ err) {
    using A = AccT<T>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ A rv[kBW];
    __shared__ int ri[kBW], rc[kBW];
    __shared__ int job_s;
    const BLds<T> L = carve<T>(lds_raw, n_max, k_max, dim);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    for (;;) {
        if (tid == 0) job_s = atomicAdd(queue, 1);
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(job_s);
        __syncthreads();   // everyone has read job_s before thread 0 writes it again
        if (job >= n_tick) break;
        const int j = tk_inst[job];
        const int mem = tk_mem[job];      // member of the instance's team
        const int tsize = tsz[j];         // team size
        const int cb0 = mem * kBT, cstr = tsize * kBT;   // this member's candidates
        int gen = 0;                      // team steps so far
        const int64_t base = soff[j];
        const int n = (int)(soff[j + 1] - base);
        const int k = kin[j];

        // ---- points of the sample into LDS (indices were checked by k_check_sidx)
        for (int e = tid; e < n * dim; e += kBT) {
            const int t = e / dim, d = e - t * dim;
            L.P[e] = X[(int64_t)sidx[base + t] * dim + d];
        }
        for (int o = tid; o < n; o += kBT) { L.dn[o] = VT<T>::inf(); L.is_med[o] = 0; }
        __syncthreads();

        // ---- BUILD (Alg. 1): A(c) = sum_o min(d(o,c), dn(o)); step 0 has dn = inf.
        // Each lane keeps A of its candidates across steps.  After the first two
        // steps only objects whose dn dropped change A:
        //   A(c) += sum over them of min(d, dn_new) - min(d, dn_old),
        // taken from a stable list (ascending object) of those objects in LDS
        // (srow: object, sdn: old dn, sds: new dn; free until SWAP).
        A acand[kBR];
        int nchg = 0, rows = 0;
        bool failed = false;   // uniform: no candidate had a finite BUILD sum
        for (int step = 0; step < k; ++step) {
            A bv = VT<T>::acc_inf();
            int bc = INT_MAX, zero = 0;
            for (int r = 0; r < kBR; ++r) {
                const int c = cb0 + tid + r * cstr;
                if (c >= n || L.is_med[c]) continue;
                T b[MD];
                load_pt<T, MD, FULL>(L.P + (size_t)c * dim, dim, b);
                A acc;
                if (step < 2) {
                    acc = 0;
                    for (int o = 0; o < n; ++o)
                        acc += (A)vmin(pdist<MD, FULL>(L.P + (size_t)o * dim, b, dim), L.dn[o]);
                } else {
                    acc = acand[r];
                    // four listed objects at a time, their LDS reads issued
                    // together (same order of additions)
                    int q = 0;
                    for (; q + 4 <= nchg; q += 4) {
                        int32_t ob[4];
                        T d[4], lo[4], hi[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            ob[u] = L.srow[q + u]; lo[u] = L.sdn[q + u]; hi[u] = L.sds[q + u];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) d[u] = pdist<MD, FULL>(L.P + (size_t)ob[u] * dim, b, dim);
#pragma unroll
                        for (int u = 0; u < 4; ++u) acc += (A)vmin(d[u], hi[u]) - (A)vmin(d[u], lo[u]);
                    }
                    for (; q < nchg; ++q) {
                        const T d = pdist<MD, FULL>(L.P + (size_t)L.srow[q] * dim, b, dim);
                        acc += (A)vmin(d, L.sds[q]) - (A)vmin(d, L.sdn[q]);
                    }
                }
                acand[r] = acc;
                if (excl && step > 0) acc += (A)L.dn[c];
                if (acc < bv) { bv = acc; bc = c; }
            }
            wg_argmin3<A>(bv, zero, bc, rv, ri, rc);
            if (!team_argmin3<T>(bv, zero, bc, tsize, mem, j, gen, bar, xch, err, rv, ri, rc)) return;
            // Every sum compared false: NaN distances (non-finite coordinates).
            // bc is work-group (and team) uniform, so the whole instance stops
            // here; its medoids are reported as -1 and the call fails.
            if (bc == INT_MAX) {
                if (tid == 0) atomicOr(err, 8);
                failed = true;
                break;
            }
            const int m = bc;
            if (tid == 0) { L.med[step] = m; L.is_med[m] = 1; }
            T b[MD];
            load_pt<T, MD, FULL>(L.P + (size_t)m * dim, dim, b);
            // dn update and the list of objects whose dn dropped
            int base = 0;
            for (int b0 = 0; b0 < n; b0 += kBT) {
                const int o = b0 + tid;
                bool chg = false;
                T old = 0, nw = 0;
                if (o < n) {
                    const T d = pdist<MD, FULL>(L.P + (size_t)o * dim, b, dim);
                    old = L.dn[o];
                    nw = (step == 0) ? d : vmin(old, d);
                    chg = nw < old;
                    L.dn[o] = nw;
                }
                const unsigned long long msk = __ballot(chg);
                if (lane == 0) L.wcnt[wv] = __popcll(msk);
                __syncthreads();
                int pre = 0, tot = 0;
                for (int u = 0; u < kBW; ++u) {
                    const int c = L.wcnt[u];
                    if (u < wv) pre += c;
                    tot += c;
                }
                if (chg) {
                    const int p = base + pre + __popcll(msk & ((1ull << lane) - 1ull));
                    L.srow[p] = o; L.sdn[p] = old; L.sds[p] = nw;
                }
                base += tot;
                __syncthreads();
            }
            nchg = base;
            if (step >= 1 && step + 1 < k) rows += nchg;   // read by the next step
        }
        A tdb = 0;
        for (int o = tid; o < n; o += kBT) tdb += (A)L.dn[o];
        tdb = wg_sum<A>(tdb, rv);

        // ---- FastPAM1 SWAP (Alg. 3)
        int iters = 0, swaps = 0;
        if (!failed && k >= 2 && k < n) {
            b_caches<T, MD, FULL>(L, n, k, dim);
            __syncthreads();
            while (iters < max_iter) {
                ++iters;
                // stable counting sort of the objects by nearest slot
                if (tid < k) L.seg[tid] = 0;
                __syncthreads();
                for (int b0 = 0; b0 < n; b0 += kBT) {
                    const int o = b0 + tid;
                    const int s = (o < n) ? L.near[o] : -1;
                    int rank = 0;
                    for (int q = 0; q < k; ++q) {
                        const unsigned long long msk = __ballot(s == q);
                        if (s == q) rank = __popcll(msk & ((1ull << lane) - 1ull));
                        if (lane == 0) L.wcnt[wv * k + q] = __popcll(msk);
                    }
                    __syncthreads();
                    if (tid < k) {
                        int run = L.seg[tid];
                        for (int u = 0; u < kBW; ++u) {
                            const int c = L.wcnt[u * k + tid];
                            L.wcnt[u * k + tid] = run;
                            run += c;
                        }
                        L.seg[tid] = run;
                    }
                    __syncthreads();
                    if (o < n) L.pos[o] = L.wcnt[wv * k + s] + rank;
                    __syncthreads();
                }
                if (tid == 0) {
                    int run = 0;
                    for (int s = 0; s < k; ++s) { const int c = L.seg[s]; L.seg[s] = run; run += c; }
                    L.seg[k] = run;
                }
                __syncthreads();
                for (int o = tid; o < n; o += kBT) {
                    const int p = L.seg[L.near[o]] + L.pos[o];
                    L.srow[p] = o; L.sdn[p] = L.dn[o]; L.sds[p] = L.ds[o];
                }
                __syncthreads();
                if (tid < k) {
                    A x = 0;
                    for (int q = L.seg[tid]; q < L.seg[tid + 1]; ++q) x += (A)L.sdn[q];
                    L.DN[tid] = x;
                }
                A td = 0, sds_sum = 0;
                for (int o = tid; o < n; o += kBT) { td += (A)L.dn[o]; sds_sum += (A)L.ds[o]; }
                td = wg_sum<A>(td, rv);
                sds_sum = wg_sum<A>(sds_sum, rv);   // (its barriers also publish DN)
                int empty = INT_MAX;
                for (int s = 0; s < k; ++s)
                    if (L.seg[s] == L.seg[s + 1]) { empty = s; break; }

                // the loss-change pass: each candidate of this lane over all objects
                // in segment order (one candidate at a time keeps the live state small)
                A bestv = VT<T>::acc_inf();
                int besti = INT_MAX, bestc = INT_MAX;
                for (int r = 0; r < kBR; ++r) {
                    const int c = cb0 + tid + r * cstr;
                    if (c >= n || L.is_med[c]) continue;
                    T cb[MD];
                    load_pt<T, MD, FULL>(L.P + (size_t)c * dim, dim, cb);
                    A accA = 0, bv = VT<T>::acc_inf();
                    int bi = INT_MAX;
                    for (int s = 0; s < k; ++s) {
                        const int q0 = L.seg[s], q1 = L.seg[s + 1];
                        if (q0 == q1) continue;
                        A M = 0;
                        // four objects of the segment at a time, their LDS
                        // reads issued together (same order of additions)
                        int q = q0;
                        for (; q + 4 <= q1; q += 4) {
                            int32_t ob[4];
                            T d[4], lo[4], hi[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                ob[u] = L.srow[q + u]; lo[u] = L.sdn[q + u]; hi[u] = L.sds[q + u];
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) d[u] = pdist<MD, FULL>(L.P + (size_t)ob[u] * dim, cb, dim);
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                accA += (A)vmin(d[u], lo[u]);
                                M += (A)vmed3(d[u], lo[u], hi[u]);
                            }
                        }
                        for (; q < q1; ++q) {
                            const T d = pdist<MD, FULL>(L.P + (size_t)L.srow[q] * dim, cb, dim);
                            const T lo = L.sdn[q], hi = L.sds[q];
                            accA += (A)vmin(d, lo);
                            M += (A)vmed3(d, lo, hi);
                        }
                        const A v = M - L.DN[s];
                        if (v < bv) { bv = v; bi = s; }
                    }
                    if (empty != INT_MAX && lt2((A)0, empty, bv, bi)) { bv = 0; bi = empty; }
                    const A dl = bv + (accA - td);
                    if (lex_less(dl, bi, c, bestv, besti, bestc)) { bestv = dl; besti = bi; bestc = c; }
                }
                wg_argmin3<A>(bestv, besti, bestc, rv, ri, rc);
                if (!team_argmin3<T>(bestv, besti, bestc, tsize, mem, j, gen, bar, xch, err, rv, ri, rc))
                    return;
                A thr;
                if constexpr (std::is_same<T, float>::value)
                    thr = -4.0 * ((double)n + 68.0) * 0x1p-53 * (double)sds_sum;
                else
                    thr = 0;
                if (!(bestc != INT_MAX && bestv < thr)) break;   // converged (uniform)
                if (tid == 0) {
                    L.is_med[L.med[besti]] = 0;
                    L.is_med[bestc] = 1;
                    L.med[besti] = bestc;
                }
                ++swaps;
                __syncthreads();
                b_caches<T, MD, FULL>(L, n, k, dim);
                __syncthreads();
            }
        }
        // ---- results: global medoid indices, TD of the sample (fresh sum)
        if (failed || (k >= 2 && k < n)) {
            // caches are current after the last swap (a failed instance
            // reports no medoids)
        } else {
            b_caches<T, MD, FULL>(L, n, k, dim);
        }
        __syncthreads();
        A td = 0;
        for (int o = tid; o < n; o += kBT) td += (A)L.dn[o];
        td = wg_sum<A>(td, rv);
        if (mem == 0) {   // one member writes the instance's results
            for (int s = tid; s < k; s += kBT) med_out[moff[j] + s] = failed ? -1 : sidx[base + L.med[s]];
        }
        if (tid == 0 && mem == 0) {
            td_out[j] = (double)td;
            tdb_out[j] = (double)tdb;
            it_out[j] = iters;
            rows_out[j] = rows;
            sw_out[j] = swaps;
        }
        __syncthreads();
    }
}

// Every sample index must lie in [0, N); checked before any instance runs.
__global__ __launch_bounds__(256) void k_check_sidx(const int32_t *__restrict__ sidx, int64_t total,
                                                    int64_t N, int32_t *__restrict__ err) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int32_t g = sidx[t];
    if (g < 0 || (int64_t)g >= N) atomicOr(err, 1);
}

// TD of instance j's medoids over all N points: one partial per block.
// Runs after k_clara: if that kernel flagged a bad sample index, some
// instances wrote no medoids, so nothing is read; every medoid index is also
// checked against [0, N) before it addresses X.
template <typename T, int MD, bool FULL>
__global__ __launch_bounds__(256) void k_full_assign(const T *__restrict__ X, int64_t N,
                                                     int32_t dim,
                                                     const int32_t *__restrict__ med_out,
                                                     const int64_t *__restrict__ moff,
                                                     int32_t nblk, double *__restrict__ part,
                                                     int32_t *__restrict__ err) {
    using A = AccT<T>;
    __shared__ T mc[kBMaxK * kBMaxDim];
    __shared__ A red[256];
    __shared__ int bad;
    if (*err) return;   // uniform: one address for the whole grid
    const int j = blockIdx.y;
    const int64_t m0 = moff[j];
    const int k = (int)(moff[j + 1] - m0);
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < k * dim; e += 256) {
        const int m = e / dim, d = e - m * dim;
        const int32_t g = med_out[m0 + m];
        if (g < 0 || (int64_t)g >= N) { bad = 1; mc[e] = T(0); }
        else mc[e] = X[(int64_t)g * dim + d];
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) { atomicOr(err, 2); part[(int64_t)j * nblk + blockIdx.x] = 0.0; }
        return;
    }
    A s = 0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (int64_t)nblk * 256) {
        T b[MD];
        load_pt<T, MD, FULL>(X + p * dim, dim, b);
        T best = VT<T>::inf();
        for (int m = 0; m < k; ++m) best = vmin(best, pdist<MD, FULL>(mc + m * dim, b, dim));
        s += (A)best;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)j * nblk + blockIdx.x] = (double)red[0];
}

__global__ __launch_bounds__(256) void k_full_reduce(const double *__restrict__ part, int32_t n_inst,
                                                     int32_t nblk, double *__restrict__ td_full) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n_inst) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)j * nblk + b];
    td_full[j] = s;
}

size_t batched_lds_bytes_host(int n_max, int k_max, int dim, size_t esz) {
    return batched_lds_bytes(n_max, k_max, dim, esz);
}

template <typename T, int MD, bool FULL>
static hipError_t launch_clara_md(const T *X, int64_t N, int32_t dim, const BatchArgs &a,
                                  hipStream_t s) {
    const size_t lds = batched_lds_bytes(a.n_max, a.k_max, dim, sizeof(T));
    const void *fn = reinterpret_cast<const void *>(&k_clara<T, MD, FULL>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (!a.coop) {
        hipLaunchKernelGGL((k_clara<T, MD, FULL>), dim3(a.grid), dim3(kBT), lds, s, X, N, dim, a.soff,
                           a.sidx, a.kin, a.moff, a.tk_inst, a.tk_mem, a.tsz, a.n_tick, a.max_iter,
                           a.excl, a.n_max, a.k_max, a.med_out, a.td_out, a.tdb_out, a.it_out,
                           a.sw_out, a.rows_out, a.queue, a.bar, a.xch, a.err);
        return hipGetLastError();
    }
    // teams: every work-group resident at once
    const T *p_X = X;
    int64_t p_N = N;
    int32_t p_dim = dim;
    const int64_t *p_soff = a.soff;
    const int32_t *p_sidx = a.sidx, *p_kin = a.kin;
    const int64_t *p_moff = a.moff;
    const int32_t *p_tki = a.tk_inst, *p_tkm = a.tk_mem, *p_tsz = a.tsz;
    int32_t p_ntick = a.n_tick, p_maxit = a.max_iter, p_excl = a.excl, p_nmax = a.n_max,
            p_kmax = a.k_max;
    int32_t *p_med = a.med_out;
    double *p_td = a.td_out, *p_tdb = a.tdb_out;
    int32_t *p_it = a.it_out, *p_sw = a.sw_out, *p_rows = a.rows_out, *p_queue = a.queue,
            *p_bar = a.bar, *p_err = a.err;
    unsigned long long *p_xch = a.xch;
    void *args[] = {&p_X,    &p_N,    &p_dim,  &p_soff, &p_sidx,  &p_kin,  &p_moff, &p_tki,
                    &p_tkm,  &p_tsz,  &p_ntick, &p_maxit, &p_excl, &p_nmax, &p_kmax, &p_med,
                    &p_td,   &p_tdb,  &p_it,   &p_sw,   &p_rows,  &p_queue, &p_bar, &p_xch,
                    &p_err};
    return hipLaunchCooperativeKernel(fn, dim3(a.grid), dim3(kBT), args, (unsigned)lds, s);
}

template <typename T, int MD, bool FULL>
static int resident_md1(size_t lds) {
    const void *fn = reinterpret_cast<const void *>(&k_clara<T, MD, FULL>);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_clara<T, MD, FULL>, kBT, lds) !=
        hipSuccess)
        return 0;
    return per;
}
// the variant launch_clara picks for this dimension
template <typename T, int MD>
static int resident_md(int32_t dim, size_t lds) {
    return dim == MD ? resident_md1<T, MD, true>(lds) : resident_md1<T, MD, false>(lds);
}

int batched_resident(int32_t dim, size_t lds, int32_t dtype, int *coop) {
    int dev = 0, cus = 0, c = 0;
    *coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (cooperative_allowed() &&
        hipDeviceGetAttribute(&c, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess)
        *coop = c;
    int per;
    if (dtype == PAMX_F32)
        per = dim <= 4 ? resident_md<float, 4>(dim, lds)
                       : (dim <= 8 ? resident_md<float, 8>(dim, lds)
                                   : resident_md<float, kBMaxDim>(dim, lds));
    else
        per = dim <= 4 ? resident_md<int32_t, 4>(dim, lds)
                       : (dim <= 8 ? resident_md<int32_t, 8>(dim, lds)
                                   : resident_md<int32_t, kBMaxDim>(dim, lds));
    return per * cus;
}

template <typename T>
hipError_t launch_clara(const T *X, int64_t N, int32_t dim, const BatchArgs &a, hipStream_t s) {
    if (dim == 4) return launch_clara_md<T, 4, true>(X, N, dim, a, s);
    if (dim < 4) return launch_clara_md<T, 4, false>(X, N, dim, a, s);
    if (dim == 8) return launch_clara_md<T, 8, true>(X, N, dim, a, s);
    if (dim < 8) return launch_clara_md<T, 8, false>(X, N, dim, a, s);
    if (dim == kBMaxDim) return launch_clara_md<T, kBMaxDim, true>(X, N, dim, a, s);
    return launch_clara_md<T, kBMaxDim, false>(X, N, dim, a, s);
}

template <typename T, int MD>
static void launch_full_md(const T *X, int64_t N, int32_t dim, const BatchArgs &a, hipStream_t s) {
    if (dim == MD)
        hipLaunchKernelGGL((k_full_assign<T, MD, true>), dim3(a.nblk, a.n_inst), dim3(256), 0, s, X,
                           N, dim, (const int32_t *)a.med_out, a.moff, a.nblk, a.part, a.err);
    else
        hipLaunchKernelGGL((k_full_assign<T, MD, false>), dim3(a.nblk, a.n_inst), dim3(256), 0, s,
                           X, N, dim, (const int32_t *)a.med_out, a.moff, a.nblk, a.part, a.err);
}

template <typename T>
hipError_t launch_full_assign(const T *X, int64_t N, int32_t dim, const BatchArgs &a,
                              hipStream_t s) {
    if (dim <= 4) launch_full_md<T, 4>(X, N, dim, a, s);
    else if (dim <= 8) launch_full_md<T, 8>(X, N, dim, a, s);
    else launch_full_md<T, kBMaxDim>(X, N, dim, a, s);
    hipLaunchKernelGGL(k_full_reduce, dim3((a.n_inst + 255) / 256), dim3(256), 0, s,
                       (const double *)a.part, a.n_inst, a.nblk, a.td_full);
    return hipGetLastError();
}

hipError_t launch_check_sidx(const int32_t *sidx, int64_t total, int64_t N, int32_t *err,
                             hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_sidx, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, sidx,
                       total, N, err);
    return hipGetLastError();
}

template hipError_t launch_clara<float>(const float *, int64_t, int32_t, const BatchArgs &, hipStream_t);
template hipError_t launch_clara<int32_t>(const int32_t *, int64_t, int32_t, const BatchArgs &,
                                          hipStream_t);
template hipError_t launch_full_assign<float>(const float *, int64_t, int32_t, const BatchArgs &,
                                              hipStream_t);
template hipError_t launch_full_assign<int32_t>(const int32_t *, int64_t, int32_t,
                                                const BatchArgs &, hipStream_t);

}  // namespace pamx
