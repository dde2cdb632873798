// init.hip -- the faster initialisations of Sec. 3.3 on gfx950.
//
// Distance-weighted seeding: the k-means++ idea with the distance to the
// nearest seed (the k-medoids loss term) as weight.  The first seed is
// floor(u_0 n); seed t is the first object, in index order, whose running
// weight sum exceeds u_t W, W the sum of all weights.  Seeds weigh 0 and are
// never drawn again; if W = 0 the smallest-index non-seed is taken.
//
// LAB (linear approximative BUILD): every BUILD step is restricted to a
// subsample listed by the caller: its non-medoid members are the candidates
// (in listed order, first strict minimum), its members the objects of the
// change, with the candidate's own drop to distance 0 counted unless the
// literal loop bounds are requested (as in BUILD).  If every member is a
// medoid the smallest-index non-medoid is taken.
//
// The uniforms and the subsamples are inputs, drawn by the caller.  Integer
// matrices: weights and changes are summed exactly in int64; FP32 ones in
// FP64 in a fixed order.
#include "pamx_internal.h"

namespace pamx {

constexpr int kIB = 256;   // objects per block

// Inclusive scan of one value per thread over a 256-thread block in a fixed
// order: wave scans, then the wave totals in order.  `total` receives the
// block's sum, which equals the last thread's inclusive value.
template <typename A>
__device__ A block_scan256(A x, A &total) {
    __shared__ A wt[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        const A y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wt[w] = x;
    __syncthreads();
    A off = 0;
    for (int u = 0; u < w; ++u) off += wt[u];
    total = ((wt[0] + wt[1]) + wt[2]) + wt[3];
    __syncthreads();
    return off + x;
}

// smallest index not among med[0..t)
__device__ int64_t first_free(const int32_t *med, int32_t t, int64_t n) {
    for (int64_t o = 0; o < n; ++o) {
        bool used = false;
        for (int32_t j = 0; j < t; ++j) used |= (med[j] == o);
        if (!used) return o;
    }
    return n - 1;
}

// One seeding step.  Every block finds seed t from the weights of step t-1
// (dn_in and its block sums bs_in: the same scan code made both, so the
// search sees the same sums in every block), then updates the weights of its
// own objects with the new seed's row (D symmetric) into dn_out / bs_out.
template <typename T>
__global__ __launch_bounds__(kIB) void k_dw_step(const T *__restrict__ D, int64_t ld, int64_t n,
                                                 int32_t t, const double *__restrict__ u,
                                                 const T *__restrict__ dn_in, T *__restrict__ dn_out,
                                                 const AccT<T> *__restrict__ bs_in,
                                                 AccT<T> *__restrict__ bs_out, int32_t nblk,
                                                 int32_t *__restrict__ med) {
    using A = AccT<T>;
    __shared__ long long sel;
    __shared__ A cum[kIB];
    const int tid = threadIdx.x;
    int64_t pick;
    if (t == 0) {
        const double f = floor(u[0] * (double)n);
        pick = (f < 0) ? 0 : (f >= (double)n ? n - 1 : (int64_t)f);
    } else {
        // W: block sums scanned in chunks of 256, carried in chunk order
        A W = 0;
        for (int b0 = 0; b0 < nblk; b0 += kIB) {
            const A x = (b0 + tid < nblk) ? bs_in[b0 + tid] : (A)0;
            A tot;
            (void)block_scan256<A>(x, tot);
            W += tot;
        }
        const double ut = u[t];
        pick = -1;
        if (W > 0) {
            const double target = ut * (double)W;
            // the block whose running sum first exceeds the target
            A carry = 0;
            int bsel = -1;
            A base = 0;
            for (int b0 = 0; b0 < nblk && bsel < 0; b0 += kIB) {
                const A x = (b0 + tid < nblk) ? bs_in[b0 + tid] : (A)0;
                A tot;
                const A inc = carry + block_scan256<A>(x, tot);
                cum[tid] = inc;
                if (tid == 0) sel = LLONG_MAX;
                __syncthreads();
                if (b0 + tid < nblk && (double)inc > target) atomicMin(&sel, (long long)tid);
                __syncthreads();
                if (sel != LLONG_MAX) {
                    bsel = b0 + (int)sel;
                    base = (sel == 0) ? carry : cum[sel - 1];
                }
                carry += tot;
                __syncthreads();
            }
            if (bsel < 0) bsel = nblk - 1;   // not reached for u < 1
            // the object inside that block
            const int64_t o = (int64_t)bsel * kIB + tid;
            const A w = (o < n) ? (A)dn_in[o] : (A)0;
            A tot;
            const A inc = base + block_scan256<A>(w, tot);
            if (tid == 0) sel = LLONG_MAX;
            __syncthreads();
            if (o < n && w > 0 && (double)inc > target) atomicMin(&sel, (long long)o);
            __syncthreads();
            if (sel == LLONG_MAX) {   // rounding at the block's end: its last weighted object
                if (tid == 0) sel = -1;
                __syncthreads();
                if (o < n && w > 0) atomicMax(&sel, (long long)o);
                __syncthreads();
            }
            pick = (sel >= 0 && sel != LLONG_MAX) ? (int64_t)sel : -1;
            __syncthreads();
        }
        if (pick < 0) pick = first_free(med, t, n);
    }
    const int64_t o = (int64_t)blockIdx.x * kIB + tid;
    A x = 0;
    if (o < n) {
        const T d = D[pick * ld + o];
        const T v = (t == 0) ? d : vmin(dn_in[o], d);
        dn_out[o] = v;
        x = (A)v;
    }
    A tot;
    (void)block_scan256<A>(x, tot);
    if (tid == 0) bs_out[blockIdx.x] = tot;
    if (blockIdx.x == 0 && tid == 0) med[t] = (int32_t)pick;
}

// LAB, step t: the change of every listed candidate over the subsample
// (one wave per candidate; lanes take every 64th member, then a butterfly).
template <typename T>
__global__ __launch_bounds__(256) void k_lab_eval(const T *__restrict__ D, int64_t ld, int32_t t,
                                                  const int32_t *__restrict__ S, int32_t m,
                                                  int32_t excl, const T *__restrict__ dn,
                                                  const uint8_t *__restrict__ is_med,
                                                  AccT<T> *__restrict__ vals) {
    using A = AccT<T>;
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= m) return;
    const int64_t c = S[j];
    if (is_med[c]) {
        if (lane == 0) vals[j] = VT<T>::acc_inf();
        return;
    }
    A acc = 0;
    for (int jj = lane; jj < m; jj += 64) {
        const int64_t o = S[jj];
        if (o == c) continue;
        const T d = D[c * ld + o];
        if (t == 0) {
            acc += (A)d;
        } else if (!is_med[o]) {
            const T w = dn[o];
            if (d < w) acc += (A)d - (A)w;
        }
    }
    acc = wave_sum<A>(acc);
    if (t > 0 && !excl) acc -= (A)dn[c];
    if (lane == 0) vals[j] = acc;
}

// LAB, step t: every block takes the first strict minimum of the changes
// (the same in every block), then lowers the nearest distance of its objects
// with the new medoid's row.  Block 0 records the medoid.
template <typename T>
__global__ __launch_bounds__(256) void k_lab_select_update(
    const AccT<T> *__restrict__ vals, int32_t m, const int32_t *__restrict__ S, int32_t t,
    const T *__restrict__ D, int64_t ld, int64_t n, T *__restrict__ dn,
    uint8_t *__restrict__ is_med, int32_t *__restrict__ med) {
    using A = AccT<T>;
    __shared__ A sv[256];
    __shared__ int sj[256];
    const int tid = threadIdx.x;
    A bv = VT<T>::acc_inf();
    int bj = INT_MAX;
    for (int j = tid; j < m; j += 256) {
        const A v = vals[j];
        if (v < bv) { bv = v; bj = j; }   // ascending j per thread: first minimum
    }
    sv[tid] = bv;
    sj[tid] = bj;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w && lt2(sv[tid + w], sj[tid + w], sv[tid], sj[tid])) {
            sv[tid] = sv[tid + w];
            sj[tid] = sj[tid + w];
        }
        __syncthreads();
    }
    const bool none = !(sv[0] < VT<T>::acc_inf());
    const int64_t c = none ? first_free(med, t, n) : (int64_t)S[sj[0]];
    const int64_t o = (int64_t)blockIdx.x * 256 + tid;
    if (o < n) {
        const T d = D[c * ld + o];
        dn[o] = (t == 0) ? d : vmin(dn[o], d);
    }
    if (blockIdx.x == 0 && tid == 0) {
        med[t] = (int32_t)c;
        is_med[c] = 1;
    }
}

template <typename X>
__global__ __launch_bounds__(256) void k_init_fill(X *__restrict__ p, int64_t cnt, X v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < cnt) p[i] = v;
}

// ---------------------------------------------------------------- host side
static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

InitLayout make_init_layout(int64_t n, int32_t m) {
    InitLayout L{};
    L.nblk = (int32_t)((n + kIB - 1) / kIB);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = up256(off + (bytes ? bytes : 1)); return o; };
    L.dn0 = take((size_t)n * 4);
    L.dn1 = take((size_t)n * 4);
    L.bs0 = take((size_t)L.nblk * 8);
    L.bs1 = take((size_t)L.nblk * 8);
    L.is_med = take((size_t)n);
    L.vals = take((size_t)(m > 0 ? m : 1) * 8);
    L.err = take(4);
    L.total = off;
    return L;
}

template <typename T>
hipError_t launch_init_dw(const T *D, int64_t ld, int64_t n, int32_t k, const double *u,
                          int32_t *med, void *ws, hipStream_t s) {
    using A = AccT<T>;
    const InitLayout L = make_init_layout(n, 0);
    char *w = static_cast<char *>(ws);
    T *dn[2] = {reinterpret_cast<T *>(w + L.dn0), reinterpret_cast<T *>(w + L.dn1)};
    A *bs[2] = {reinterpret_cast<A *>(w + L.bs0), reinterpret_cast<A *>(w + L.bs1)};
    for (int32_t t = 0; t < k; ++t) {
        const int a = t & 1, b = a ^ 1;
        hipLaunchKernelGGL(k_dw_step<T>, dim3(L.nblk), dim3(kIB), 0, s, D, ld, n, t, u,
                           (const T *)dn[b], dn[a], (const A *)bs[b], bs[a], L.nblk, med);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_lab(const T *D, int64_t ld, int64_t n, int32_t k, const int32_t *S,
                           int32_t m, int32_t excl, int32_t *med, void *ws, hipStream_t s) {
    using A = AccT<T>;
    const InitLayout L = make_init_layout(n, m);
    char *w = static_cast<char *>(ws);
    T *dn = reinterpret_cast<T *>(w + L.dn0);
    uint8_t *is_med = reinterpret_cast<uint8_t *>(w + L.is_med);
    A *vals = reinterpret_cast<A *>(w + L.vals);
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_init_fill<uint8_t>, dim3(nb), dim3(256), 0, s, is_med, n, (uint8_t)0);
    for (int32_t t = 0; t < k; ++t) {
        const int32_t *St = S + (int64_t)t * m;
        hipLaunchKernelGGL(k_lab_eval<T>, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, D, ld, t,
                           St, m, excl, (const T *)dn, (const uint8_t *)is_med, vals);
        hipLaunchKernelGGL(k_lab_select_update<T>, dim3(nb), dim3(256), 0, s, (const A *)vals, m, St,
                           t, D, ld, n, dn, is_med, med);
    }
    return hipGetLastError();
}

hipError_t launch_init_zero(int32_t *p, hipStream_t s) {
    hipLaunchKernelGGL(k_init_fill<int32_t>, dim3(1), dim3(256), 0, s, p, (int64_t)1, (int32_t)0);
    return hipGetLastError();
}

template hipError_t launch_init_dw<float>(const float *, int64_t, int64_t, int32_t, const double *,
                                          int32_t *, void *, hipStream_t);
template hipError_t launch_init_dw<int32_t>(const int32_t *, int64_t, int64_t, int32_t,
                                            const double *, int32_t *, void *, hipStream_t);
template hipError_t launch_init_lab<float>(const float *, int64_t, int64_t, int32_t, const int32_t *,
                                           int32_t, int32_t, int32_t *, void *, hipStream_t);
template hipError_t launch_init_lab<int32_t>(const int32_t *, int64_t, int64_t, int32_t,
                                             const int32_t *, int32_t, int32_t, int32_t *, void *,
                                             hipStream_t);

}  // namespace pamx
