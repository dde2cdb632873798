// dist.hip -- dissimilarity matrices for PAM (which consumes an n x n matrix,
// Sec. 2 of Schubert & Rousseeuw, arXiv 2008.05171).
//
//  * k_dist_l1_i32 : exact Manhattan distances of int32 points (VALU).
//  * k_dist_l2_f32 : Euclidean distances d = sqrt(max(|x|^2 + |y|^2 - 2 x.y, 0))
//                    of mean-centred points, the Gram term x.y on the FP32 matrix cores
//                    (v_mfma_f32_32x32x2_f32), the root by the hardware instruction
//                    (within 1 ulp; its error is small beside the Gram term's), 64 x 64
//                    tiles staged in LDS and written back as full 256-byte row segments.
//  * k_dist_l2_f32_upper : the same entries for dim <= 64, computed only for
//                    the tiles at or right of the diagonal and written twice (as
//                    computed and transposed) with 16-byte row stores; a work-group
//                    keeps its rows' points and walks eight column tiles, loading
//                    the next tile's points behind the current MFMA loop.
//  All write a zero diagonal and are bitwise symmetric.
#include <type_traits>

#include "pamx_internal.h"

namespace pamx {

// ---------------------------------------------------------------- L1 int32
// 64-row blocks against kL1C column tiles of 64: the row and column points
// are staged in LDS, kL1J coordinates at a time, offset by 2^31 as unsigned
// so that |a - b| + acc is one absolute-difference instruction (v_sad_u32).
// A thread computes 4 rows x 4 columns of a tile (rows t/16 + 16 i, columns
// t%16 + 16 v: conflict-free LDS reads, 64-byte row pieces per store).  The
// coordinate range check made before any distance bounds every sum below
// INT32_MAX, so the unsigned sums are the exact distances.
constexpr int kL1T = 64, kL1J = 64, kL1C = 4;
__global__ __launch_bounds__(256) void k_dist_l1_i32(const int32_t *__restrict__ X, int64_t n,
                                                     int32_t dim, int32_t *__restrict__ D,
                                                     int64_t ld) {
    __shared__ uint32_t xr[kL1T][kL1J + 1], xc[kL1T][kL1J + 1];
    const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
    const int64_t r0 = (int64_t)blockIdx.y * kL1T;
    for (int ct = 0; ct < kL1C; ++ct) {
        const int64_t c0 = ((int64_t)blockIdx.x * kL1C + ct) * kL1T;
        if (c0 >= n) break;   // uniform over the work-group
        uint32_t acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][v] = 0;
        for (int j0 = 0; j0 < dim; j0 += kL1J) {
            const int jn = min(kL1J, dim - j0);
            for (int e = t; e < kL1T * kL1J; e += 256) {
                const int pnt = e / kL1J, j = e % kL1J;
                uint32_t vr = 0x80000000u, vc = 0x80000000u;
                if (j < jn) {
                    if (r0 + pnt < n) vr = (uint32_t)X[(r0 + pnt) * dim + j0 + j] ^ 0x80000000u;
                    if (c0 + pnt < n) vc = (uint32_t)X[(c0 + pnt) * dim + j0 + j] ^ 0x80000000u;
                }
                xr[pnt][j] = vr;
                xc[pnt][j] = vc;
            }
            __syncthreads();
            for (int j = 0; j < jn; ++j) {
                uint32_t a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) { a[i] = xr[tr + 16 * i][j]; b[i] = xc[tc + 16 * i][j]; }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[i][v] += (a[i] > b[v]) ? (a[i] - b[v]) : (b[v] - a[i]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + tr + 16 * i;
            if (r >= n) continue;
            int32_t *row = D + r * ld;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t c = c0 + tc + 16 * v;
                if (c < n) row[c] = (int32_t)acc[i][v];
            }
        }
    }
}

hipError_t launch_dist_l1_i32(const int32_t *X, int64_t n, int32_t dim, int32_t *D, int64_t ld,
                              hipStream_t s) {
    const int64_t span = (int64_t)kL1T * kL1C;
    dim3 grid((unsigned)((n + span - 1) / span), (unsigned)((n + kL1T - 1) / kL1T));
    hipLaunchKernelGGL(k_dist_l1_i32, grid, dim3(256), 0, s, X, n, dim, D, ld);
    return hipGetLastError();
}

// ---------------------------------------------------------------- L1 range
// Per-coordinate minimum and maximum of integer points.  No L1 distance
// exceeds the sum over coordinates of (max - min); the host compares that
// sum with the int32 range of the stored distances before any distance is
// formed.  mm[2j] / mm[2j+1] receive the minimum / maximum of coordinate j.
constexpr int kRangePts = 4096;   // points per work-group
__global__ __launch_bounds__(256) void k_range_init(int32_t *__restrict__ mm, int32_t dim) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < 2 * dim) mm[t] = (t & 1) ? INT_MIN : INT_MAX;
}
__global__ __launch_bounds__(256) void k_range_i32(const int32_t *__restrict__ X, int64_t n,
                                                   int32_t dim, int32_t *__restrict__ mm) {
    const int64_t o0 = (int64_t)blockIdx.x * kRangePts;
    const int64_t o1 = min(o0 + (int64_t)kRangePts, n);
    for (int j = blockIdx.y; j < dim; j += gridDim.y) {
        int lo = INT_MAX, hi = INT_MIN;
        for (int64_t o = o0 + threadIdx.x; o < o1; o += 256) {
            const int32_t v = X[o * dim + j];
            lo = min(lo, v);
            hi = max(hi, v);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin(&mm[2 * j], lo);
            atomicMax(&mm[2 * j + 1], hi);
        }
    }
}

hipError_t launch_range_i32(const int32_t *X, int64_t n, int32_t dim, int32_t *mm, hipStream_t s) {
    hipLaunchKernelGGL(k_range_init, dim3((unsigned)((2 * dim + 255) / 256)), dim3(256), 0, s, mm, dim);
    dim3 grid((unsigned)((n + kRangePts - 1) / kRangePts), (unsigned)(dim < 1024 ? dim : 1024));
    hipLaunchKernelGGL(k_range_i32, grid, dim3(256), 0, s, X, n, dim, mm);
    return hipGetLastError();
}

// ---------------------------------------------------------------- centring
// Subtracting the mean does not change Euclidean distances but shrinks |x|^2,
// which bounds the cancellation error of the Gram form.  The mean of each
// coordinate is summed in FP64 in a fixed order (deterministic); the distance
// kernel subtracts it while staging points into LDS.
__global__ __launch_bounds__(256) void k_center_mean(const float *__restrict__ X, int64_t n,
                                                     int32_t dim, float *__restrict__ mean) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int64_t o = threadIdx.x; o < n; o += 256) acc += (double)X[o * dim + j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) mean[j] = (float)(red[0] / (double)n);
}

hipError_t launch_mean_f32(const float *X, int64_t n, int32_t dim, float *mean, hipStream_t s) {
    hipLaunchKernelGGL(k_center_mean, dim3(dim), dim3(256), 0, s, X, n, dim, mean);
    return hipGetLastError();
}

// ---------------------------------------------------------------- L2 f32 (MFMA)
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kT = 64;        // output tile edge
constexpr int kKC = 32;       // coordinates staged per LDS round (even)
constexpr int kLdsK = kKC + 1; // padded row stride of the staged points

// Work-group: 4 waves, each owns a 32 x 32 quarter of the 64 x 64 tile.
// v_mfma_f32_32x32x2_f32 operand layout (wave64): lane l supplies A[l%32][l/32]
// and B[l/32][l%32]; accumulator element v of lane l is C[8*(v/4) + 4*(l/32) +
// v%4][l%32].
__global__ __launch_bounds__(256) void k_dist_l2_f32(const float *__restrict__ X,
                                                     const float *__restrict__ mean, int64_t n,
                                                     int32_t dim, float *__restrict__ D,
                                                     int64_t ld) {
    __shared__ float xa[kT * kLdsK];
    __shared__ float xb[kT * kLdsK];
    __shared__ float na[kT], nb[kT];
    __shared__ float tile[kT * (kT + 4)];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * kT;   // rows (objects o)
    const int64_t c0 = (int64_t)blockIdx.x * kT;   // columns (candidates c)
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    float nacc = 0.0f;  // threads 0..63: row norms, 64..127: column norms

    for (int k0 = 0; k0 < dim; k0 += kKC) {
        const int kc = min(kKC, dim - k0);
        __syncthreads();
        for (int e = tid; e < kT * kKC; e += 256) {
            const int r = e / kKC, kk = e % kKC;
            float va = 0.0f, vb = 0.0f;
            if (kk < kc) {
                const float mu = mean[k0 + kk];
                if (r0 + r < n) va = X[(r0 + r) * dim + k0 + kk] - mu;
                if (c0 + r < n) vb = X[(c0 + r) * dim + k0 + kk] - mu;
            }
            xa[r * kLdsK + kk] = va;
            xb[r * kLdsK + kk] = vb;
        }
        __syncthreads();
        if (tid < 128) {
            const float *src = (tid < 64) ? &xa[tid * kLdsK] : &xb[(tid - 64) * kLdsK];
            for (int kk = 0; kk < kc; ++kk) nacc = fmaf(src[kk], src[kk], nacc);
        }
        const int i = lane & 31, h = lane >> 5;
        for (int kk = 0; kk < kc; kk += 2) {
            const float a = xa[(wr + i) * kLdsK + kk + h];
            const float b = xb[(wc + i) * kLdsK + kk + h];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    }
    if (tid < 64) na[tid] = nacc;
    else if (tid < 128) nb[tid - 64] = nacc;
    __syncthreads();

    {
        const int j = lane & 31, h = lane >> 5;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = wr + 8 * (v >> 2) + 4 * h + (v & 3);
            const int c = wc + j;
            const float s = (na[r] + nb[c]) - 2.0f * acc[v];
            float d = __builtin_amdgcn_sqrtf(fmaxf(s, 0.0f));   // within 1 ulp; subnormals to 0
            if (r0 + r == c0 + c) d = 0.0f;
            tile[r * (kT + 4) + c] = d;
        }
    }
    __syncthreads();
    // write 64 rows x 64 columns: each thread stores 4 float4 (16 per row)
    const bool full = (c0 + kT <= n) && ((ld & 3) == 0);
    for (int e = tid; e < kT * (kT / 4); e += 256) {
        const int r = e >> 4, q = (e & 15) * 4;
        const int64_t o = r0 + r;
        if (o >= n) continue;
        const float *t = &tile[r * (kT + 4) + q];
        float *dst = D + o * ld + c0 + q;
        if (full) {
            *reinterpret_cast<float4 *>(dst) = make_float4(t[0], t[1], t[2], t[3]);
        } else {
            for (int v = 0; v < 4; ++v)
                if (c0 + q + v < n) dst[v] = t[v];
        }
    }
}

// Upper-triangle form for dim <= kSD.  D is symmetric, so work-group (x, y)
// computes only the 64 x 64 tiles (y, t) with t >= y among its column tiles
// x*kCT .. x*kCT+kCT-1 and writes each twice: as computed (rows of block y)
// and transposed (rows of block t), both with 16-byte row stores from an LDS
// copy of the tile.  The MFMA work and the point loads are half the full
// matrix's; the stores are the same 4 n^2 bytes.  The work-group keeps its
// 64 rows' points in LDS; the next column tile's points are loaded into
// registers before the current tile's MFMA loop and first used when they are
// staged.  Every entry is one computed value written at (r, c) and at (c, r),
// so D is bitwise symmetric; the diagonal tile is written once with a zero
// diagonal.  Squared norms are summed by four threads per point in a fixed
// order.
// DP = the dimension padded to 16, 32 or 64 with zeros (0 x 0 products leave
// every sum unchanged).
// Measured on the 1e5 x 32 points (40 GB matrix): 7.55 ms = 5.3 TB/s, 94 % of
// the same stores alone (pamx_write_probe); 4 column tiles per work-group
// 7.78 ms, 16: 7.61.  The full-matrix strip form it replaced took 12.0 ms (its
// stores went from the MFMA accumulators, two 128-byte row pieces per store
// instruction; writing the transposed tile that way takes 32-byte pieces,
// 23.6 ms).  A load under a branch, or one used at once, ends in a wait for
// every outstanding memory operation of the wave, stores included (one
// in-order count on gfx950), hence the clamped, deferred point loads.
constexpr int kSD = 64;       // largest dimension of this form
constexpr int kCT = 8;        // column tiles per work-group
constexpr int kTL = kT + 1;   // odd row stride of the LDS tile: row and column reads both conflict-free
template <int DP>
__global__ __launch_bounds__(256) void k_dist_l2_f32_upper(const float *__restrict__ X,
                                                           const float *__restrict__ mean,
                                                           int64_t n, int32_t dim,
                                                           float *__restrict__ D, int64_t ld) {
    constexpr int kSLd = DP + 1;           // padded row stride of the staged points
    __shared__ float xa[kT * kSLd];
    __shared__ float xb[kT * kSLd];
    __shared__ float na[kT], nb[kT];
    __shared__ float smean[DP];
    __shared__ float tb[kT * kTL];
    constexpr int kPer = kT * DP / 256;    // staged values per thread
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t yb = blockIdx.y;
    const int64_t r0 = yb * kT;
    const int64_t nT = (n + kT - 1) / kT;
    int64_t t0 = (int64_t)blockIdx.x * kCT;
    if (t0 + kCT <= yb) return;   // every tile left of the diagonal (uniform)
    if (t0 < yb) t0 = yb;
    const int64_t tend = min(nT, (int64_t)blockIdx.x * kCT + kCT);
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

    // coordinates of 64 points (rows p0..p0+63) into registers, raw, from
    // clamped (always valid) addresses
    auto load = [&](int64_t p0, float (&v)[kPer]) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * 256;
            const int r = e / DP, kk = e % DP;
            const int kc = kk < dim ? kk : dim - 1;
            const int64_t pr = p0 + r < n ? p0 + r : n - 1;
            v[u] = X[pr * dim + kc];
        }
    };
    // centre and pad while staging: (x - mean) * 0 is the padding's 0 (x is a
    // finite coordinate of a valid point)
    auto store = [&](float *x, const float (&v)[kPer], int64_t p0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * 256;
            const int r = e / DP, kk = e % DP;
            const float keep = (kk < dim && p0 + r < n) ? 1.0f : 0.0f;
            x[r * kSLd + kk] = (v[u] - smean[kk]) * keep;
        }
    };
    // squared norms of the 64 staged points: four threads per point, each
    // over a quarter of the (padded) coordinates, then a fixed butterfly
    auto norms = [&](const float *x, float *nrm) {
        const int pnt = tid >> 2, part = tid & 3;
        float s2 = 0.0f;
#pragma unroll
        for (int kk = part * (DP / 4); kk < (part + 1) * (DP / 4); ++kk)
            s2 = fmaf(x[pnt * kSLd + kk], x[pnt * kSLd + kk], s2);
        s2 += __shfl_xor(s2, 1);
        s2 += __shfl_xor(s2, 2);
        if (part == 0) nrm[pnt] = s2;
    };
    if (tid < DP) smean[tid] = tid < dim ? mean[tid] : 0.0f;
    float va[kPer], vb[kPer];
    load(r0, va);
    load(t0 * kT, vb);
    __syncthreads();   // smean
    store(xa, va, r0);
    __syncthreads();
    norms(xa, na);
    const int i = lane & 31, h = lane >> 5;
    typedef float f4 __attribute__((ext_vector_type(4)));
    for (int64_t t = t0; t < tend; ++t) {
        const int64_t c0 = t * kT;
        __syncthreads();      // the previous tile's reads of xb and tb are done
        store(xb, vb, c0);
        __syncthreads();
        if (t + 1 < tend) load(c0 + kT, vb);   // next tile, in flight
        norms(xb, nb);
        floatx16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll 8
        for (int kk = 0; kk < DP; kk += 2) {
            const float a = xa[(wr + i) * kSLd + kk + h];
            const float b = xb[(wc + i) * kSLd + kk + h];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();      // nb complete
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = wr + 8 * (v >> 2) + 4 * h + (v & 3);
            const float s = (na[r] + nb[wc + i]) - 2.0f * acc[v];
            float d = __builtin_amdgcn_sqrtf(fmaxf(s, 0.0f));   // within 1 ulp; subnormals to 0
            if (r0 + r == c0 + wc + i) d = 0.0f;
            tb[r * kTL + wc + i] = d;
        }
        __syncthreads();
        const bool full = r0 + kT <= n && c0 + kT <= n;
        // as computed: D[r0 + r][c0 + q .. c0 + q + 3]; streaming stores (the
        // matrix is far larger than the caches)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + j * 256;
            const int r = e >> 4, q = (e & 15) * 4;
            const float *src = tb + r * kTL + q;
            if (full) {
                const f4 val = {src[0], src[1], src[2], src[3]};
                __builtin_nontemporal_store(val, reinterpret_cast<f4 *>(D + (r0 + r) * ld + c0 + q));
            } else if (r0 + r < n) {
                for (int u = 0; u < 4; ++u)
                    if (c0 + q + u < n) D[(r0 + r) * ld + c0 + q + u] = src[u];
            }
        }
        if (t != yb) {
            // transposed: D[c0 + c][r0 + q .. r0 + q + 3] = tile rows q..q+3 of column c
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = tid + j * 256;
                const int c = e >> 4, q = (e & 15) * 4;
                const float *src = tb + q * kTL + c;
                if (full) {
                    const f4 val = {src[0], src[kTL], src[2 * kTL], src[3 * kTL]};
                    __builtin_nontemporal_store(val, reinterpret_cast<f4 *>(D + (c0 + c) * ld + r0 + q));
                } else if (c0 + c < n) {
                    for (int u = 0; u < 4; ++u)
                        if (r0 + q + u < n) D[(c0 + c) * ld + r0 + q + u] = src[u * kTL];
                }
            }
        }
    }
}

// Measurement: the stores of k_dist_l2_f32_upper alone -- the same grid,
// work-group shape and store pattern (per 64 x 64 tile at or right of the
// diagonal, 16-byte streaming row stores as computed and transposed) writing
// the value v, with no loads and no arithmetic.  Entries (r, c), r, c < n,
// are written.
__global__ __launch_bounds__(256) void k_write_probe(float *__restrict__ D, int64_t n, int64_t ld,
                                                     float v) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x;
    const int64_t yb = blockIdx.y;
    const int64_t r0 = yb * kT;
    const int64_t nT = (n + kT - 1) / kT;
    int64_t t0 = (int64_t)blockIdx.x * kCT;
    if (t0 + kCT <= yb) return;
    if (t0 < yb) t0 = yb;
    const int64_t tend = min(nT, (int64_t)blockIdx.x * kCT + kCT);
    const f4 val = {v, v, v, v};
    for (int64_t t = t0; t < tend; ++t) {
        const int64_t c0 = t * kT;
        const bool full = r0 + kT <= n && c0 + kT <= n;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + j * 256;
            const int r = e >> 4, q = (e & 15) * 4;
            if (full) {
                __builtin_nontemporal_store(val, reinterpret_cast<f4 *>(D + (r0 + r) * ld + c0 + q));
                if (t != yb)
                    __builtin_nontemporal_store(val, reinterpret_cast<f4 *>(D + (c0 + r) * ld + r0 + q));
            } else {
                for (int u = 0; u < 4; ++u) {
                    if (r0 + r < n && c0 + q + u < n) D[(r0 + r) * ld + c0 + q + u] = v;
                    if (t != yb && c0 + r < n && r0 + q + u < n) D[(c0 + r) * ld + r0 + q + u] = v;
                }
            }
        }
    }
}

hipError_t launch_write_probe(float *D, int64_t n, int64_t ld, float v, hipStream_t s) {
    const int64_t nT = (n + kT - 1) / kT;
    dim3 grid((unsigned)((nT + kCT - 1) / kCT), (unsigned)nT);
    hipLaunchKernelGGL(k_write_probe, grid, dim3(256), 0, s, D, n, ld, v);
    return hipGetLastError();
}

hipError_t launch_dist_l2_f32(const float *X, int64_t n, int32_t dim, float *D, int64_t ld,
                              float *mean, hipStream_t s) {
    hipLaunchKernelGGL(k_center_mean, dim3(dim), dim3(256), 0, s, X, n, dim, mean);
    if (dim <= kSD) {
        const int64_t nT = (n + kT - 1) / kT;
        dim3 grid((unsigned)((nT + kCT - 1) / kCT), (unsigned)nT);
        if (dim <= 16)
            hipLaunchKernelGGL(k_dist_l2_f32_upper<16>, grid, dim3(256), 0, s, X,
                               (const float *)mean, n, dim, D, ld);
        else if (dim <= 32)
            hipLaunchKernelGGL(k_dist_l2_f32_upper<32>, grid, dim3(256), 0, s, X,
                               (const float *)mean, n, dim, D, ld);
        else
            hipLaunchKernelGGL(k_dist_l2_f32_upper<64>, grid, dim3(256), 0, s, X,
                               (const float *)mean, n, dim, D, ld);
    } else {
        dim3 grid((unsigned)((n + kT - 1) / kT), (unsigned)((n + kT - 1) / kT));
        hipLaunchKernelGGL(k_dist_l2_f32, grid, dim3(256), 0, s, X, (const float *)mean, n, dim, D,
                           ld);
    }
    return hipGetLastError();
}

// ---- transpose of a rows x cols matrix of 4-byte elements (DT[c][r] =
// D[r][c]) through 64 x 64 tiles in LDS (one padding column against bank
// conflicts), both sides read and written along rows.
__global__ __launch_bounds__(256) void k_transpose(const uint32_t *__restrict__ D, int64_t ld,
                                                   int64_t rows, int64_t cols,
                                                   uint32_t *__restrict__ DT, int64_t ldt) {
    __shared__ uint32_t tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = D[r * ld + c];
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows) DT[c * ldt + r] = tile[tx][i];
    }
}

// ---- validation of a dissimilarity matrix (the properties PAM's arithmetic
// relies on, Sec. 2): symmetric, zero diagonal, finite and non-negative.
// Work-group (bi, bj) with bi <= bj compares tile (bi, bj) with the transpose
// of tile (bj, bi) through LDS, so every entry is read once; an offending
// pair {i, j} (i <= j) sets bits of flags[0] (vector atomic) and adds one to
// flags[1].
template <typename T>
__device__ __forceinline__ int entry_flags(T v) {
    if constexpr (std::is_same<T, float>::value) {
        if (!(v == v) || v == __builtin_huge_valf() || v == -__builtin_huge_valf())
            return PAMX_DIS_NONFINITE;
        return v < 0.0f ? PAMX_DIS_NEGATIVE : 0;
    } else {
        return v < 0 ? PAMX_DIS_NEGATIVE : 0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_check_dis(const T *__restrict__ D, int64_t n, int64_t ld,
                                                   int32_t *__restrict__ flags) {
    __shared__ T tile[64][65];
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;   // lower tiles are compared from their upper partners
    const int64_t r0 = bi * 64, c0 = bj * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // tile (bj, bi) into LDS, transposed on the way out
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = c0 + i, c = r0 + tx;
        if (r < n && c < n) tile[i][tx] = D[r * ld + c];
    }
    __syncthreads();
    // positions r <= c only: each unordered pair {r, c} once, with both entries
    int f = 0, cnt = 0;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r >= n || c >= n || r > c) continue;
        const T v = D[r * ld + c];
        int e = entry_flags<T>(v);
        if (r == c) {
            if (v != T(0)) e |= PAMX_DIS_DIAGONAL;
        } else {
            const T w = tile[tx][i];   // D[c][r]
            if (!(v == w)) e |= PAMX_DIS_ASYMMETRIC;
            e |= entry_flags<T>(w);
        }
        f |= e;
        cnt += (e != 0);
    }
    if (f) atomicOr(&flags[0], f);
    if (cnt) atomicAdd(&flags[1], cnt);
}

hipError_t launch_check_dis(const void *D, int32_t dtype, int64_t n, int64_t ld, int32_t *flags,
                            hipStream_t s) {
    const unsigned nt = (unsigned)((n + 63) / 64);
    if (dtype == PAMX_F32)
        hipLaunchKernelGGL(k_check_dis<float>, dim3(nt, nt), dim3(256), 0, s,
                           static_cast<const float *>(D), n, ld, flags);
    else
        hipLaunchKernelGGL(k_check_dis<int32_t>, dim3(nt, nt), dim3(256), 0, s,
                           static_cast<const int32_t *>(D), n, ld, flags);
    return hipGetLastError();
}

// ---- reference read: the SWAP pass's access with none of its arithmetic.
// Work-group (tile, chunk) reads rows [chunk * L, +L) of columns
// [tile * 1024, +1024), one 16-byte non-temporal load per lane and row, four
// rows in flight (as the pass), and writes the sum of what it read.
template <bool PF>
__global__ __launch_bounds__(256) void k_read_probe(const float *__restrict__ D, int64_t ld, int64_t n,
                                                   int32_t L, float *__restrict__ sums) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int U = 4;
    const int64_t a = (int64_t)blockIdx.y * L;
    const int64_t b = min(a + (int64_t)L, n);
    const int64_t c0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    float acc = 0.f;
    if (c0 < n) {   // c0 + 3 < ld: ld is a multiple of 4
        int64_t o = a;
        auto ld4 = [&](int64_t o0, f4 (&v)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(D + (o0 + u) * ld + c0));
        };
        auto sum4 = [&](const f4 (&v)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (v[u][0] + v[u][1]) + (v[u][2] + v[u][3]);
        };
        if constexpr (PF) {   // the pass's prefetching loop: next block issued first
            if (o + U <= b) {
                f4 v[U];
                ld4(o, v);
                for (; o + 2 * U <= b; o += U) {
                    f4 w[U];
                    ld4(o + U, w);
                    sum4(v);
#pragma unroll
                    for (int u = 0; u < U; ++u) v[u] = w[u];
                }
                sum4(v);
                o += U;
            }
        } else {
            for (; o + U <= b; o += U) {
                f4 v[U];
                ld4(o, v);
                sum4(v);
            }
        }
        for (; o < b; ++o) {
            const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(D + o * ld + c0));
            acc += (v[0] + v[1]) + (v[2] + v[3]);
        }
    }
    __shared__ float wsum[4];
    for (int w = 32; w >= 1; w >>= 1) acc += __shfl_xor(acc, w);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        sums[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

hipError_t launch_read_probe(const float *D, int64_t n, int64_t ld, int32_t L, float *sums,
                             hipStream_t s) {
    const dim3 grid((unsigned)((n + 1023) / 1024), (unsigned)((n + L - 1) / L));
    if (L >= kPfChunk)
        hipLaunchKernelGGL(k_read_probe<true>, grid, dim3(256), 0, s, D, ld, n, L, sums);
    else
        hipLaunchKernelGGL(k_read_probe<false>, grid, dim3(256), 0, s, D, ld, n, L, sums);
    return hipGetLastError();
}

hipError_t launch_transpose(const void *D, int64_t ld, int64_t rows, int64_t cols, void *DT,
                            int64_t ldt, hipStream_t s) {
    const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, static_cast<const uint32_t *>(D), ld,
                       rows, cols, static_cast<uint32_t *>(DT), ldt);
    return hipGetLastError();
}

}  // namespace pamx
