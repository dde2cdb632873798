// precision.hip -- the mixed-precision form of FastPAM1 SWAP for Euclidean
// points: distances recomputed per tile from split-BF16 points on the matrix
// cores (no n x n matrix), loss changes summed in FP64 or FP32, and every
// candidate that could still be the best swap re-scored in FP64 from the
// original FP32 points, so the decisions are those of FP64 arithmetic.
// BUILD of this form (Alg. 1) runs in FP64 directly, incrementally after its
// first two steps.
//
// Paper: Schubert & Rousseeuw, arXiv 2008.05171 -- Alg. 1 (BUILD), Alg. 3
// and Eq. better-change3 (FastPAM1).  The paper fixes no precision; this form
// trades the O(n^2) matrix for recomputation and keeps exactness through a
// rigorous error bound:
//
//   d~(o,c) = sqrt(max(|x~o|^2 + |x~c|^2 - 2 x~o.x~c, 0)), x~ = bf16(x - mu)
//   |d~ - d| <= 2 e_max + g_max + 2^-22 d~            (per pair)
//     e_max = max_o |x~o - (x_o - mu)|    (BF16 rounding, exact in FP64)
//     g_max = sqrt((KP + 8) 2^-20 max_o |x~o|^2)   (FP32 norms and Gram)
//
// The loss change of an object depends on d(o,c) only while d < ds(o) (the
// second-nearest distance), so for every swap
//   |Delta~(i,c) - Delta(i,c)| <= cnt(c) * eps1 + eps_acc
// where cnt(c) counts objects with d~(o,c) below ds(o) + eps, and eps_acc
// bounds the FP32 summation.  Candidates whose lower bound reaches the best
// upper bound are re-scored exactly.
#include "pamx_internal.h"

namespace pamx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kRT = 256;       // lanes per work-group, one candidate each
constexpr int kRB = 32;        // objects per Gram block
constexpr int kGS = kRB + 1;   // padded stride (floats) of the transposed tile, per candidate
constexpr int kAS = 72;        // padded row stride (bf16) of the staged object block

// ---------------------------------------------------------------- FP64 distance
// The reference distance of this form: Euclidean, FP64, from the original
// FP32 coordinates (differences of two floats are exact in FP64).
// Coordinates are loaded in unrolled groups of 16 from clamped (always
// valid) indices, with no branch between the loads, so a group's loads are in
// flight together; coordinates past dim add an exact 0.  The FMA order is
// k = 0 .. dim-1.
__device__ __forceinline__ double d64(const float *__restrict__ X, int dim, int64_t a, int64_t b) {
    const float *x = X + a * dim;
    const float *y = X + b * dim;
    double s = 0.0;
    if ((dim & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
        // rows are 16-byte aligned: 16-byte loads, same FMA order
        const float4 *x4 = reinterpret_cast<const float4 *>(x);
        const float4 *y4 = reinterpret_cast<const float4 *>(y);
        const int d4 = dim >> 2;
#pragma unroll
        for (int k0 = 0; k0 < kRcMaxDim / 4; k0 += 4) {
            if (k0 < d4) {
                float4 xv[4], yv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kk = min(k0 + u, d4 - 1);
                    xv[u] = x4[kk];
                    yv[u] = y4[kk];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool in = k0 + u < d4;
                    const double t0 = in ? (double)xv[u].x - (double)yv[u].x : 0.0;
                    const double t1 = in ? (double)xv[u].y - (double)yv[u].y : 0.0;
                    const double t2 = in ? (double)xv[u].z - (double)yv[u].z : 0.0;
                    const double t3 = in ? (double)xv[u].w - (double)yv[u].w : 0.0;
                    s = fma(t0, t0, s);
                    s = fma(t1, t1, s);
                    s = fma(t2, t2, s);
                    s = fma(t3, t3, s);
                }
            }
        }
        return sqrt(s);
    }
#pragma unroll
    for (int k0 = 0; k0 < kRcMaxDim; k0 += 16) {
        if (k0 < dim) {
            float xv[16], yv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int kk = min(k0 + u, dim - 1);
                xv[u] = x[kk];
                yv[u] = y[kk];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const double t = (k0 + u < dim) ? (double)xv[u] - (double)yv[u] : 0.0;
                s = fma(t, t, s);
            }
        }
    }
    return sqrt(s);
}

// ---------------------------------------------------------------- prep
// Split BF16 representation of the centred points: hi = bf16(x - mu),
// lo = bf16((x - mu) - hi); the effective point x~ = hi + lo is exact in
// FP32.  Rows hold hi[KP] then lo[KP].  Also the FP32 squared norm of x~ and
// the FP64 residual |x~ - (x - mu)|.
__global__ __launch_bounds__(256) void k_rc_prep(const float *__restrict__ X, int64_t n, int32_t dim,
                                                 int32_t KP, const float *__restrict__ mean,
                                                 __bf16 *__restrict__ Xs, float *__restrict__ nb,
                                                 double *__restrict__ eo) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    float nrm = 0.0f;
    double res = 0.0;
    __bf16 *row = Xs + o * 2 * KP;
    for (int k = 0; k < KP; ++k) {
        float v = 0.0f;
        double exact = 0.0;
        if (k < dim) {
            const float x = X[o * dim + k];
            v = x - mean[k];
            exact = (double)x - (double)mean[k];
        }
        const __bf16 hi = (__bf16)v;
        const __bf16 lo = (__bf16)(v - (float)hi);
        row[k] = hi;
        row[KP + k] = lo;
        const float eff = (float)hi + (float)lo;
        nrm = fmaf(eff, eff, nrm);
        const double r = (double)eff - exact;
        res = fma(r, r, res);
    }
    nb[o] = nrm;
    eo[o] = sqrt(res);
}

// max of eo and of nb (single work-group): mx[0] = e_max, mx[1] = max |x~|^2
__global__ __launch_bounds__(1024) void k_rc_prep_max(const double *__restrict__ eo,
                                                      const float *__restrict__ nb, int64_t n,
                                                      double *__restrict__ out) {
    __shared__ double s1[1024], s2[1024];
    double a = 0.0, b = 0.0;
    for (int64_t o = threadIdx.x; o < n; o += 1024) {
        a = fmax(a, eo[o]);
        b = fmax(b, (double)nb[o]);
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = s1[0]; out[1] = s2[0]; }
}

// Per-pair distance bounds (eps0):
//   sigma bounds |s~ - s| for s = |x~o - x~c|^2: FP32 norms (KP terms), the
//   3 KP split-product Gram terms summed in FP32 by the matrix cores, the
//   dropped lo*lo' term, the final fma -- all relative to |x~o|^2 + |x~c|^2,
//   with a factor 2 of slack.  Then |d~ - |x~o - x~c|| <= min(sqrt(sigma),
//   sigma / d~), and |x~o - x~c| is within 2 e_max of the true distance.
//   eps0[0] = e_near = 2 e_max + sqrt(sigma)            (d~ <  delta0)
//   eps0[1] = e_far  = 2 e_max + sigma / delta0         (d~ >= delta0)
//   eps0[2] = delta0 = 8 sqrt(sigma);  eps0[3] = a bound on any d~
__global__ void k_rc_eps(const double *__restrict__ mx, int32_t KP, double *__restrict__ eps0) {
    if (threadIdx.x != 0) return;
    const double emax = mx[0], nbmax = mx[1];
    const double rel = 3.0 * KP * 0x1p-25 * 1.01 + KP * 0x1p-24 + 0x1p-19 + 0x1p-22;
    const double sigma = 2.0 * (2.0 * nbmax) * rel;
    const double d0 = 8.0 * sqrt(sigma);
    eps0[0] = 2.0 * emax + sqrt(sigma);
    eps0[1] = 2.0 * emax + sigma / d0;
    eps0[2] = d0;
    eps0[3] = 2.0 * sqrt(nbmax) * (1.0 + 0x1p-20) + sqrt(sigma);
}

// ---------------------------------------------------------------- Gram tile
// One work-group, one block of 32 (sorted) objects: stage their split BF16
// rows and their four per-row values in LDS; every wave computes the 32 x 64
// Gram tile of the block against its 64 candidates on the matrix cores
// (hi.hi' + hi.lo' + lo.hi' per 16-wide k step, v_mfma_f32_32x32x16_bf16)
// and writes it transposed -- g[candidate][object] -- to its own LDS region.
// Operand layout (wave64, 32x32x16): lane l supplies A[l%32][8(l/32)..+7]
// and B[8(l/32)..+7][l%32] of each k step; accumulator element v of lane l
// is C[(v%4) + 8(v/4) + 4(l/32)][l%32].
// The staged rows As are read only before the second barrier, so the next
// block may overwrite them; the row values Rv are read after it, while a
// faster wave may already stage the next block, so callers alternate two Rv
// buffers by block parity (no wave can be two blocks ahead of another).
struct RowVals {
    const float *v0, *v1, *v2, *v3;   // per (sorted) position; v3 may be null
};

// Registers holding one block's staged data in flight (software pipeline:
// the next block's global loads overlap the current block's MFMA and row loop).
template <int KS>
struct Stage {
    static constexpr int kPieces = KS * 4;                            // 16-byte pieces per split row
    static constexpr int kPer = (kRB * kPieces + kRT - 1) / kRT;      // pieces per lane
    bf16x8 v[kPer];
    float4 rv;
};

template <int KS>
__device__ __forceinline__ void stage_load(Stage<KS> &st, const __bf16 *__restrict__ Xs, int KP,
                                           const int32_t *__restrict__ rows, int64_t j0, int64_t jend,
                                           const RowVals &rvals) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < Stage<KS>::kPer; ++u) {
        const int e = tid + u * kRT;
        const int r = e / Stage<KS>::kPieces, p = e - r * Stage<KS>::kPieces;
        const int64_t j = j0 + r;
        if (e < kRB * Stage<KS>::kPieces && j < jend) {
            const int64_t o = rows ? rows[j] : j;
            st.v[u] = *reinterpret_cast<const bf16x8 *>(Xs + o * 2 * KP + p * 8);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) st.v[u][q] = (__bf16)0.0f;
        }
    }
    st.rv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tid < kRB) {
        const int64_t j = j0 + tid;
        if (j < jend)
            st.rv = make_float4(rvals.v0[j], rvals.v1[j], rvals.v2[j], rvals.v3 ? rvals.v3[j] : 0.f);
    }
}

template <int KS>
__device__ __forceinline__ void stage_store(const Stage<KS> &st, int KP, __bf16 *__restrict__ As,
                                            float4 *__restrict__ Rv) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < Stage<KS>::kPer; ++u) {
        const int e = tid + u * kRT;
        if (e < kRB * Stage<KS>::kPieces) {
            const int r = e / Stage<KS>::kPieces, p = e - r * Stage<KS>::kPieces;
            const int half = (p * 8) / KP, off = (p * 8) % KP;   // hi to [0, KP), lo to [kAS, kAS + KP)
            *reinterpret_cast<bf16x8 *>(As + r * 2 * kAS + half * kAS + off) = st.v[u];
        }
    }
    if (tid < kRB) Rv[tid] = st.rv;
}

// The Gram tile of the staged block (after the barrier that publishes it):
// hi.hi' + hi.lo' + lo.hi' per k step, then the transposed store.
template <int KS>
__device__ __forceinline__ void gram_tile(const __bf16 *__restrict__ As, float *__restrict__ Gw,
                                          const bf16x8 (&bh)[2][KS], const bf16x8 (&bl)[2][KS]) {
    const int lane = threadIdx.x & 63;
    floatx16 acc0, acc1;
#pragma unroll
    for (int v = 0; v < 16; ++v) { acc0[v] = 0.0f; acc1[v] = 0.0f; }
    const int i = lane & 31, h = lane >> 5;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(As + i * 2 * kAS + s * 16 + h * 8);
        const bf16x8 al = *reinterpret_cast<const bf16x8 *>(As + i * 2 * kAS + kAS + s * 16 + h * 8);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[0][s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[1][s], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[0][s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[1][s], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[0][s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[1][s], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = (v & 3) + 8 * (v >> 2) + 4 * h;
        Gw[i * kGS + r] = acc0[v];
        Gw[(32 + i) * kGS + r] = acc1[v];
    }
}

// B operands (hi and lo) of a wave's two column blocks for its 64 candidates
template <int KS>
__device__ __forceinline__ void load_bq(const __bf16 *__restrict__ Xs, int KP, int64_t n,
                                        int64_t cbase, bf16x8 (&bh)[2][KS], bf16x8 (&bl)[2][KS]) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 31, h = lane >> 5;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int64_t c = cbase + cb * 32 + i;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (c < n) {
                bh[cb][s] = *reinterpret_cast<const bf16x8 *>(Xs + c * 2 * KP + s * 16 + h * 8);
                bl[cb][s] = *reinterpret_cast<const bf16x8 *>(Xs + c * 2 * KP + KP + s * 16 + h * 8);
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) { bh[cb][s][u] = (__bf16)0.0f; bl[cb][s][u] = (__bf16)0.0f; }
            }
        }
    }
}

// The hardware square root (v_sqrt_f32): within 1 ulp of the exact root for
// normal arguments and 0 for subnormal ones -- one instruction instead of the
// correctly rounded sequence; the per-pair bound covers both (k_rc_iter_bounds).
__device__ __forceinline__ float rc_dist(float g, float no, float nc) {
    return __builtin_amdgcn_sqrtf(fmaxf(fmaf(-2.0f, g, no + nc), 0.0f));
}

// ---------------------------------------------------------------- SWAP pass
// The FastPAM1 pass (Eq. better-change3) over a chunk of segment-sorted
// objects: B(c) += min(d~ - dn, 0); S_i(c) += med3(d~, dn, ds) - ds; at the
// end of a segment complete in the chunk, v = R_i + S_i and the running best
// (v, i); head and tail carries as in the stored-matrix pass.  Outputs per
// candidate and chunk: part[q][0..3] = B, head, tail, best value (ACC);
// part_i[q][0..3] = best slot, far count, near count.  Register use is held
// to three waves per SIMD (the LDS of three work-groups per CU).
template <int KS, typename ACC>
__global__ __launch_bounds__(kRT) __attribute__((amdgpu_waves_per_eu(3))) void k_rc_swap_pass(
    const __bf16 *__restrict__ Xs, int32_t KP, const float *__restrict__ nb, int64_t n, int32_t k,
    const int32_t *__restrict__ srow, const float *__restrict__ sdn, const float *__restrict__ sds,
    const float *__restrict__ sthr, const float *__restrict__ snb, const double *__restrict__ eps0,
    const int32_t *__restrict__ seg_off, const double *__restrict__ R64, const int32_t *__restrict__ cinfo4,
    int32_t L, int64_t ncp, ACC *__restrict__ part, int32_t *__restrict__ part_i,
    const DevState *__restrict__ st) {
    if (st->done) return;
    __shared__ __align__(16) __bf16 As[kRB * 2 * kAS];
    __shared__ float4 Rv[2][kRB];   // by block parity: a wave is at most one block ahead
    __shared__ float G[4][64 * kGS];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int q = blockIdx.y;
    const int64_t a = (int64_t)q * L, b = min(a + (int64_t)L, n);
    const int64_t cbase = (int64_t)blockIdx.x * kRT + w * 64;
    const int64_t c = cbase + lane;
    const int sa = cinfo4[4 * q], sb = cinfo4[4 * q + 1], flags = cinfo4[4 * q + 2];
    bf16x8 bh[2][KS], bl[2][KS];
    load_bq<KS>(Xs, KP, n, cbase, bh, bl);
    const float nc = (c < n) ? nb[c] : 0.0f;
    const float d0 = (float)eps0[2];
    ACC accB = 0, S = 0, bv = (ACC)__builtin_huge_val();
    int bi = INT_MAX, cf = 0, cn = 0;
    ACC *pq = part + (int64_t)q * 4 * ncp + c;
    int cs = sa;
    int64_t ce = seg_off[sa + 1];
    auto finish = [&](int s) {
        if (s == sa && (flags & 1)) pq[1 * ncp] = S;
        else if (s == sb && (flags & 2)) pq[2 * ncp] = S;
        else {
            const ACC v = (ACC)R64[s] + S;
            if (v < bv) { bv = v; bi = s; }
        }
        S = 0;
    };
    float *Gw = G[w];
    const RowVals rv{snb, sdn, sds, sthr};
    Stage<KS> stg;
    stage_load<KS>(stg, Xs, KP, srow, a, b, rv);
    for (int64_t j0 = a; j0 < b; j0 += kRB) {
        float4 *Rb = Rv[((j0 - a) / kRB) & 1];
        stage_store<KS>(stg, KP, As, Rb);
        __syncthreads();
        if (j0 + kRB < b) stage_load<KS>(stg, Xs, KP, srow, j0 + kRB, b, rv);
        gram_tile<KS>(As, Gw, bh, bl);
        __syncthreads();
        const int m = (int)min((int64_t)kRB, b - j0);
        ACC bblk = 0, sblk = 0;
        const float *Gl = Gw + lane * kGS;
        // one pair: loss-change terms and the bound's counts
        auto pair = [&](float g, float4 q4) {   // q4 = no, dn, ds, thr
            const float d = rc_dist(g, q4.x, nc);
            bblk += (ACC)fminf(d - q4.y, 0.0f);
            sblk += (ACC)(__builtin_amdgcn_fmed3f(d, q4.y, q4.z) - q4.z);
            const bool cnt = d < q4.w;
            cf += (cnt && d >= d0) ? 1 : 0;
            cn += (cnt && d < d0) ? 1 : 0;
        };
        int r = 0;
        while (r < m) {
            if (j0 + r == ce) {        // uniform: segment boundary
                S += sblk;
                sblk = 0;
                finish(cs);
                do { ++cs; } while (seg_off[cs + 1] == seg_off[cs]);
                ce = seg_off[cs + 1];
            }
            // the objects up to the next boundary, eight (then four) at a time
            // with their LDS reads issued together, so LDS latency overlaps
            // arithmetic (same order of additions as one at a time)
            const int re = (int)min((int64_t)m, ce - j0);
            for (; r + 8 <= re; r += 8) {
                float4 q[8];
                float g[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) { q[u] = Rb[r + u]; g[u] = Gl[r + u]; }
#pragma unroll
                for (int u = 0; u < 8; ++u) pair(g[u], q[u]);
            }
            for (; r + 4 <= re; r += 4) {
                float4 q[4];
                float g[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) { q[u] = Rb[r + u]; g[u] = Gl[r + u]; }
#pragma unroll
                for (int u = 0; u < 4; ++u) pair(g[u], q[u]);
            }
            for (; r < re; ++r) pair(Gl[r], Rb[r]);
        }
        accB += bblk;
        S += sblk;
    }
    finish(cs);
    pq[0] = accB;
    pq[3 * ncp] = bv;
    int32_t *pi = part_i + (int64_t)q * 4 * ncp + c;
    pi[0] = bi;
    pi[ncp] = cf;
    pi[2 * ncp] = cn;
}

// ---------------------------------------------------------------- merge
// SWAP: chunk carries and bests -> per candidate Delta~_c and its bound.
// bnd[0] = e_far, bnd[1] = e_near, bnd[2] = absolute summation bound.
template <typename ACC>
__global__ __launch_bounds__(256) void k_rc_swap_merge(
    const ACC *__restrict__ part, const int32_t *__restrict__ part_i,
    const int32_t *__restrict__ cinfo4, int32_t Q, int64_t n, int32_t k, int64_t ncp,
    const double *__restrict__ R64, const uint8_t *__restrict__ is_med,
    const DevState *__restrict__ st, const double *__restrict__ bnd, double *__restrict__ cand_v,
    double *__restrict__ cand_b, double *__restrict__ wg_u) {
    __shared__ double red[256];
    if (st->done) return;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double up = __builtin_huge_val();
    if (c < n) {
        ACC accB = 0, bestv = (ACC)__builtin_huge_val(), run_m = 0;
        int besti = INT_MAX, run_s = -1;
        int64_t cf = 0, cn = 0;
        auto flush = [&]() {
            if (run_s >= 0) {
                const ACC v = (ACC)R64[run_s] + run_m;
                if (lt2(v, run_s, bestv, besti)) { bestv = v; besti = run_s; }
            }
        };
        for (int q = 0; q < Q; ++q) {
            const ACC *pq = part + (int64_t)q * 4 * ncp + c;
            const int32_t *pi = part_i + (int64_t)q * 4 * ncp + c;
            accB += pq[0];
            cf += pi[ncp];
            cn += pi[2 * ncp];
            const int32_t i = pi[0];
            if (i != INT_MAX && lt2(pq[3 * ncp], i, bestv, besti)) { bestv = pq[3 * ncp]; besti = i; }
            const int sa = cinfo4[4 * q], sb = cinfo4[4 * q + 1], fl = cinfo4[4 * q + 2];
            if (fl & 1) {
                if (sa == run_s) run_m += pq[1 * ncp];
                else { flush(); run_s = sa; run_m = pq[1 * ncp]; }
            }
            if (fl & 2) {
                if (sb == run_s) run_m += pq[2 * ncp];
                else { flush(); run_s = sb; run_m = pq[2 * ncp]; }
            }
        }
        flush();
        const int e = st->empty_slot;
        if (e < k && lt2((ACC)0, e, bestv, besti)) { bestv = 0; besti = e; }
        const double dl = (double)bestv + (double)accB;
        const double b = ((double)cf * bnd[0] + (double)cn * bnd[1] + bnd[2]) * 1.0001 + 1e-300;
        if (!is_med[c]) {
            cand_v[c] = dl;
            cand_b[c] = b;
            up = dl + b;
        } else {
            cand_v[c] = __builtin_huge_val();
            cand_b[c] = 0.0;
        }
    }
    red[threadIdx.x] = up;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) wg_u[blockIdx.x] = red[0];
}

// Global minimum upper bound U*, then the list of candidates whose lower
// bound reaches it (and, for SWAP, lies below the application threshold).
__global__ __launch_bounds__(1024) void k_rc_upper(const double *__restrict__ wg_u, int32_t nwg,
                                                   DevState *__restrict__ st) {
    __shared__ double red[1024];
    if (st->done) return;
    double u = __builtin_huge_val();
    for (int i = threadIdx.x; i < nwg; i += 1024) u = fmin(u, wg_u[i]);
    red[threadIdx.x] = u;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) { st->f32_best = red[0]; st->n_list = 0; }
}

__global__ __launch_bounds__(256) void k_rc_mark(const double *__restrict__ cand_v,
                                                 const double *__restrict__ cand_b, int64_t n,
                                                 int32_t swap_mode, int32_t *__restrict__ list,
                                                 DevState *__restrict__ st) {
    if (st->done) return;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const double v = cand_v[c];
    if (v == __builtin_huge_val()) return;
    const double lo = v - cand_b[c];
    bool take = lo <= st->f32_best;
    if (swap_mode) take = take && (lo < -st->margin);
    if (take) list[atomicAdd(&st->n_list, 1)] = (int32_t)c;
}

// ---------------------------------------------------------------- FP64 re-score
// One work-group per listed candidate, fixed summation order.
// SWAP: exact Delta(i,c) = R_i + B(c) + S_i(c) for every slot i.  Thread t
// walks a contiguous range of the sorted objects; segments complete in its
// range go to LDS directly, the partial first/last ones are combined
// afterwards in thread order.
constexpr int kRsT = 256;    // threads per (candidate, object group)
// A listed candidate's sorted objects are split into G contiguous groups,
// one work-group each, so that a short list still fills the chip; each group
// writes its per-slot partial sums and its part of B, and a second kernel
// adds the groups in order.  At most kRsParts (candidate, group) partials are
// held at once: G = min(kRsGmax, kRsParts / m), and G = 1 (no partials, the
// work-group finishes the candidate) for lists longer than kRsParts.
constexpr int kRsParts = 4096;
constexpr int kRsGmax = 16;

__device__ __forceinline__ int rs_groups(int m) {
    const int g = kRsParts / (m > 0 ? m : 1);
    return g < 1 ? 1 : (g > kRsGmax ? kRsGmax : g);
}

template <int KS>
__global__ __launch_bounds__(kRsT) void k_rc_swap_rescore(
    const float *__restrict__ X, int32_t dim, int64_t n, int32_t k, const int32_t *__restrict__ srow,
    const double *__restrict__ dn64, const double *__restrict__ ds64,
    const int32_t *__restrict__ near, const double *__restrict__ R64,
    const int32_t *__restrict__ list, const DevState *__restrict__ st,
    double *__restrict__ res_v, int32_t *__restrict__ res_i, double *__restrict__ rs_part) {
    extern __shared__ __align__(16) unsigned char rs_raw[];
    double *sarr = reinterpret_cast<double *>(rs_raw);          // k per-slot sums
    __shared__ double hv[kRsT], tv[kRsT], red[kRsT];
    __shared__ int hs[kRsT], ts[kRsT], ri[kRsT];
    const int t = threadIdx.x;
    const int m = st->n_list;
    const int G = rs_groups(m);
    for (int b = blockIdx.x; b < m * G; b += gridDim.x) {
        const int idx = b / G, g = b - idx * G;
        const int64_t c = list[idx];
        for (int i = t; i < k; i += kRsT) sarr[i] = 0.0;
        __syncthreads();
        // this group's sorted positions, then this thread's part of them
        const int64_t g0 = n * g / G, g1 = n * (g + 1) / G;
        const int64_t per = (g1 - g0 + kRsT - 1) / kRsT;
        const int64_t j0 = min(g1, g0 + (int64_t)t * per), j1 = min(g1, j0 + per);
        double B = 0.0, S = 0.0, first = 0.0;
        int cur = -1, fs = -1;
        for (int64_t j = j0; j < j1; ++j) {
            const int64_t o = srow[j];
            const int sl = near[o];
            if (sl != cur) {
                if (cur >= 0) {
                    if (fs < 0) { fs = cur; first = S; }   // first segment of the range
                    else sarr[cur] = S;                    // complete inside the range
                }
                cur = sl;
                S = 0.0;
            }
            const double d = d64(X, dim, o, c), lo = dn64[o], hi = ds64[o];
            B += fmin(d - lo, 0.0);
            S += fmin(fmax(d, lo), hi) - hi;
        }
        // head = first segment of the range, tail = last (may coincide)
        if (cur >= 0 && fs < 0) { fs = cur; first = S; cur = -1; }
        hs[t] = fs; hv[t] = first;
        ts[t] = cur; tv[t] = S;
        red[t] = B;
        __syncthreads();
        if (t == 0) {
            int rs = -1;
            double rm = 0.0;
            for (int u = 0; u < kRsT; ++u) {
                if (hs[u] >= 0) {
                    if (hs[u] == rs) rm += hv[u];
                    else { if (rs >= 0) sarr[rs] += rm; rs = hs[u]; rm = hv[u]; }
                }
                if (ts[u] >= 0) {
                    if (ts[u] == rs) rm += tv[u];
                    else { if (rs >= 0) sarr[rs] += rm; rs = ts[u]; rm = tv[u]; }
                }
            }
            if (rs >= 0) sarr[rs] += rm;
        }
        for (int w = kRsT / 2; w > 0; w >>= 1) {
            __syncthreads();
            if (t < w) red[t] += red[t + w];
        }
        __syncthreads();
        if (G > 1) {   // partial sums of this group; k_rc_rescore_combine finishes
            double *pp = rs_part + (int64_t)b * (k + 1);
            for (int i = t; i < k; i += kRsT) pp[i] = sarr[i];
            if (t == 0) pp[k] = red[0];
            __syncthreads();
            continue;
        }
        // best slot: smallest R_i + S_i, smallest i on ties
        double bv = __builtin_huge_val();
        int bi = INT_MAX;
        for (int i = t; i < k; i += kRsT) {
            const double v = R64[i] + sarr[i];
            if (v < bv) { bv = v; bi = i; }
        }
        hv[t] = bv; ri[t] = bi;
        __syncthreads();
        for (int w = kRsT / 2; w > 0; w >>= 1) {
            if (t < w && lt2(hv[t + w], ri[t + w], hv[t], ri[t])) { hv[t] = hv[t + w]; ri[t] = ri[t + w]; }
            __syncthreads();
        }
        if (t == 0) { res_v[idx] = hv[0] + red[0]; res_i[idx] = ri[0]; }
        __syncthreads();
    }
}

// Sum of a candidate's group partials in group order, then its best slot.
__global__ __launch_bounds__(kRsT) void k_rc_rescore_combine(
    const double *__restrict__ rs_part, int32_t k, const double *__restrict__ R64,
    const DevState *__restrict__ st, double *__restrict__ res_v, int32_t *__restrict__ res_i) {
    __shared__ double hv[kRsT];
    __shared__ int ri[kRsT];
    const int t = threadIdx.x;
    const int m = st->n_list;
    const int G = rs_groups(m);
    if (G == 1) return;
    for (int idx = blockIdx.x; idx < m; idx += gridDim.x) {
        const double *pp = rs_part + (int64_t)idx * G * (k + 1);
        double bv = __builtin_huge_val();
        int bi = INT_MAX;
        for (int i = t; i < k; i += kRsT) {
            double S = 0.0;
            for (int g = 0; g < G; ++g) S += pp[(int64_t)g * (k + 1) + i];
            const double v = R64[i] + S;
            if (v < bv) { bv = v; bi = i; }
        }
        hv[t] = bv; ri[t] = bi;
        __syncthreads();
        for (int w = kRsT / 2; w > 0; w >>= 1) {
            if (t < w && lt2(hv[t + w], ri[t + w], hv[t], ri[t])) { hv[t] = hv[t + w]; ri[t] = ri[t + w]; }
            __syncthreads();
        }
        if (t == 0) {
            double B = 0.0;
            for (int g = 0; g < G; ++g) B += pp[(int64_t)g * (k + 1) + k];
            res_v[idx] = hv[0] + B;
            res_i[idx] = ri[0];
        }
        __syncthreads();
    }
}

template <int KS>
static hipError_t rc_rescore_launch(const float *X, int32_t dim, int64_t n, int32_t k,
                                    const int32_t *srow, const double *dn64, const double *ds64,
                                    const int32_t *near, const double *R64, const int32_t *list,
                                    const DevState *st, double *res_v, int32_t *res_i,
                                    double *rs_part, hipStream_t s) {
    const size_t lds = (size_t)k * 8;   // the per-slot sums, beside 9 KB of fixed LDS
    if (lds > 49152) {
        const hipError_t e = hipFuncSetAttribute((const void *)k_rc_swap_rescore<KS>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_rc_swap_rescore<KS>), dim3(1024), dim3(kRsT), lds, s, X, dim, n, k,
                       srow, dn64, ds64, near, R64, list, st, res_v, res_i, rs_part);
    hipLaunchKernelGGL(k_rc_rescore_combine, dim3(1024), dim3(kRsT), 0, s, (const double *)rs_part,
                       k, R64, st, res_v, res_i);
    return hipGetLastError();
}

static hipError_t rc_rescore(int KP, const float *X, int32_t dim, int64_t n, int32_t k,
                             const int32_t *srow, const double *dn64, const double *ds64,
                             const int32_t *near, const double *R64, const int32_t *list,
                             const DevState *st, double *res_v, int32_t *res_i, double *rs_part,
                             hipStream_t s) {
    switch (KP / 16) {
        case 1: return rc_rescore_launch<1>(X, dim, n, k, srow, dn64, ds64, near, R64, list, st, res_v, res_i, rs_part, s);
        case 2: return rc_rescore_launch<2>(X, dim, n, k, srow, dn64, ds64, near, R64, list, st, res_v, res_i, rs_part, s);
        case 3: return rc_rescore_launch<3>(X, dim, n, k, srow, dn64, ds64, near, R64, list, st, res_v, res_i, rs_part, s);
        default: return rc_rescore_launch<4>(X, dim, n, k, srow, dn64, ds64, near, R64, list, st, res_v, res_i, rs_part, s);
    }
}

// Lexicographic minimum over the re-scored list; the swap is applied if its
// exact change is below -margin.
__global__ __launch_bounds__(1024) void k_rc_pick(const double *__restrict__ res_v,
                                                  const int32_t *__restrict__ res_i,
                                                  const int32_t *__restrict__ list,
                                                  int32_t *__restrict__ med,
                                                  uint8_t *__restrict__ is_med, DevState *__restrict__ st,
                                                  pamx_swap_record *__restrict__ trace) {
    if (st->done) return;
    const int m = st->n_list;
    double v = __builtin_huge_val();
    int i = INT_MAX, c = INT_MAX;
    for (int idx = threadIdx.x; idx < m; idx += 1024) {
        const double vv = res_v[idx];
        const int ii = res_i[idx], cc = list[idx];
        if (lex_less(vv, ii, cc, v, i, c)) { v = vv; i = ii; c = cc; }
    }
    block_argmin3<double, 1024>(v, i, c);
    if (threadIdx.x != 0) return;
    st->rescored += m;
    st->iter += 1;
    st->best_i = i;
    st->best_c = c;
    st->best_v = v;
    if (!(c != INT_MAX && v < -st->margin)) {
        st->done = 1;
        st->swapped = 0;
        return;
    }
    const int old = med[i];
    is_med[old] = 0;
    is_med[c] = 1;
    med[i] = c;
    st->old_med = old;
    st->new_slot = i;
    st->new_med = c;
    st->swapped = 1;
    st->td += v;
    if (trace && st->swaps < st->trace_cap) trace[st->swaps] = pamx_swap_record{i, c, v};
    st->swaps += 1;
}

// ---------------------------------------------------------------- caches (FP64)
// nearest / second over the k medoids with FP64 distances; FP32 copies
__device__ __forceinline__ void rc_scan(const float *__restrict__ X, int dim, int k,
                                        const int32_t *__restrict__ med, int64_t o, int lane,
                                        bool wave, int &nr, int &sc, double &dn, double &ds) {
    double d1 = __builtin_huge_val(), d2 = __builtin_huge_val();
    int j1 = INT_MAX, j2 = INT_MAX;
    const int j0 = wave ? lane : 0, js = wave ? 64 : 1;
    for (int j = j0; j < k; j += js) {
        const double d = d64(X, dim, o, med[j]);
        if (lt2(d, j, d1, j1)) { d2 = d1; j2 = j1; d1 = d; j1 = j; }
        else if (lt2(d, j, d2, j2)) { d2 = d; j2 = j; }
    }
    if (wave) {
        for (int w = 32; w >= 1; w >>= 1) {
            const double e1 = __shfl_xor(d1, w), e2 = __shfl_xor(d2, w);
            const int f1 = __shfl_xor(j1, w), f2 = __shfl_xor(j2, w);
            if (lt2(e1, f1, d1, j1)) {
                if (lt2(e2, f2, d1, j1)) { d2 = e2; j2 = f2; } else { d2 = d1; j2 = j1; }
                d1 = e1; j1 = f1;
            } else if (lt2(e1, f1, d2, j2)) { d2 = e1; j2 = f1; }
        }
    }
    nr = (j1 == INT_MAX) ? 0 : j1;   // NaN distances only: keep the slot in range
    sc = (j2 == INT_MAX) ? -1 : j2; dn = d1; ds = d2;
}

__global__ __launch_bounds__(256) void k_rc_cache_init(const float *__restrict__ X, int32_t dim,
                                                       int64_t n, int32_t k,
                                                       const int32_t *__restrict__ med,
                                                       int32_t *__restrict__ near, int32_t *__restrict__ sec,
                                                       double *__restrict__ dn64, double *__restrict__ ds64,
                                                       float *__restrict__ dn32, float *__restrict__ ds32,
                                                       int32_t *__restrict__ labels) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    int nr, sc;
    double a, b;
    rc_scan(X, dim, k, med, o, 0, false, nr, sc, a, b);
    near[o] = nr; sec[o] = sc; dn64[o] = a; ds64[o] = b;
    dn32[o] = (float)a; ds32[o] = (float)b;
    if (labels) labels[o] = nr;
}

__global__ __launch_bounds__(256) void k_rc_cache_update(const float *__restrict__ X, int32_t dim,
                                                         int64_t n, int32_t *__restrict__ near,
                                                         int32_t *__restrict__ sec,
                                                         double *__restrict__ dn64, double *__restrict__ ds64,
                                                         float *__restrict__ dn32, float *__restrict__ ds32,
                                                         int32_t *__restrict__ rlist,
                                                         DevState *__restrict__ st) {
    if (st->done || !st->swapped) return;
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    const int slot = st->new_slot;
    int nr = near[o], sc = sec[o];
    if (nr == slot || sc == slot) {
        rlist[atomicAdd(&st->n_list, 1)] = (int32_t)o;
        return;
    }
    const double dnew = d64(X, dim, o, st->new_med);
    double a = dn64[o], b = ds64[o];
    if (lt2(dnew, slot, a, nr)) { sc = nr; b = a; nr = slot; a = dnew; }
    else if (lt2(dnew, slot, b, sc)) { sc = slot; b = dnew; }
    near[o] = nr; sec[o] = sc; dn64[o] = a; ds64[o] = b;
    dn32[o] = (float)a; ds32[o] = (float)b;
}

__global__ __launch_bounds__(256) void k_rc_cache_rescan(const float *__restrict__ X, int32_t dim,
                                                         int32_t k, const int32_t *__restrict__ med,
                                                         int32_t *__restrict__ near, int32_t *__restrict__ sec,
                                                         double *__restrict__ dn64, double *__restrict__ ds64,
                                                         float *__restrict__ dn32, float *__restrict__ ds32,
                                                         const int32_t *__restrict__ rlist,
                                                         const DevState *__restrict__ st) {
    if (st->done || !st->swapped) return;
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * 4;
    const int m = st->n_list;
    for (int idx = blockIdx.x * 4 + (threadIdx.x >> 6); idx < m; idx += nw) {
        const int64_t o = rlist[idx];
        int nr, sc;
        double a, b;
        rc_scan(X, dim, k, med, o, lane, true, nr, sc, a, b);
        if (lane == 0) {
            near[o] = nr; sec[o] = sc; dn64[o] = a; ds64[o] = b;
            dn32[o] = (float)a; ds32[o] = (float)b;
        }
    }
}

// Per segment: R_i = sum (ds64 - dn64) in sorted order (one wave per slot);
// FP32 copy.  Sorted FP32 thresholds and norms for the pass.
__global__ __launch_bounds__(256) void k_rc_seg_const(const int32_t *__restrict__ srow,
                                                      const int32_t *__restrict__ seg_off, int32_t k,
                                                      const double *__restrict__ dn64,
                                                      const double *__restrict__ ds64,
                                                      double *__restrict__ R64,
                                                      const DevState *__restrict__ st) {
    if (st->done) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= k) return;
    double s = 0.0;
    for (int64_t j = seg_off[i] + lane; j < seg_off[i + 1]; j += 64) {
        const int64_t o = srow[j];
        s += ds64[o] - dn64[o];
    }
    for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w);
    if (lane == 0) R64[i] = s;
}

__global__ __launch_bounds__(256) void k_rc_sorted_aux(const int32_t *__restrict__ srow, int64_t n,
                                                       const float *__restrict__ sds,
                                                       const float *__restrict__ nb,
                                                       const double *__restrict__ eps0,
                                                       float *__restrict__ sthr, float *__restrict__ snb,
                                                       const DevState *__restrict__ st) {
    if (st->done) return;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    // the change of an object depends on d only below ds: count d~ < ds + e_near
    sthr[j] = (float)(((double)sds[j] + eps0[0]) * (1.0 + 0x1p-20) + 1e-30);
    snb[j] = nb[srow[j]];
}

// TD, sum of ds, max ds, max R -> bounds of this iteration (SWAP):
// bnd[0] = e_far, bnd[1] = e_near (per counted object, incl. the FP32
// rounding of the object's terms), bnd[2] = summation bound (absolute).
__global__ __launch_bounds__(1024) void k_rc_iter_bounds(const double *__restrict__ dn64,
                                                         const double *__restrict__ ds64, int64_t n,
                                                         const double *__restrict__ R64, int32_t k,
                                                         int32_t L, int32_t Q, int32_t acc64,
                                                         const double *__restrict__ eps0,
                                                         double *__restrict__ bnd, DevState *__restrict__ st) {
    __shared__ double r1[1024], r2[1024], r3[1024];
    if (st->done) return;
    const int t = threadIdx.x;
    double td = 0.0, sds = 0.0, mx = 0.0;
    for (int64_t o = t; o < n; o += 1024) { td += dn64[o]; sds += ds64[o]; mx = fmax(mx, ds64[o]); }
    r1[t] = td; r2[t] = sds; r3[t] = mx;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) { r1[t] += r1[t + w]; r2[t] += r2[t + w]; r3[t] = fmax(r3[t], r3[t + w]); }
        __syncthreads();
    }
    const double tdv = r1[0], sdsv = r2[0], dsmax = r3[0];
    __syncthreads();
    double rmax = 0.0;
    for (int i = t; i < k; i += 1024) rmax = fmax(rmax, R64[i]);
    r1[t] = rmax;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) r1[t] = fmax(r1[t], r1[t + w]);
        __syncthreads();
    }
    if (t == 0) {
        const double rm = r1[0];
        const double thr = (dsmax + eps0[0]) * (1.0 + 0x1p-20);
        // FP32 terms and the hardware square root: 2 ulp of the root, plus
        // 2^-62 for a subnormal argument, whose root is returned as 0
        const double small = 0x1p-22 * thr + 3.0 * 0x1p-24 * thr + 0x1p-62;
        bnd[0] = eps0[1] + small;
        bnd[1] = eps0[0] + small;
        const double chain = acc64 ? ((double)L + Q + 64.0) * 0x1p-52
                                   : (32.0 + (L + 31) / 32 + Q + 10.0) * 0x1p-24 * 1.02;
        bnd[2] = chain * (tdv + rm) + (acc64 ? 0.0 : 0x1p-23 * rm);
        st->td = tdv;
        st->margin = 4.0 * ((double)n + 256.0 + k + 68.0) * 0x1p-53 * sdsv;
    }
}

__global__ void k_rc_reset_list(DevState *st) {
    if (threadIdx.x == 0 && !st->done) st->n_list = 0;
}

template <typename X>
__global__ __launch_bounds__(256) void k_rc_copy(const X *__restrict__ src, X *__restrict__ dst,
                                                 int64_t cnt) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < cnt) dst[t] = src[t];
}


// ================================================================ BUILD (FP64)
// BUILD of this form runs in FP64, so its choices need no error bound:
// A(c) = sum_o min(d64(o,c), dn(o)) over all objects in the first two steps,
// then, per step, the change sum over the objects whose dn dropped of
// min(d64, dn_new) - min(d64, dn_old).  One thread per candidate with its
// point in registers as doubles; objects in tiles of 32 staged in LDS as
// doubles (every lane reads the same entry); d64 is the same expression as
// the re-scoring distance (coordinates past dim add an exact 0).
constexpr int kB64Tile = 32;

template <int KS>
__global__ __launch_bounds__(256) void k_rc64_build_pass(
    const float *__restrict__ X, int32_t dim, int64_t n, const int32_t *__restrict__ rows,
    const double *__restrict__ vold, const double *__restrict__ vnew,
    const DevState *__restrict__ st, int64_t ncp, double *__restrict__ part) {
    constexpr int MD = 16 * KS;
    __shared__ __align__(16) double xs[kB64Tile][MD];
    __shared__ double vo[kB64Tile], vn[kB64Tile];
    const int tid = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * 256 + tid;
    const int64_t m = rows ? (int64_t)st->n_chg : n;
    const int Qd = gridDim.y, q = blockIdx.y;
    const int64_t Ld = (m + Qd - 1) / Qd;
    const int64_t a = min((int64_t)q * Ld, m), b = min(a + Ld, m);
    double xc[MD];
#pragma unroll
    for (int k = 0; k < MD; ++k) xc[k] = (c < n && k < dim) ? (double)X[c * dim + k] : 0.0;
    for (int e = tid; e < kB64Tile * MD; e += 256) xs[e / MD][e % MD] = 0.0;   // padding stays 0
    double acc = 0.0;
    for (int64_t j0 = a; j0 < b; j0 += kB64Tile) {
        const int cnt = (int)min((int64_t)kB64Tile, b - j0);
        __syncthreads();
        // all loads of the tile first (clamped, always valid), then the stores
        constexpr int kIt = (kB64Tile * MD + 255) / 256;
        float v[kIt];
        const int tot = cnt * dim;
#pragma unroll
        for (int u = 0; u < kIt; ++u) {
            const int e = min(tid + u * 256, tot - 1);
            const int r = e / dim, kk = e - r * dim;
            const int64_t o = rows ? (int64_t)rows[j0 + r] : j0 + r;
            v[u] = X[o * dim + kk];
        }
#pragma unroll
        for (int u = 0; u < kIt; ++u) {
            const int e = tid + u * 256;
            if (e < tot) {
                const int r = e / dim, kk = e - r * dim;
                xs[r][kk] = (double)v[u];
            }
        }
        if (tid < cnt) {
            vn[tid] = vnew[j0 + tid];
            vo[tid] = vold ? vold[j0 + tid] : 0.0;
        }
        __syncthreads();
        for (int r = 0; r < cnt; ++r) {
            double s2 = 0.0;
#pragma unroll
            for (int k = 0; k < MD; ++k) {
                const double t = xs[r][k] - xc[k];
                s2 = fma(t, t, s2);
            }
            const double d = sqrt(s2);
            acc += vold ? fmin(d, vn[r]) - fmin(d, vo[r]) : fmin(d, vn[r]);
        }
    }
    part[(int64_t)q * ncp + c] = acc;
}

// A(c) <- (full ? 0 : A(c)) + chunk sums in chunk order; the work-group's
// best (value, candidate) among non-medoids (value + dn(c) for the literal
// reading of Alg. 1).
__global__ __launch_bounds__(256) void k_rc64_build_merge(
    const double *__restrict__ part, int32_t Q, int64_t ncp, int64_t n, int32_t full,
    double *__restrict__ acur, const double *__restrict__ dn64, const uint8_t *__restrict__ is_med,
    int32_t add_self, double *__restrict__ wg_v, int32_t *__restrict__ wg_c) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v = __builtin_huge_val();
    int ci = INT_MAX;
    if (c < n) {
        double s2 = 0.0;
        for (int q = 0; q < Q; ++q) s2 += part[(int64_t)q * ncp + c];
        const double a2 = full ? s2 : acur[c] + s2;
        acur[c] = a2;
        if (!is_med[c]) {
            v = add_self ? a2 + dn64[c] : a2;
            ci = (int)c;
        }
    }
    int dummy = 0;
    block_argmin3<double, 256>(v, dummy, ci);
    if (threadIdx.x == 0) {
        wg_v[blockIdx.x] = v;
        wg_c[blockIdx.x] = ci;
    }
}

// The step's medoid (every block reduces the merge partials: smallest value,
// smallest index on ties; block 0 records it), then dn' = min(dn, d64(., m))
// into the other buffer and the per-block count of objects whose dn dropped.
__global__ __launch_bounds__(kObjBlk) void k_rc64_select_update(
    const double *__restrict__ wg_v, const int32_t *__restrict__ wg_c, int32_t nwg, int32_t t,
    int32_t *__restrict__ med, uint8_t *__restrict__ is_med, const float *__restrict__ X,
    int32_t dim, int64_t n, const double *__restrict__ dn64, double *__restrict__ dn64n,
    float *__restrict__ dn32n, DevState *__restrict__ st, int32_t *__restrict__ blkcnt) {
    double v = __builtin_huge_val();
    int c = INT_MAX, dummy = 0;
    for (int w = threadIdx.x; w < nwg; w += kObjBlk)
        if (lex_less(wg_v[w], 0, wg_c[w], v, 0, c)) { v = wg_v[w]; c = wg_c[w]; }
    block_argmin3<double, kObjBlk>(v, dummy, c);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->best_c = c;
        if (c != INT_MAX) {
            med[t] = c;
            is_med[c] = 1;
        } else {
            st->bad_medoids = 1;  // no candidate left (cannot happen for k <= n)
        }
    }
    const int64_t o = (int64_t)blockIdx.x * kObjBlk + threadIdx.x;
    int chg = 0;
    if (o < n) {
        const double old = dn64[o];
        double nw = old;
        if (c != INT_MAX) nw = fmin(old, d64(X, dim, o, c));
        dn64n[o] = nw;
        dn32n[o] = (float)nw;
        chg = nw < old;
    }
    const int cnt = __syncthreads_count(chg);
    if (threadIdx.x == 0) blkcnt[blockIdx.x] = cnt;
}

// Stable list (ascending object) of the objects whose dn dropped, with their
// old and new dn; the total goes to the device state.
__global__ __launch_bounds__(kObjBlk) void k_rc64_compact(
    const double *__restrict__ dn_old, const double *__restrict__ dn_new, int64_t n,
    const int32_t *__restrict__ blkcnt, int32_t nblk, int32_t *__restrict__ lobj,
    double *__restrict__ lold, double *__restrict__ lnew, DevState *__restrict__ st) {
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
    double old = 0.0, nw = 0.0;
    bool chg = false;
    if (o < n) {
        old = dn_old[o];
        nw = dn_new[o];
        chg = nw < old;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long msk = __ballot(chg);
    if (lane == 0) wcnt[wv] = __popcll(msk);
    __syncthreads();
    int rank = __popcll(msk & ((1ull << lane) - 1ull));
    for (int w = 0; w < wv; ++w) rank += wcnt[w];
    if (chg) {
        const int pos = pre + rank;
        lobj[pos] = (int32_t)o;
        lold[pos] = old;
        lnew[pos] = nw;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_chg = tot;
        st->build_rows += tot;
    }
}

// ================================================================ host side
struct RcPtrs {
    __bf16 *Xs;
    float *nb, *dn32, *ds32, *sdn, *sds, *sthr, *snb;
    void *part;
    double *eo, *dn64, *ds64, *R64, *mx, *eps0, *bnd, *wg_u, *res_v, *cand_v, *cand_b, *tdp;
    int32_t *near, *sec, *srow, *blkcnt, *segtot, *seg_off, *cinfo4, *part_i, *list, *res_i, *rlist;
    uint8_t *is_med;
    DevState *st;
    double *acur, *lold, *lnew;
    double *rs_part;   // re-score partials of (candidate, object group)
};

template <int KS, typename ACC>
static void rc_swap_pass_launch(const RcPtrs &p, const RcLayout &R, int64_t n, int k, hipStream_t s) {
    hipLaunchKernelGGL((k_rc_swap_pass<KS, ACC>), dim3(R.n_ctiles, R.Q), dim3(kRT), 0, s,
                       (const __bf16 *)p.Xs, R.KP, (const float *)p.nb, n, k,
                       (const int32_t *)p.srow, (const float *)p.sdn, (const float *)p.sds,
                       (const float *)p.sthr, (const float *)p.snb, (const double *)p.eps0,
                       (const int32_t *)p.seg_off, (const double *)p.R64, (const int32_t *)p.cinfo4,
                       R.L, R.ncp, static_cast<ACC *>(p.part), p.part_i, (const DevState *)p.st);
}

template <typename ACC>
static void rc_swap_pass_any(const RcPtrs &p, const RcLayout &R, int64_t n, int k, hipStream_t s) {
    switch (R.KP / 16) {
        case 1: rc_swap_pass_launch<1, ACC>(p, R, n, k, s); break;
        case 2: rc_swap_pass_launch<2, ACC>(p, R, n, k, s); break;
        case 3: rc_swap_pass_launch<3, ACC>(p, R, n, k, s); break;
        default: rc_swap_pass_launch<4, ACC>(p, R, n, k, s); break;
    }
}

static void rc64_build_pass(const RcPtrs &p, const RcLayout &R, const float *X, int32_t dim,
                            int64_t n, const int32_t *rows, const double *vold, const double *vnew,
                            int32_t Q, hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)Q);
#define PAMX_B64(KS)                                                                            \
    hipLaunchKernelGGL((k_rc64_build_pass<KS>), grid, dim3(256), 0, s, X, dim, n, rows, vold, vnew, \
                       (const DevState *)p.st, R.ncp, static_cast<double *>(p.part))
    switch (R.KP / 16) {
        case 1: PAMX_B64(1); break;
        case 2: PAMX_B64(2); break;
        case 3: PAMX_B64(3); break;
        default: PAMX_B64(4); break;
    }
#undef PAMX_B64
}

static RcPtrs rc_ptrs(const RcLayout &R, void *ws) {
    char *w = static_cast<char *>(ws);
    RcPtrs p;
    p.Xs = reinterpret_cast<__bf16 *>(w + R.Xb);
    p.nb = reinterpret_cast<float *>(w + R.nb);
    p.eo = reinterpret_cast<double *>(w + R.eo);
    p.dn64 = reinterpret_cast<double *>(w + R.dn64);
    p.ds64 = reinterpret_cast<double *>(w + R.ds64);
    p.dn32 = reinterpret_cast<float *>(w + R.dn32);
    p.ds32 = reinterpret_cast<float *>(w + R.ds32);
    p.sdn = reinterpret_cast<float *>(w + R.sdn);
    p.sds = reinterpret_cast<float *>(w + R.sds);
    p.sthr = reinterpret_cast<float *>(w + R.sthr);
    p.snb = reinterpret_cast<float *>(w + R.snb);
    p.R64 = reinterpret_cast<double *>(w + R.R64);
    p.part = w + R.part;
    p.part_i = reinterpret_cast<int32_t *>(w + R.part_i);
    p.cand_v = reinterpret_cast<double *>(w + R.cand_v);
    p.cand_b = reinterpret_cast<double *>(w + R.cand_b);
    p.wg_u = reinterpret_cast<double *>(w + R.wg_u);
    p.list = reinterpret_cast<int32_t *>(w + R.list);
    p.res_v = reinterpret_cast<double *>(w + R.res_v);
    p.res_i = reinterpret_cast<int32_t *>(w + R.res_i);
    p.rs_part = reinterpret_cast<double *>(w + R.rs_part);
    p.rlist = reinterpret_cast<int32_t *>(w + R.rlist);
    p.near = reinterpret_cast<int32_t *>(w + R.near);
    p.sec = reinterpret_cast<int32_t *>(w + R.sec);
    p.srow = reinterpret_cast<int32_t *>(w + R.srow);
    p.blkcnt = reinterpret_cast<int32_t *>(w + R.blkcnt);
    p.tdp = reinterpret_cast<double *>(w + R.tdp);
    p.segtot = reinterpret_cast<int32_t *>(w + R.segtot);
    p.seg_off = reinterpret_cast<int32_t *>(w + R.seg_off);
    p.cinfo4 = reinterpret_cast<int32_t *>(w + R.cinfo);
    p.is_med = reinterpret_cast<uint8_t *>(w + R.is_med);
    p.mx = reinterpret_cast<double *>(w + R.mx);
    p.eps0 = reinterpret_cast<double *>(w + R.eps0);
    p.bnd = reinterpret_cast<double *>(w + R.bnd);
    p.st = reinterpret_cast<DevState *>(w + R.state);
    p.acur = reinterpret_cast<double *>(w + R.acur);
    p.lold = reinterpret_cast<double *>(w + R.lold);
    p.lnew = reinterpret_cast<double *>(w + R.lnew);
    return p;
}

template <typename X>
__global__ void k_rc_fill(X *p, int64_t cnt, X v) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < cnt) p[t] = v;
}
template <typename X>
static void rc_fill(X *p, int64_t cnt, X v, hipStream_t s) {
    if (cnt > 0) hipLaunchKernelGGL(k_rc_fill<X>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, cnt, v);
}

__global__ void k_rc_state_init(DevState *st, int32_t max_iter, int32_t trace_cap) {
    if (threadIdx.x == 0) {
        DevState z{};
        z.max_iter = max_iter;
        z.trace_cap = trace_cap;
        *st = z;
    }
}

// prep + BUILD (Alg. 1) in the mixed-precision form
hipError_t rc_prep_build(const float *X, int32_t dim, const RcLayout &R, int32_t k,
                         const pamx_options &opt, int32_t *medoids, void *ws, hipStream_t s,
                         const float *mean) {
    RcPtrs p = rc_ptrs(R, ws);
    const int64_t n = R.n;
    const bool acc64 = opt.accum != PAMX_ACC_F32;
    const unsigned ob = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_rc_prep, dim3(ob), dim3(256), 0, s, X, n, dim, R.KP, mean, p.Xs, p.nb, p.eo);
    hipLaunchKernelGGL(k_rc_prep_max, dim3(1), dim3(1024), 0, s, (const double *)p.eo,
                       (const float *)p.nb, n, p.mx);
    hipLaunchKernelGGL(k_rc_eps, dim3(1), dim3(1), 0, s, (const double *)p.mx, R.KP, p.eps0);
    hipLaunchKernelGGL(k_rc_state_init, dim3(1), dim3(1), 0, s, p.st, opt.max_iter,
                       opt.trace ? opt.trace_cap : 0);
    rc_fill<uint8_t>(p.is_med, n, 0, s);
    rc_fill<double>(p.dn64, n, __builtin_huge_val(), s);
    rc_fill<float>(p.dn32, n, __builtin_huge_valf(), s);
    const int nmwg = (int)((n + 255) / 256);
    const unsigned nblk = (unsigned)R.n_oblk;
    // object chunks of the FP64 passes: about two work-groups per CU for the
    // full steps, four chunks for the short lists of later steps
    const int64_t nct = (n + 255) / 256;
    int32_t qf = (int32_t)(512 / nct);
    if (qf < 1) qf = 1;
    if (qf > R.Q * 4) qf = R.Q * 4;   // the partial buffer holds 4 Q rows
    const int32_t qd = 4 <= R.Q * 4 ? 4 : 1;
    // dn ping-pongs between the dn and ds buffers (free until SWAP)
    double *d64b[2] = {p.dn64, p.ds64};
    float *d32b[2] = {p.dn32, p.ds32};
    int cur = 0;
    for (int32_t t = 0; t < k; ++t) {
        const int add_self = (opt.build_exclude_self && t > 0) ? 1 : 0;
        const bool full = t < 2;
        if (full) {
            rc64_build_pass(p, R, X, dim, n, nullptr, nullptr, d64b[cur], qf, s);
        } else {
            hipLaunchKernelGGL(k_rc64_compact, dim3(nblk), dim3(kObjBlk), 0, s,
                               (const double *)d64b[cur ^ 1], (const double *)d64b[cur], n,
                               (const int32_t *)p.blkcnt, R.n_oblk, p.srow, p.lold, p.lnew, p.st);
            rc64_build_pass(p, R, X, dim, n, p.srow, p.lold, p.lnew, qd, s);
        }
        hipLaunchKernelGGL(k_rc64_build_merge, dim3(nmwg), dim3(256), 0, s,
                           (const double *)p.part, full ? qf : qd, R.ncp, n, (int32_t)full, p.acur,
                           (const double *)d64b[cur], (const uint8_t *)p.is_med, add_self, p.wg_u,
                           p.res_i);
        hipLaunchKernelGGL(k_rc64_select_update, dim3(nblk), dim3(kObjBlk), 0, s,
                           (const double *)p.wg_u, (const int32_t *)p.res_i, nmwg, t, medoids,
                           p.is_med, X, dim, n, (const double *)d64b[cur], d64b[cur ^ 1],
                           d32b[cur ^ 1], p.st, p.blkcnt);
        cur ^= 1;
    }
    if (cur == 1) {   // the caller reads dn from the dn buffers
        hipLaunchKernelGGL(k_rc_copy<double>, dim3(ob), dim3(256), 0, s, (const double *)p.ds64,
                           p.dn64, n);
        hipLaunchKernelGGL(k_rc_copy<float>, dim3(ob), dim3(256), 0, s, (const float *)p.ds32,
                           p.dn32, n);
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_rc_td(const double *__restrict__ dn64, int64_t n,
                                                DevState *__restrict__ st) {
    double s = 0.0;
    for (int64_t o = threadIdx.x; o < n; o += 1024) s += dn64[o];
    s = block_sum<double, 1024>(s);
    if (threadIdx.x == 0) st->td = s;
}

hipError_t rc_td(const RcLayout &R, void *ws, hipStream_t s) {
    RcPtrs p = rc_ptrs(R, ws);
    hipLaunchKernelGGL(k_rc_td, dim3(1), dim3(1024), 0, s, (const double *)p.dn64, R.n, p.st);
    return hipGetLastError();
}

hipError_t rc_swap_init(const float *X, int32_t dim, const RcLayout &R, const int32_t *medoids,
                        const pamx_options &opt, void *ws, hipStream_t s) {
    RcPtrs p = rc_ptrs(R, ws);
    const int64_t n = R.n;
    hipLaunchKernelGGL(k_rc_state_init, dim3(1), dim3(1), 0, s, p.st, opt.max_iter,
                       opt.trace ? opt.trace_cap : 0);
    hipLaunchKernelGGL(k_rc_cache_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, dim, n,
                       R.k, medoids, p.near, p.sec, p.dn64, p.ds64, p.dn32, p.ds32, (int32_t *)nullptr);
    return hipGetLastError();
}

// segment kernels of swap.hip, reused on the FP32 cache copies
hipError_t launch_segments_f32(const int32_t *near, const float *dn, const float *ds, int64_t n,
                               int32_t k, int32_t n_oblk, int32_t *blkcnt, double *tdp,
                               int32_t *segtot, int32_t *seg_off, int32_t L, int32_t Q, void *cinfo,
                               int32_t *srow, float *sdn, float *sds, DevState *st, hipStream_t s);

hipError_t rc_swap_iteration(const float *X, int32_t dim, const RcLayout &R, int32_t *medoids,
                             const pamx_options &opt, void *ws, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1) {
    RcPtrs p = rc_ptrs(R, ws);
    const int64_t n = R.n;
    const int32_t k = R.k;
    const bool acc64 = opt.accum != PAMX_ACC_F32;
    const unsigned ob = (unsigned)((n + 255) / 256);
    const int nmwg = (int)((n + 255) / 256);
    hipError_t e = launch_segments_f32(p.near, p.dn32, p.ds32, n, k, R.n_oblk, p.blkcnt, p.tdp,
                                       p.segtot, p.seg_off, R.L, R.Q, p.cinfo4, p.srow, p.sdn, p.sds,
                                       p.st, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rc_seg_const, dim3((k + 3) / 4), dim3(256), 0, s, (const int32_t *)p.srow,
                       (const int32_t *)p.seg_off, k, (const double *)p.dn64, (const double *)p.ds64,
                       p.R64, (const DevState *)p.st);
    hipLaunchKernelGGL(k_rc_iter_bounds, dim3(1), dim3(1024), 0, s, (const double *)p.dn64,
                       (const double *)p.ds64, n, (const double *)p.R64, k, R.L, R.Q, (int32_t)acc64,
                       (const double *)p.eps0, p.bnd, p.st);
    hipLaunchKernelGGL(k_rc_sorted_aux, dim3(ob), dim3(256), 0, s, (const int32_t *)p.srow, n,
                       (const float *)p.sds, (const float *)p.nb, (const double *)p.eps0, p.sthr,
                       p.snb, (const DevState *)p.st);
    if (ev0) (void)hipEventRecord(ev0, s);
    if (acc64) rc_swap_pass_any<double>(p, R, n, k, s);
    else rc_swap_pass_any<float>(p, R, n, k, s);
    if (ev1) (void)hipEventRecord(ev1, s);
    if (acc64)
        hipLaunchKernelGGL(k_rc_swap_merge<double>, dim3(nmwg), dim3(256), 0, s, (const double *)p.part,
                           (const int32_t *)p.part_i, (const int32_t *)p.cinfo4, R.Q, n, k, R.ncp,
                           (const double *)p.R64, (const uint8_t *)p.is_med, (const DevState *)p.st,
                           (const double *)p.bnd, p.cand_v, p.cand_b, p.wg_u);
    else
        hipLaunchKernelGGL(k_rc_swap_merge<float>, dim3(nmwg), dim3(256), 0, s, (const float *)p.part,
                           (const int32_t *)p.part_i, (const int32_t *)p.cinfo4, R.Q, n, k, R.ncp,
                           (const double *)p.R64, (const uint8_t *)p.is_med, (const DevState *)p.st,
                           (const double *)p.bnd, p.cand_v, p.cand_b, p.wg_u);
    hipLaunchKernelGGL(k_rc_upper, dim3(1), dim3(1024), 0, s, (const double *)p.wg_u, nmwg, p.st);
    hipLaunchKernelGGL(k_rc_mark, dim3(nmwg), dim3(256), 0, s, (const double *)p.cand_v,
                       (const double *)p.cand_b, n, 1, p.list, p.st);
    {
        const hipError_t e = rc_rescore(R.KP, X, dim, n, k, (const int32_t *)p.srow,
                                        (const double *)p.dn64, (const double *)p.ds64,
                                        (const int32_t *)p.near, (const double *)p.R64,
                                        (const int32_t *)p.list, (const DevState *)p.st, p.res_v,
                                        p.res_i, p.rs_part, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_rc_pick, dim3(1), dim3(1024), 0, s, (const double *)p.res_v,
                       (const int32_t *)p.res_i, (const int32_t *)p.list, medoids, p.is_med, p.st,
                       static_cast<pamx_swap_record *>(opt.trace));
    hipLaunchKernelGGL(k_rc_reset_list, dim3(1), dim3(1), 0, s, p.st);
    hipLaunchKernelGGL(k_rc_cache_update, dim3(ob), dim3(256), 0, s, X, dim, n, p.near, p.sec, p.dn64,
                       p.ds64, p.dn32, p.ds32, p.rlist, p.st);
    hipLaunchKernelGGL(k_rc_cache_rescan, dim3(256), dim3(256), 0, s, X, dim, k,
                       (const int32_t *)medoids, p.near, p.sec, p.dn64, p.ds64, p.dn32, p.ds32,
                       (const int32_t *)p.rlist, (const DevState *)p.st);
    return hipGetLastError();
}

hipError_t rc_finalize(const float *X, int32_t dim, const RcLayout &R, const int32_t *medoids,
                       int32_t *labels, void *ws, hipStream_t s) {
    RcPtrs p = rc_ptrs(R, ws);
    const int64_t n = R.n;
    hipLaunchKernelGGL(k_rc_cache_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, dim, n,
                       R.k, medoids, p.near, p.sec, p.dn64, p.ds64, p.dn32, p.ds32, labels);
    hipLaunchKernelGGL(k_rc_td, dim3(1), dim3(1024), 0, s, (const double *)p.dn64, n, p.st);
    return hipGetLastError();
}

}  // namespace pamx
