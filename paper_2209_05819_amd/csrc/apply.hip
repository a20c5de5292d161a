// The HODLRdD matrix-vector product (paper Alg. "HODLRdD matrix-vector
// Product") on the device.  Per call:
//   1. permute-in: x = X in tree order, compute precision;
//   2. low-rank blocks: for a stored block (A,B) with factors U (|A| x r),
//      V (r x |B|): t = V x_B, c_A = U t, and when the block also stands for
//      its transpose, s = U^T x_A, c_B = V^T s.  c_A and c_B go to the block's
//      segments of a contribution buffer.  A block small enough for one wave
//      is done entirely by that wave: projection, then expansion re-reading
//      the factors it has just streamed (cache hits).  Larger blocks are split
//      into row ranges (projection) and 64-row chunks (expansion);
//   3. gather + near field + permute-out, one wave per 64 rows of a leaf: the
//      contributions of every level's box containing the rows are summed in
//      interaction-list order, the near field is evaluated on the fly, and the
//      result goes to Y in user order.
// Each output is produced by one lane in a fixed order: results are bitwise
// reproducible and no floating-point atomics are used.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int TP = 256;   // split projection workgroup (4 waves)
constexpr int TE = 256;   // split expansion workgroup (4 waves share 64 rows)
constexpr int KB = 16;    // rows reduced together in the fused projection
constexpr int kFusedMaxRank = 64;   // projections a fused wave keeps in LDS at once
constexpr int kNumClasses = kApplyClasses;  // block size classes of the one-workgroup kernels
// class-5 blocks (up to 4608 rows) take the segmented route in the persistent
// plan: streaming one of them per workgroup needs more registers than the
// other work of the persistent kernel and would cut its occupancy for all


// Cross-lane moves that stay in the vector ALU: DPP row permutations for
// lane distances up to 8, and the permlane swaps of CDNA4 for 16 and 32
// (lanes exchange whole 16- or 32-lane halves between two registers).  None
// of them goes through the LDS crossbar, unlike a general shuffle.
template <int OFF>
__device__ __forceinline__ int dpp_xor(int v) {
    static_assert(OFF == 1 || OFF == 2 || OFF == 4 || OFF == 8, "DPP distance");
    if constexpr (OFF == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad [1,0,3,2]
    if constexpr (OFF == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
    if constexpr (OFF == 4)   // quad [3,2,1,0] then mirror within 8 lanes: l -> l ^ 4
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, false),
                                        0x141, 0xF, 0xF, false);
    if constexpr (OFF == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);  // rotate row by 8
}

template <int OFF, typename C>
__device__ __forceinline__ C lane_xor(C v) {
    if constexpr (sizeof(C) == 4) {
        return __int_as_float(dpp_xor<OFF>(__float_as_int(v)));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = dpp_xor<OFF>((int)(b & 0xffffffffLL)), hi = dpp_xor<OFF>((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}

// Given a and b in every lane, returns in lane L the sum a_L + a_{L^OFF}
// when bit OFF of L is clear and b_L + b_{L^OFF} when it is set (OFF = 16 or
// 32).  One swap moves a's upper halves and b's lower halves across, so the
// sum is a single add.
template <int OFF>
__device__ __forceinline__ void half_swap(unsigned int& a, unsigned int& b) {
    if constexpr (OFF == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        static_assert(OFF == 16, "swap distance");
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int OFF, typename C>
__device__ __forceinline__ C pair_sum(C a, C b) {
    if constexpr (sizeof(C) == 4) {
        unsigned int x = __float_as_uint(a), y = __float_as_uint(b);
        half_swap<OFF>(x, y);
        return __uint_as_float(x) + __uint_as_float(y);
    } else {
        const unsigned long long ab = (unsigned long long)__double_as_longlong(a);
        const unsigned long long bb = (unsigned long long)__double_as_longlong(b);
        unsigned int alo = (unsigned int)ab, ahi = (unsigned int)(ab >> 32);
        unsigned int blo = (unsigned int)bb, bhi = (unsigned int)(bb >> 32);
        half_swap<OFF>(alo, blo);
        half_swap<OFF>(ahi, bhi);
        return __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo)) +
               __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
    }
}

// One halving step of multi_reduce at lane distance OFF over the first
// 2 HALF values: afterwards p[kk] (kk < HALF) holds row kk's pair sum in
// lanes with bit OFF clear and row HALF + kk's in lanes with it set.
template <int OFF, int HALF, typename C, int K>
__device__ __forceinline__ void reduce_step(C (&p)[K]) {
    if constexpr (OFF >= 16) {
#pragma unroll
        for (int kk = 0; kk < HALF; ++kk) p[kk] = pair_sum<OFF>(p[kk], p[HALF + kk]);
    } else {
        const bool upper = ((threadIdx.x & 63) & OFF) != 0;
#pragma unroll
        for (int kk = 0; kk < HALF; ++kk) {
            const C keep = upper ? p[HALF + kk] : p[kk];
            const C give = upper ? p[kk] : p[HALF + kk];
            p[kk] = keep + lane_xor<OFF>(give);
        }
    }
}

// Sum of v over groups of 2 OFF lanes (then OFF / 2, ... down to 1 lane).
template <int OFF, typename C>
__device__ __forceinline__ C lane_sum_to(C v) {
    if constexpr (OFF >= 16) {
        v = pair_sum<OFF>(v, v);
    } else {
        v += lane_xor<OFF>(v);
    }
    if constexpr (OFF > 1) {
        return lane_sum_to<OFF / 2>(v);
    } else {
        return v;
    }
}

// Reduce K = 2^q partial sums per lane over the 64 lanes at once: at each
// halving step a lane keeps half of its values and receives its partner's
// matching half, so K sums cost K-1 exchanges plus 6-q plain steps (instead
// of 6 K).  On return lane L holds the full sum of row (L >> (6 - q)).
template <int OFF, int WIDTH, typename C, int K>
__device__ __forceinline__ C multi_reduce_from(C (&p)[K]) {
    if constexpr (WIDTH > 1) {
        reduce_step<OFF, WIDTH / 2>(p);
        return multi_reduce_from<OFF / 2, WIDTH / 2>(p);
    } else {
        return lane_sum_to<OFF>(p[0]);
    }
}

template <typename C, int K>
__device__ __forceinline__ C multi_reduce(C (&p)[K]) {
    return multi_reduce_from<32, K>(p);
}

template <typename C>
__device__ __forceinline__ C wsum(C v) {
    return lane_sum_to<32>(v);
}

// Value of v in lane L (a compile-time constant) as a wave-uniform scalar.
template <int L, typename C>
__device__ __forceinline__ C lane_value(C v) {
    if constexpr (sizeof(C) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), L);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), L);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}

// out[k] = v in lane k 2^(6-Q), k < K: the row sums multi_reduce leaves.
template <int Q, int KK = 0, typename C, int K>
__device__ __forceinline__ void row_values(C v, C (&out)[K]) {
    out[KK] = lane_value<(KK << (6 - Q))>(v);
    if constexpr (KK + 1 < K) row_values<Q, KK + 1>(v, out);
}

template <int K>
struct Log2;
template <>
struct Log2<1> { static constexpr int v = 0; };
template <>
struct Log2<2> { static constexpr int v = 1; };
template <>
struct Log2<4> { static constexpr int v = 2; };
template <>
struct Log2<8> { static constexpr int v = 3; };
template <>
struct Log2<16> { static constexpr int v = 4; };

template <typename XT, typename C>
__global__ void k_permute_in(const XT* __restrict__ X, int64_t ldx, int nrhs, int64_t N,
                             const int32_t* __restrict__ perm, C* __restrict__ x) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t u = perm[p];
    for (int c = 0; c < nrhs; ++c) x[c * N + p] = (C)X[c * ldx + u];
}

// Y[:, c0 + c] = the level sums yl[c] plus the near sums yn[c] (both in tree
// order), in user order, c < nc.
template <typename XT>
__global__ void k_permute_out(const float* __restrict__ yl, const float* __restrict__ yn,
                              int64_t N, int nc, int c0, const int32_t* __restrict__ perm,
                              XT* __restrict__ Y, int64_t ldy) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t u = perm[p];
    for (int c = 0; c < nc; ++c)
        Y[(int64_t)(c0 + c) * ldy + u] = (XT)(yl[(int64_t)c * N + p] + yn[(int64_t)c * N + p]);
}

// Loads and stores of the vectors one launch both writes and reads (x, the
// contributions, projections and near sums).  CO: device-coherent accesses
// (relaxed agent-scope atomics, which neither stop at nor hit stale lines of
// an XCD's own L2), for a launch whose workgroups hand these vectors to each
// other; otherwise plain ones.
// (The vectors live in global memory: saying so gives global instead of
// flat instructions, which would also wait on the LDS.)
template <bool CO, typename C>
__device__ __forceinline__ C ldv(const C* p) {
    if constexpr (CO)
        return __hip_atomic_load((const C __attribute__((address_space(1)))*)p, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}
template <bool CO, typename C>
__device__ __forceinline__ void stv(C* p, C v) {
    if constexpr (CO)
        __hip_atomic_store((C __attribute__((address_space(1)))*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// Orders a wave's LDS writes before its later reads by other lanes of the
// same wave (the LDS runs one wave's instructions in order; only the
// compiler must not move them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave applies one stored block with NR right-hand sides: the
// projections of up to RMAX terms (multi-row reductions in batches of K),
// then their expansion re-reading the factors (cache hits); repeated over
// chunks of RMAX terms, accumulating into the contribution segments.
// The body works on one wave's own LDS (tw, sw: RMAX x NR each) and
// synchronises within the wave only, so the waves of a larger workgroup can
// each apply a block of their own.
template <typename S, typename C, int NR, int RMAX, bool CO = false>
__device__ __forceinline__ void lr_fused_body(const BlockDesc& b, int sym,
                                              const C* __restrict__ x, int64_t N, int nrhs,
                                              int c0, int64_t CT, C* __restrict__ contrib,
                                              C (*tw)[NR], C (*sw)[NR]) {
    constexpr int K = NR == 1 ? KB : 4;
    constexpr int Q = Log2<K>::v;
    const int lane = threadIdx.x & 63;
    const gptr_t<S> U = as_global<S>(b.U);
    const gptr_t<S> V = as_global<S>(b.V);
    const int nc = min(NR, nrhs - c0);
    const int r = b.rank, m = b.m, n = b.n;
    const int64_t lu = fstride<S>(m), lv = fstride<S>(n);
    const C* __restrict__ xA = x + (int64_t)c0 * N + b.a0;
    const C* __restrict__ xB = x + (int64_t)c0 * N + b.b0;
    for (int kc = 0; kc == 0 || kc < r; kc += RMAX) {
        const int rc = min(RMAX, r - kc);   // terms of this chunk (0 if r == 0)
        for (int k0 = 0; k0 < rc; k0 += K) {
            C pv[NR][K], pu[NR][K];
#pragma unroll
            for (int c = 0; c < NR; ++c)
#pragma unroll
                for (int kk = 0; kk < K; ++kk) pv[c][kk] = pu[c][kk] = 0;
            const int kr = min(K, rc - k0);
            for (int j = lane; j < n; j += 64) {
                C xv[NR];
#pragma unroll
                for (int c = 0; c < NR; ++c) xv[c] = c < nc ? ldv<CO>(xB + (int64_t)c * N + j) : (C)0;
#pragma unroll
                for (int kk = 0; kk < K; ++kk)
                    if (kk < kr) {
                        const C v = ldf<C>(V, (int64_t)(kc + k0 + kk) * lv + j);
#pragma unroll
                        for (int c = 0; c < NR; ++c) pv[c][kk] += v * xv[c];
                    }
            }
            if (sym) {
                for (int i = lane; i < m; i += 64) {
                    C xu[NR];
#pragma unroll
                    for (int c = 0; c < NR; ++c)
                        xu[c] = c < nc ? ldv<CO>(xA + (int64_t)c * N + i) : (C)0;
#pragma unroll
                    for (int kk = 0; kk < K; ++kk)
                        if (kk < kr) {
                            const C u = ldf<C>(U, (int64_t)(kc + k0 + kk) * lu + i);
#pragma unroll
                            for (int c = 0; c < NR; ++c) pu[c][kk] += u * xu[c];
                        }
                }
            }
            const int row = lane >> (6 - Q);
            const bool writer = (lane & ((1 << (6 - Q)) - 1)) == 0 && row < kr;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const C tv = multi_reduce<C, K>(pv[c]);
                if (writer) tw[k0 + row][c] = tv;
                if (sym) {
                    const C sv = multi_reduce<C, K>(pu[c]);
                    if (writer) sw[k0 + row][c] = sv;
                }
            }
        }
        wave_sync();
        // expansion of this chunk: c_A += U t (and c_B += V^T s)
        for (int i = lane; i < m; i += 64) {
            C acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = (kc > 0 && c < nc) ? ldv<CO>(contrib + (int64_t)c * CT + b.cfwd + i) : (C)0;
#pragma unroll 4
            for (int k = 0; k < rc; ++k) {
                const C u = ldf<C>(U, (int64_t)(kc + k) * lu + i);
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += u * tw[k][c];
            }
            for (int c = 0; c < nc; ++c) stv<CO>(contrib + (int64_t)c * CT + b.cfwd + i, acc[c]);
        }
        if (sym) {
            for (int j = lane; j < n; j += 64) {
                C acc[NR];
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    acc[c] =
                        (kc > 0 && c < nc) ? ldv<CO>(contrib + (int64_t)c * CT + b.cbwd + j) : (C)0;
#pragma unroll 4
                for (int k = 0; k < rc; ++k) {
                    const C v = ldf<C>(V, (int64_t)(kc + k) * lv + j);
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += v * sw[k][c];
                }
                for (int c = 0; c < nc; ++c)
                    stv<CO>(contrib + (int64_t)c * CT + b.cbwd + j, acc[c]);
            }
        }
        wave_sync();
    }
}

template <typename S, typename C, int NR, int RMAX>
__global__ __launch_bounds__(64) void k_lr_fused(const BlockDesc* __restrict__ blocks, int sym,
                                                 const C* __restrict__ x, int64_t N, int nrhs,
                                                 int c0, int64_t CT, C* __restrict__ contrib) {
    __shared__ C tw[RMAX][NR], sw[RMAX][NR];
    lr_fused_body<S, C, NR, RMAX>(blocks[blockIdx.x], sym, x, N, nrhs, c0, CT, contrib, tw, sw);
}

// Single pass over a block's factors.  Each rank term k contributes
// independently: t_k = V[k,:] x_B, s_k = U[:,k] x_A, then c_A += U[:,k] t_k
// and c_B += V[k,:]^T s_k.  A workgroup of W waves streams the terms in
// batches of KB, each lane holding CH rows of A and CH columns of B (so
// |A|, |B| <= 64 W CH): a batch's factor values stay in registers between the
// dot products and the accumulation, so every factor byte is read from
// memory exactly once.  Two register buffers alternate: the loads of the next
// batch are in flight while the current one is reduced and accumulated.
template <typename S, typename C, int W, int CH, int KB>
struct StreamBatch {
    C u[KB][CH], v[KB][CH];
};

template <typename S, typename C, int W, int CH, int KB>
__device__ __forceinline__ void stream_load(StreamBatch<S, C, W, CH, KB>& bt, gptr_t<S> U,
                                            gptr_t<S> V, int k0, int r, int m, int n,
                                            int base) {
    const int kr = r - k0;   // may be <= 0: nothing is loaded
    const int lu = (int)fstride<S>(m), lv = (int)fstride<S>(n);
    gptr_t<S> Vk = V + k0 * lv;
    gptr_t<S> Uk = U + k0 * lu;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + c * 64;
            bt.v[kk][c] = (kk < kr && i < n) ? ldf_once<C>(Vk, kk * lv + i) : (C)0;
            bt.u[kk][c] = (kk < kr && i < m) ? ldf_once<C>(Uk, kk * lu + i) : (C)0;
        }
}

template <typename S, typename C, int W, int CH, int KB>
__device__ __forceinline__ void stream_step(const StreamBatch<S, C, W, CH, KB>& bt, int sym,
                                            const C (&xa)[CH], const C (&xb)[CH], C (&ca)[CH],
                                            C (&cb)[CH], C (*part)[2][KB]) {
    constexpr int Q = Log2<KB>::v;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    C pt[KB], ps[KB];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
        pt[kk] = ps[kk] = 0;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            pt[kk] += bt.v[kk][c] * xb[c];
            ps[kk] += bt.u[kk][c] * xa[c];
        }
    }
    const C tv = multi_reduce<C, KB>(pt);
    const C sv = sym ? multi_reduce<C, KB>(ps) : (C)0;
    C tk[KB], sk[KB];
    if (W == 1) {
        row_values<Q>(tv, tk);
        if (sym) {
            row_values<Q>(sv, sk);
        } else {
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) sk[kk] = 0;
        }
    } else {
        const int row = lane >> (6 - Q);
        if ((lane & ((1 << (6 - Q)) - 1)) == 0) {
            part[wv][0][row] = tv;
            part[wv][1][row] = sv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            C a = 0, s2 = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                a += part[w][0][kk];
                s2 += part[w][1][kk];
            }
            tk[kk] = a;
            sk[kk] = s2;
        }
        __syncthreads();
    }
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            ca[c] += bt.u[kk][c] * tk[kk];
            cb[c] += bt.v[kk][c] * sk[kk];
        }
}

// wv: the wave's index within the W waves applying the block (0 when W = 1,
// whatever the wave's place in a larger workgroup)
template <typename S, typename C, int W, int CH, int KB, bool CO = false>
__device__ __forceinline__ void lr_stream_body(const BlockDesc& b, int sym,
                                               const C* __restrict__ x, C* __restrict__ contrib,
                                               C (*part)[2][KB], int wv) {
    const int lane = threadIdx.x & 63;
    const int r = b.rank, m = b.m, n = b.n;
    const gptr_t<S> U = as_global<S>(b.U);
    const gptr_t<S> V = as_global<S>(b.V);
    const int base = wv * 64 * CH + lane;
    C xa[CH], xb[CH], ca[CH], cb[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int i = base + c * 64;
        xa[c] = i < m ? ldv<CO>(x + b.a0 + i) : (C)0;
        xb[c] = i < n ? ldv<CO>(x + b.b0 + i) : (C)0;
        ca[c] = cb[c] = 0;
    }
    StreamBatch<S, C, W, CH, KB> b0, b1;
    stream_load(b0, U, V, 0, r, m, n, base);
    for (int k0 = 0; k0 < r; k0 += 2 * KB) {
        stream_load(b1, U, V, k0 + KB, r, m, n, base);
        stream_step(b0, sym, xa, xb, ca, cb, part);
        if (k0 + KB >= r) break;
        stream_load(b0, U, V, k0 + 2 * KB, r, m, n, base);
        stream_step(b1, sym, xa, xb, ca, cb, part);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int i = base + c * 64;
        if (i < m) stv<CO>(contrib + b.cfwd + i, ca[c]);
        if (sym && i < n) stv<CO>(contrib + b.cbwd + i, cb[c]);
    }
}

template <typename S, typename C, int W, int CH, int KB>
__global__ __launch_bounds__(64 * W) void k_lr_stream(const BlockDesc* __restrict__ blocks, int sym,
                                                      const C* __restrict__ x,
                                                      C* __restrict__ contrib) {
    __shared__ C part[W][2][KB];
    lr_stream_body<S, C, W, CH, KB>(blocks[blockIdx.x], sym, x, contrib, part,
                                    W == 1 ? 0 : (int)(threadIdx.x >> 6));
}

// Reduction of G values per lane over a group of G lanes (G a power of two):
// lane g of the group returns the group sum of row g.
template <typename C, int G>
__device__ __forceinline__ C group_reduce_rows(C (&p)[G]) {
    const int g = threadIdx.x & (G - 1);
    int width = G;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        const int half = width >> 1;
        const bool upper = (g & off) != 0;
#pragma unroll
        for (int kk = 0; kk < G / 2; ++kk) {
            if (kk < half) {
                const C keep = upper ? p[half + kk] : p[kk];
                const C give = upper ? p[kk] : p[half + kk];
                p[kk] = keep + __shfl_xor(give, off, 64);
            }
        }
        width = half;
    }
    return p[0];
}

// Blocks with |A|, |B|, rank <= G: a group of G lanes applies one block
// (64/G blocks per wave).  Lane g holds column g of U^T (row g of U) in
// registers; V is read twice, the second time from cache.
// A 256-thread workgroup applies the blocks first .. first + 256 / G - 1.
template <typename S, typename C, int G, bool CO = false>
__device__ __forceinline__ void lr_group_body(const BlockDesc* __restrict__ blocks,
                                              int64_t first, int64_t nitems, int sym,
                                              const C* __restrict__ x, C* __restrict__ contrib) {
    const int g = threadIdx.x & (G - 1);
    const int base = (threadIdx.x & 63) & ~(G - 1);   // first lane of the group
    const int64_t item = first + threadIdx.x / G;
    const bool valid = item < nitems;
    BlockDesc b{};
    if (valid) b = blocks[item];
    const int r = valid ? b.rank : 0, m = b.m, n = b.n;
    const gptr_t<S> U = as_global<S>(b.U);
    const gptr_t<S> V = as_global<S>(b.V);
    C u[G], v[G], p[G];
    const int lu = (int)fstride<S>(m), lv = (int)fstride<S>(n);
#pragma unroll
    for (int k = 0; k < G; ++k) {
        u[k] = (k < r && g < m) ? ldf<C>(U, k * lu + g) : (C)0;
        v[k] = (k < r && g < n) ? ldf<C>(V, k * lv + g) : (C)0;
    }
    const C xa = (valid && g < m) ? ldv<CO>(x + b.a0 + g) : (C)0;
    const C xb = (valid && g < n) ? ldv<CO>(x + b.b0 + g) : (C)0;
#pragma unroll
    for (int k = 0; k < G; ++k) p[k] = v[k] * xb;
    const C t = group_reduce_rows<C, G>(p);    // t_g = V[g,:] . x_B
    C s = 0;
    if (sym) {
#pragma unroll
        for (int k = 0; k < G; ++k) p[k] = u[k] * xa;
        s = group_reduce_rows<C, G>(p);          // s_g = U[:,g] . x_A
    }
    C ca = 0, cb = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        ca += u[k] * __shfl(t, base + k, 64);
        cb += v[k] * __shfl(s, base + k, 64);
    }
    if (valid && g < m) stv<CO>(contrib + b.cfwd + g, ca);
    if (valid && sym && g < n) stv<CO>(contrib + b.cbwd + g, cb);
}

template <typename S, typename C, int G>
__global__ __launch_bounds__(256) void k_lr_group(const BlockDesc* __restrict__ blocks,
                                                  int64_t nitems, int sym,
                                                  const C* __restrict__ x,
                                                  C* __restrict__ contrib) {
    lr_group_body<S, C, G>(blocks, (int64_t)blockIdx.x * (256 / G), nitems, sym, x, contrib);
}

// ---------------------------------------------------------------------------
// Matrix-core product of BF16 factors with NRP = 16 CT right-hand sides.
//
// Each factor element takes part in two contractions (over the rows of the
// block in the projection, over the rank in the expansion), so the product
// runs in two passes that each read every factor once:
//   pass 1 (k_mproj): per stored block t = V x_B and, when the block also
//     stands for its transpose, s = U^T x_A, on 16x16x32 BF16 matrix cores;
//     a workgroup of W waves takes a panel of at most 64 W G columns, 64 G
//     per wave, 16 terms at a time, and sums its waves' partials through
//     LDS (32 right-hand sides, panels up to 64 columns: W = 1, G = 1;
//     128: 1, 2; 256: 2, 2; 512: 2, 4 -- fewer waves with more columns each
//     meet less often; 16 right-hand sides: W = 1, 2, 4, 8 and G = 1).
//     Blocks wider than 512 are projected in several panels whose FP32
//     partials k_mreduce adds in panel order.  Projections are stored in
//     BF16 in the operand layout of pass 2.
//   pass 2 (k_mexp): one wave per 16 RT rows of a target box A at a
//     level (boxes up to 192 rows: one wave; larger ones: workgroups of 4
//     waves x 128 rows sharing the projections) accumulates, over A's
//     interaction-list entries in order,
//     C += F_e t_e (F_e the entry's factor with |A| rows: U of (A,B), or V of
//     the stored (B,A) whose s it takes) on 16x16x16 BF16 matrix cores, in
//     FP32 registers, and adds C to the level sum y once.  No per-block
//     output buffer: a box's result leaves the chip once per level.
// Pass 2 needs 4 consecutive terms of a row per lane while the factor is
// stored term by term: each 16-term chunk of the tile is staged in LDS with
// 16-byte loads and read back transposed.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4_t __attribute__((ext_vector_type(4)));
typedef short s16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int MR = 64;        // factor columns per wave in a projection job
constexpr int MPANEL = 512;   // widest projection panel (8 waves)
constexpr int MSMALL = 192;   // boxes up to this many rows: one wave (12 row tiles)
constexpr int MBIGW = 4;      // larger boxes: workgroups of 4 waves x 128 rows
constexpr int MPAD = 8;       // LDS row padding of a staged chunk (elements)

// Workgroups are dispatched to the 8 XCDs in turn (workgroup i to XCD i mod
// 8), each XCD with its own L2.  With a grid of 8 ceil(n / 8) workgroups,
// this maps the workgroups of one XCD to one contiguous range of the n
// items, so items that read the same data (jobs sorted by the x slice they
// read) share that XCD's L2.  Returns -1 for the padding past n.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t n) {
    const int64_t per = (n + kXcds - 1) / kXcds;
    const int64_t j = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    return j < n ? j : -1;
}
inline unsigned xcd_grid(int64_t n) { return (unsigned)(kXcds * ((n + kXcds - 1) / kXcds)); }

// orders this wave's LDS accesses (a staged chunk is written and read by
// different lanes of the same wave).  The LDS executes one wave's
// instructions in issue order, so only the compiler must not move them
// across: wavefront-scope fences and a wave barrier, which emit no wait (an
// explicit wait here would also hold back the prefetched global loads).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x in tree order, row-major N x nrp, BF16 (columns c0 .. c0 + nc of X; the
// remaining columns zero)
template <typename XT>
__global__ void k_rows_bf16(const XT* __restrict__ X, int64_t ldx, int c0, int nc, int64_t N,
                            const int32_t* __restrict__ perm, int nrp, uint16_t* __restrict__ xr) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * nrp) return;
    const int64_t p = t / nrp;
    const int c = (int)(t - p * nrp);
    xr[t] = c < nc ? bf16_from_float((float)X[(int64_t)(c0 + c) * ldx + perm[p]]) : (uint16_t)0;
}

template <typename C>
__global__ void k_fill_zero(C* __restrict__ p, int64_t n) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) p[t] = (C)0;
}

// index of projection (term k, right-hand side c) in the BF16 projection
// layout: groups of 4 terms, then the right-hand side, then the term in the
// group (a pass-2 lane loads 4 consecutive terms of one column as 8 bytes)
__device__ __forceinline__ int64_t tidx(int64_t base, int k, int c, int nrp) {
    return base + ((int64_t)(k >> 2) * nrp + c) * 4 + (k & 3);
}

// G: 64-column groups per wave (a panel of at most 64 W G columns)
template <int W, int CT, int G = 1>
__global__ __launch_bounds__(64 * W) void k_mproj(const MJob* __restrict__ jobs, int64_t njobs,
                                                  const uint16_t* __restrict__ xr,
                                                  uint16_t* __restrict__ tproj,
                                                  float* __restrict__ part) {
    constexpr int NRP = 16 * CT;
    constexpr int KT = 2 * G;   // 32-column steps per wave
    __shared__ f32x4_t red[W > 1 ? W : 1][CT][64];
    const int64_t jx = xcd_item(njobs);
    if (jx < 0) return;   // padding of the last XCD's range (whole workgroup)
    const MJob J = jobs[jx];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int a = lane & 15, q = lane >> 4;
    const int64_t ld = fstride<bf16>(J.len);
    const int col0 = J.p0 + wv * MR * G;
    const int cend = J.p0 + J.plen;
    // Buffer loads throughout: a lane with nothing to read (column past the
    // panel, term past the rank, no next chunk) gets an offset moved past
    // the range by adding 2^31 and reads zero, so no load sits behind a
    // per-lane branch and the waits count loads exactly.
    auto rsrc = [](uint64_t base) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
    };
    // x operand (K = factor column, N = right-hand side): lane holds columns
    // col0 + 32 kt + 8 q + e (e < 8) of right-hand side 16 ct + a
    const __amdgpu_buffer_rsrc_t xrs = rsrc((uint64_t)(xr + (int64_t)J.x0 * NRP));
    bf16x8_t xs[KT][CT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            u16x8_t u;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int j = col0 + 32 * kt + 8 * q + e;
                const uint32_t off = (uint32_t)(2 * (j * NRP + 16 * ct + a)) + ((uint32_t)(j >= cend) << 31);
                u[e] = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(xrs, (int)off, 0, 0);
            }
            xs[kt][ct] = __builtin_bit_cast(bf16x8_t, u);
        }
    // factor words of a 16-term chunk: lane holds term k0 + a, columns
    // col0 + 32 kt + 8 q .. + 7
    const __amdgpu_buffer_rsrc_t frs = rsrc(J.F);
    auto load_chunk = [&](int k0, u32x4 (&w)[KT]) {
        const int k = k0 + a;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int c8 = col0 + 32 * kt + 8 * q;
            const bool ok = k < J.r && c8 < cend;
            const uint32_t off = (uint32_t)(2 * ((int64_t)k * ld + c8)) + ((uint32_t)!ok << 31);
            w[kt] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(frs, (int)off, 0, 0));
        }
    };
    auto process = [&](int k0, const u32x4 (&wc)[KT]) {
        f32x4_t t[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) t[ct] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const bf16x8_t fv = __builtin_bit_cast(bf16x8_t, wc[kt]);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                t[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fv, xs[kt][ct], t[ct], 0, 0, 0);
        }
        if (W > 1) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) red[wv][ct][lane] = t[ct];
            __syncthreads();
            if (wv == 0)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    f32x4_t v = red[0][ct][lane];
#pragma unroll
                    for (int w2 = 1; w2 < W; ++w2) v += red[w2][ct][lane];
                    t[ct] = v;
                }
            __syncthreads();
        }
        if (wv == 0) {
            // lane (a, q) holds t[term k0 + 4 q + e][rhs 16 ct + a]
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                if (J.fin) {
                    u16x4_t o;
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = bf16_from_float(t[ct][e]);
                    *reinterpret_cast<u16x4_t*>(tproj + tidx(J.out * NRP, k0 + 4 * q, 16 * ct + a, NRP)) = o;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        part[(J.out + k0 + 4 * q + e) * NRP + 16 * ct + a] = t[ct][e];
                }
            }
        }
    };
    // two register buffers in turn: the next chunk's loads are in flight
    // while the current one is multiplied (no copy between the buffers)
    u32x4 wa[KT], wb[KT];
    load_chunk(0, wa);
    for (int k0 = 0;;) {
        load_chunk(k0 + 16, wb);
        __builtin_amdgcn_sched_barrier(0);
        process(k0, wa);
        __builtin_amdgcn_sched_barrier(0);
        k0 += 16;
        if (k0 >= J.r) break;
        load_chunk(k0 + 16, wa);
        __builtin_amdgcn_sched_barrier(0);
        process(k0, wb);
        __builtin_amdgcn_sched_barrier(0);
        k0 += 16;
        if (k0 >= J.r) break;
    }
}

// projections of the blocks done in np panels: sum of the panel partials
// (layout [panel][term][rhs], r16 terms each) in panel order
__global__ void k_mreduce(const MRed* __restrict__ reds, const float* __restrict__ part, int nrp,
                          uint16_t* __restrict__ tproj) {
    const MRed R = reds[blockIdx.x];
    const int64_t per = (int64_t)R.r16 * nrp;
    const float* __restrict__ pp = part + R.part * nrp;
    for (int64_t t = threadIdx.x; t < per; t += blockDim.x) {
        float v = 0.f;
        for (int p = 0; p < R.np; ++p) v += pp[p * per + t];
        const int k = (int)(t / nrp), c = (int)(t - (int64_t)k * nrp);
        tproj[tidx(R.out * nrp, k, c, nrp)] = bf16_from_float(v);
    }
}

// One workgroup of TW waves per tile of a target box; wave w takes the rows
// [rowoff + 16 RT w, rowoff + 16 RT (w + 1)) of the tile.  With TW > 1 the
// projection chunk every wave multiplies by is loaded once by wave 0 and
// shared through LDS (one barrier per chunk, two buffers).
template <int CT, int RT, int TW>
__global__ __launch_bounds__(64 * TW, RT > 8 ? 2 : 4) void k_mexp(
    const MTile* __restrict__ tiles, const MEnt* __restrict__ ents,
    const uint16_t* __restrict__ tproj, int64_t N, int nc, float* __restrict__ yl) {
    constexpr int NRP = 16 * CT;
    constexpr int WR = 16 * RT;              // rows per wave
    constexpr int NWORD = WR / 8 * 16 / 64;  // 16-byte factor words per lane and chunk
    __shared__ __attribute__((aligned(16))) uint16_t stg[TW][16][WR + MPAD];
    __shared__ __attribute__((aligned(16))) uint16_t s_t[TW > 1 ? 2 : 1][16 * NRP];
    const MTile T = tiles[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int a = lane & 15, q = lane >> 4;
    const int64_t ld = fstride<bf16>(T.len);
    const int wrow = wv * WR;                       // first row of this wave in the tile
    const int wrows = min(WR, T.rows - wrow);       // may be <= 0 (idle wave)
    f32x4_t acc[RT][CT];
#pragma unroll
    for (int it = 0; it < RT; ++it)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[it][ct] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    // (entry, 16-term chunk) pairs in order; the loads of the next pair are
    // issued before the current one is multiplied
    // Buffer loads: a lane with nothing to load (term past the rank, row past
    // the box, or no next chunk) gets an offset past the resource's range
    // and reads zero by the hardware range check, so the loads carry no
    // per-lane branch and no select on their results; the wait before a
    // multiply then counts only that chunk's loads.  The whole offset is the
    // per-lane operand (the one the range check covers).
    auto rsrc = [](uint64_t base) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
    };
    auto load_words = [&](const MEnt& E, int k0, u32x4 (&w)[NWORD], bool valid = true) {
        const __amdgpu_buffer_rsrc_t rs = rsrc(E.F);
#pragma unroll
        for (int sI = 0; sI < NWORD; ++sI) {
            const int f = lane + 64 * sI, tt = f / (WR / 8), g = f % (WR / 8);
            const bool ok = valid && k0 + tt < E.r && 8 * g < wrows;
            // below 2^31 for any term up to r + 16 of a factor; moved past the
            // range by adding 2^31 (arithmetic, not a select the compiler
            // could turn into branches)
            const uint32_t off = (uint32_t)(2 * ((int64_t)(k0 + tt) * ld + T.rowoff + wrow + 8 * g)) +
                                 ((uint32_t)!ok << 31);
            w[sI] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
        }
    };
    // the chunk's projections, 16 terms x NRP contiguous (16-byte word per lane)
    auto load_t = [&](const MEnt& E, int k0, u32x4& tw, bool valid = true) {
        const __amdgpu_buffer_rsrc_t rs = rsrc((uint64_t)(tproj + (E.t + k0) * NRP));
        const bool ok = valid && 8 * lane < 16 * NRP;
        const uint32_t off = (uint32_t)(16 * lane) + ((uint32_t)!ok << 31);
        tw = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
    };
    // the (entry, chunk) sequence: the pair after (e, k0) of entry E
    auto advance = [&](int& ee, int& kk, MEnt& EE) {
        kk += 16;
        if (kk >= EE.r) {
            kk = 0;
            ++ee;
            while (ee < T.ne && (EE = ents[T.e0 + ee]).r <= 0) ++ee;
        }
    };
    int par = 0;
    // multiply one staged chunk (projections tw, factor words w)
    auto process = [&](const u32x4 (&w)[NWORD], const u32x4& tw) {
        // the projections as the A operand: lane (a, q) takes terms
        // k0 + 4 q .. + 3 of right-hand side 16 ct + a
        s16x4_t ta[CT];
        if (TW == 1) {
            wave_lds_fence();
            if (8 * lane < 16 * NRP) *reinterpret_cast<u32x4*>(&s_t[0][8 * lane]) = tw;
            wave_lds_fence();
        } else {
            if (wv == 0 && 8 * lane < 16 * NRP) *reinterpret_cast<u32x4*>(&s_t[par][8 * lane]) = tw;
            __syncthreads();
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            ta[ct] = __builtin_bit_cast(
                s16x4_t, *reinterpret_cast<const u16x4_t*>(&s_t[TW > 1 ? par : 0][(q * NRP + 16 * ct + a) * 4]));
        // stage this chunk of the wave's rows: 16 terms x WR/8 words
        wave_lds_fence();
#pragma unroll
        for (int sI = 0; sI < NWORD; ++sI) {
            const int f = lane + 64 * sI, tt = f / (WR / 8), g = f % (WR / 8);
            *reinterpret_cast<u32x4*>(&stg[wv][tt][8 * g]) = w[sI];
        }
        wave_lds_fence();
#pragma unroll
        for (int it = 0; it < RT; ++it) {
            if (16 * it < wrows) {
                s16x4_t up;
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) up[e2] = (short)stg[wv][4 * q + e2][16 * it + a];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
                    acc[it][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ta[ct], up, acc[it][ct], 0, 0, 0);
            }
        }
        par ^= 1;
    };
    int e = 0, k0 = 0;
    MEnt E{};
    while (e < T.ne && (E = ents[T.e0 + e]).r <= 0) ++e;
    {
        // two register buffers in turn: while one chunk is multiplied the
        // loads of the next are in flight (no copy between the buffers, which
        // would wait for those loads).  The loads are issued every time (past
        // the last chunk all lanes read zero), so the wait before a multiply
        // can count the other buffer's loads as still in flight.  With
        // several waves only wave 0 loads the projections.
        const bool ldt = TW == 1 || wv == 0;
        u32x4 wa[NWORD], ta_w, wb[NWORD], tb_w;
        load_words(E, k0, wa, e < T.ne);
        load_t(E, k0, ta_w, e < T.ne && ldt);
        for (;;) {
            if (e >= T.ne) break;
            advance(e, k0, E);   // the chunk after the one in wa
            load_words(E, k0, wb, e < T.ne);
            load_t(E, k0, tb_w, e < T.ne && ldt);
            __builtin_amdgcn_sched_barrier(0);
            process(wa, ta_w);
            __builtin_amdgcn_sched_barrier(0);
            if (e >= T.ne) break;
            advance(e, k0, E);   // the chunk after the one in wb
            load_words(E, k0, wa, e < T.ne);
            load_t(E, k0, ta_w, e < T.ne && ldt);
            __builtin_amdgcn_sched_barrier(0);
            process(wb, tb_w);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // lane (a, q) holds C[row 16 it + a][rhs 16 ct + 4 q + e]
#pragma unroll
    for (int it = 0; it < RT; ++it) {
        const int i = 16 * it + a;
        if (i < wrows)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) {
                    const int c = 16 * ct + 4 * q + e2;
                    if (c < nc) yl[(int64_t)c * N + T.row0 + wrow + i] += acc[it][ct][e2];
                }
    }
}

// One term (row of V, column of U) of a large block per workgroup: the 256
// threads stride over the row with four independent partial sums, then a
// workgroup reduction gives t_k (and s_k).
template <typename C, int NR, bool CO = false>
__device__ __forceinline__ void wg_reduce_store(C (&acc)[NR], C (*red)[NR], int nc, C* out,
                                                int64_t stride) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = wsum(acc[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NR; ++c) red[wv][c] = acc[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < nc; ++c) {
            C v = 0;
            for (int w = 0; w < TP / 64; ++w) v += red[w][c];
            stv<CO>(out + (int64_t)c * stride, v);
        }
    __syncthreads();
}

template <typename S, typename C, int NR, bool CO = false>
__device__ __forceinline__ void row_dot(gptr_t<S> row, int len,
                                        const C* __restrict__ xs, int64_t N, int nc,
                                        C (&acc)[NR]) {
    C a[4][NR];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NR; ++c) a[u][c] = 0;
    int j = threadIdx.x;
    for (; j + 3 * TP < len; j += 4 * TP) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const C v = ldf<C>(row, j + u * TP);
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nc) a[u][c] += v * ldv<CO>(xs + (int64_t)c * N + j + u * TP);
        }
    }
    for (; j < len; j += TP) {
        const C v = ldf<C>(row, j);
#pragma unroll
        for (int c = 0; c < NR; ++c)
            if (c < nc) a[0][c] += v * ldv<CO>(xs + (int64_t)c * N + j);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = (a[0][c] + a[1][c]) + (a[2][c] + a[3][c]);
}

template <typename S, typename C, int NR, bool CO = false>
__device__ __forceinline__ void project_body(const BlockDesc* __restrict__ blocks,
                                             const ProjSeg& it, int sym,
                                             const C* __restrict__ x, int64_t N, int nrhs,
                                             int c0, C* __restrict__ part, C (*red)[NR]) {
    const BlockDesc b = blocks[it.blk];
    const int nc = min(NR, nrhs - c0);
    const int k = it.k;
    C acc[NR];
    {   // t_k partial: V[k, j0:j1] x_B[j0:j1]
        const int ln = (b.n + it.nseg - 1) / it.nseg, j0 = it.seg * ln;
        const int len = max(0, min(b.n, j0 + ln) - j0);
        row_dot<S, C, NR, CO>(as_global<S>(b.V) + (int64_t)k * fstride<S>(b.n) + j0, len,
                              x + (int64_t)c0 * N + b.b0 + j0, N, nc, acc);
        wg_reduce_store<C, NR, CO>(acc, red, nc,
                               part + ((it.p * 2 + 0) * kProjSegMax + it.seg) * NR, 1);
    }
    if (sym) {   // s_k partial: U[i0:i1, k]^T x_A[i0:i1]
        const int ln = (b.m + it.nseg - 1) / it.nseg, i0 = it.seg * ln;
        const int len = max(0, min(b.m, i0 + ln) - i0);
        row_dot<S, C, NR, CO>(as_global<S>(b.U) + (int64_t)k * fstride<S>(b.m) + i0, len,
                              x + (int64_t)c0 * N + b.a0 + i0, N, nc, acc);
        wg_reduce_store<C, NR, CO>(acc, red, nc,
                               part + ((it.p * 2 + 1) * kProjSegMax + it.seg) * NR, 1);
    }
}

template <typename S, typename C, int NR>
__global__ __launch_bounds__(TP) void k_project(const BlockDesc* __restrict__ blocks,
                                                const ProjSeg* __restrict__ items, int sym,
                                                const C* __restrict__ x, int64_t N, int nrhs,
                                                int c0, C* __restrict__ part) {
    __shared__ C red[TP / 64][NR];
    project_body<S, C, NR>(blocks, items[blockIdx.x], sym, x, N, nrhs, c0, part, red);
}

// t_k (and s_k) of the segmented projections: the partials summed in segment
// order, one thread per (term, side, column)
// thread t of the nsum * 2 * NR (term, side, column) sums; part read through
// P (a plain or a device-coherent load)
template <typename C, int NR, bool CO = false, typename P>
__device__ __forceinline__ void proj_sum_body(int64_t t, const ProjSum* __restrict__ sums,
                                              int64_t nsum, int sym, int nc, P part, int64_t TT,
                                              C* __restrict__ tb, C* __restrict__ sb) {
    if (t >= nsum * 2 * NR) return;
    const int c = (int)(t % NR), side = (int)((t / NR) & 1);
    const int64_t i = t / (2 * NR);
    if (c >= nc || (side == 1 && !sym)) return;
    const ProjSum S = sums[i];
    const int64_t pp = (S.p * 2 + side) * kProjSegMax * NR + c;
    C v = 0;
    for (int g = 0; g < S.nseg; ++g) v += part(pp + (int64_t)g * NR);
    stv<CO>((side ? sb : tb) + (int64_t)c * TT + S.dst, v);
}

template <typename C, int NR>
__global__ void k_proj_sum(const ProjSum* __restrict__ sums, int64_t nsum, int sym, int nc,
                           const C* __restrict__ part, int64_t TT, C* __restrict__ tb,
                           C* __restrict__ sb) {
    proj_sum_body<C, NR>(blockIdx.x * (int64_t)256 + threadIdx.x, sums, nsum, sym, nc,
                         [part](int64_t i) { return part[i]; }, TT, tb, sb);
}

// 64-row chunk of one side of a large block: side 0 writes U t into the rows
// of A, side 1 writes V^T s into the rows of B; the 4 waves split the terms
// coefficients (t or s) read through P (a plain or a device-coherent load)
template <typename S, typename C, int NR, bool CO = false, typename P>
__device__ __forceinline__ void expand_split_body(const BlockDesc* __restrict__ blocks,
                                                  const WorkItem& it, int nrhs, int c0,
                                                  int64_t TT, P tbs, int64_t CT,
                                                  C* __restrict__ contrib, C (*part)[NR][64]) {
    const BlockDesc b = blocks[it.id];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool tr = it.level != 0;
    const gptr_t<S> W = as_global<S>(tr ? b.V : b.U);
    const int len = tr ? b.n : b.m;
    const int64_t ld = fstride<S>(len);
    const int side = tr ? 1 : 0;
    const int o = it.lo + lane;
    const bool active = lane < it.cnt;
    const int nc = min(NR, nrhs - c0);
    C acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0;
    if (active) {
        for (int k = wv; k < b.rank; k += TE / 64) {
            const C w = ldf<C>(W, (int64_t)k * ld + o);
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] += w * tbs(side, (int64_t)c * TT + b.toff + k);
        }
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) part[wv][c][lane] = acc[c];
    __syncthreads();
    if (wv == 0 && active) {
        const int64_t seg = tr ? b.cbwd : b.cfwd;
        for (int c = 0; c < nc; ++c) {
            C s = part[0][c][lane];
            for (int w = 1; w < TE / 64; ++w) s += part[w][c][lane];
            stv<CO>(contrib + (int64_t)c * CT + seg + o, s);
        }
    }
}

template <typename S, typename C, int NR>
__global__ __launch_bounds__(TE) void k_expand_split(const BlockDesc* __restrict__ blocks,
                                                     const WorkItem* __restrict__ items, int nrhs,
                                                     int c0, int64_t TT, const C* __restrict__ tb,
                                                     const C* __restrict__ sb, int64_t CT,
                                                     C* __restrict__ contrib) {
    __shared__ C part[TE / 64][NR][64];
    expand_split_body<S, C, NR>(
        blocks, items[blockIdx.x], nrhs, c0, TT,
        [tb, sb](int side, int64_t i) { return side ? sb[i] : tb[i]; }, CT, contrib, part);
}

// rows [lo, lo+cnt) of one leaf: near field on the fly plus the low-rank
// contributions of every level, written to Y in user order.  The 4 waves of
// the workgroup and, when cnt < 64, slices of lanes inside a wave split the
// sources and the contribution segments; partial sums meet in a fixed order.
// The leaf's source ranges and per-level segments are precomputed, so its
// loads do not depend on each other.
// MODE kNearFused: both, written to Y.  MODE kNearOnly: the near field alone,
// written to yn (tree order, column c at yn[c N + i]); it has no input from
// the low-rank stages and runs beside them.  MODE kGatherOnly: yn plus the
// contributions, written to Y.
constexpr int TG = 256;
constexpr int kNearTile = 256;         // sources per LDS tile
constexpr int kNearTileRanges = 1024;  // near boxes a tiled leaf may have
constexpr int kNearFused = 0, kNearOnly = 1, kGatherOnly = 2;

// one LDS record per near-field source: its coordinates, and for d <= 3 with
// one right-hand side its x value in the fourth slot
template <typename C>
struct alignas(4 * sizeof(C)) NearRec {
    C v[4];
};
// the near-field body's LDS (one set per kernel, shared by every
// instantiation of the body inside it)
template <typename C, int NR>
struct NearLds {
    int pre[kNearTileRanges + 1];
    int rs[kNearTileRanges];
    NearRec<C> pt[kNearTile];
    C x[NR][kNearTile];
};

// One item (rows of one leaf) of the near-field / gather kernel below.  CO:
// read data that other workgroups of the same launch produced (x, the
// contributions, the near sums) with device-coherent loads.
template <typename XT, typename C, int NR, int KIND, int MODE, bool CO = false>
__device__ __forceinline__ void gather_near_item(
    const NearItem& it, const SegRef* __restrict__ lseg,
    const int2* __restrict__ nrng, int kappa, const double* __restrict__ pts, int64_t N, int d,
    KParams kp, const C* x, const C* contrib, int64_t CT,
    const int32_t* __restrict__ perm, int nrhs, int c0, XT* __restrict__ Y, int64_t ldy,
    const C* __restrict__ ylev, C* yn, C (*red)[NR][64], NearLds<C, NR>& L) {
    auto ldx = [&](int64_t i) -> C { return ldv<CO>(x + i); };
    auto ldc = [&](const C* p) -> C { return ldv<CO>(p); };
    {
        // the wave index as a scalar: loop bounds built from it stay wave-uniform
        const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        int mp = 1;
        while (mp < it.cnt) mp <<= 1;
        const int S = 64 / mp;
        const int t = lane % mp;
        const int sg = wv * S + lane / mp;     // slice of this lane
        const int SG = (TG / 64) * S;          // slices in the workgroup
        const bool active = t < it.cnt;
        const int64_t i = it.lo + t;
        const int nc = min(NR, nrhs - c0);
        C acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = 0;
        double xi[kMaxD];
        if (MODE != kGatherOnly && active)
            for (int a = 0; a < d; ++a) xi[a] = pts[a * N + i];
        if constexpr (MODE == kGatherOnly) {
            if (active && sg == 0)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nc) acc[c] = ldc(yn + (int64_t)c * N + i);
        } else if (d <= 4 && it.nn <= kNearTileRanges) {
            // sources staged through LDS in tiles: coalesced cooperative loads,
            // then every lane reads them as broadcasts
            int* s_pre = L.pre;
            int* s_rs = L.rs;
            using C4 = NearRec<C>;
            C4* s_pt = L.pt;
            C (*s_x)[kNearTile] = L.x;
            const bool packx = NR == 1 && d <= 3;
            // coordinates in the compute type: FP64 as they are; FP32 relative to
            // the leaf's first point, so that differences of nearby points keep
            // their relative accuracy (zero beyond d)
            double ref[4];
            C xc[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                ref[a] = (sizeof(C) == 4 && a < d) ? pts[a * N + it.leaf0] : 0.0;
                xc[a] = (active && a < d) ? (C)(xi[a] - ref[a]) : (C)0;
            }
            for (int e = threadIdx.x; e < it.nn; e += TG) {
                const int2 rg = nrng[it.nb0 + e];
                s_rs[e] = rg.x;
                s_pre[e] = rg.y - rg.x;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int a = 0;
                for (int e = 0; e < it.nn; ++e) {
                    const int len = s_pre[e];
                    s_pre[e] = a;
                    a += len;
                }
                s_pre[it.nn] = a;
            }
            __syncthreads();
            const int total = s_pre[it.nn];
            // the row's own point as a position in the concatenated sources (its
            // leaf is one of the near ranges): the diagonal entry is found by
            // position, without a per-source index
            int qself = -1;
            if (active)
                for (int e = 0; e < it.nn; ++e) {
                    const int64_t rs = s_rs[e];
                    if (i >= rs && i < rs + (s_pre[e + 1] - s_pre[e])) qself = s_pre[e] + (int)(i - rs);
                }
            // A lane takes sources sg, sg + SG, ... of the tile.  The wave walks
            // the tile with one trip count for all of its lanes (they differ
            // only by their slice within the wave), so the loop has no per-lane
            // exit and the diagonal is a select; the last, partly filled step
            // reads a valid record and drops its term.
            const int sl = lane / mp;
            auto tile = [&](int t0, int tn, auto packed) {
                constexpr bool P = decltype(packed)::value;
                const int qs = qself - t0;
                auto term = [&](int q, bool ok) {
                    const C4 pq = s_pt[q];
                    C r2 = 0;
#pragma unroll
                    for (int a = 0; a < (P ? 3 : 4); ++a) {
                        const C dx = xc[a] - pq.v[a];
                        r2 += dx * dx;
                    }
                    C kij = kfun_k<KIND>(kp, r2);
                    kij = q == qs ? (C)kp.diag : kij;
                    kij = ok ? kij : (C)0;
                    if constexpr (P) {
                        acc[0] += kij * pq.v[3];
                    } else {
#pragma unroll
                        for (int c = 0; c < NR; ++c) acc[c] += kij * s_x[c][q];
                    }
                };
                int q0 = wv * S;
                for (; q0 + 3 * SG + S <= tn; q0 += 4 * SG) {   // four records read at once
#pragma unroll
                    for (int u = 0; u < 4; ++u) term(q0 + u * SG + sl, true);
                }
                for (; q0 + S <= tn; q0 += SG) term(q0 + sl, true);
                if (q0 < tn) {
                    const bool ok = q0 + sl < tn;
                    term(ok ? q0 + sl : tn - 1, ok);
                }
            };
            for (int t0 = 0; t0 < total; t0 += kNearTile) {
                const int tn = min(kNearTile, total - t0);
                for (int q = threadIdx.x; q < tn; q += TG) {
                    const int sidx = t0 + q;
                    int lo = 0, hi = it.nn - 1;   // last range starting at or before sidx
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= sidx)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    const int j = s_rs[lo] + (sidx - s_pre[lo]);
                    C4 pq;
#pragma unroll
                    for (int a = 0; a < 4; ++a) pq.v[a] = a < d ? (C)(pts[a * N + j] - ref[a]) : (C)0;
                    if (packx) {
                        pq.v[3] = ldx((int64_t)c0 * N + j);
                    } else {
#pragma unroll
                        for (int c = 0; c < NR; ++c) s_x[c][q] = c < nc ? ldx((int64_t)(c0 + c) * N + j) : (C)0;
                    }
                    s_pt[q] = pq;
                }
                __syncthreads();
                // every lane runs the tile (idle rows have zero coordinates and
                // their sums are dropped), so the wave stays converged
                if (packx)
                    tile(t0, tn, std::true_type{});
                else
                    tile(t0, tn, std::false_type{});
                __syncthreads();
            }
        } else if (active) {
            for (int e = 0; e < it.nn; ++e) {
                const int2 rg = nrng[it.nb0 + e];
                for (int64_t j = rg.x + sg; j < rg.y; j += SG) {
                    C kij;
                    if (j == i) {
                        kij = (C)kp.diag;
                    } else {
                        C r2 = 0;
                        for (int a = 0; a < d; ++a) {
                            const C dx = (C)(xi[a] - pts[a * N + j]);
                            r2 += dx * dx;
                        }
                        kij = kfun_k<KIND>(kp, r2);
                    }
#pragma unroll
                    for (int c = 0; c < NR; ++c)
                        if (c < nc) acc[c] += kij * ldx((int64_t)(c0 + c) * N + j);
                }
            }
        }
        if constexpr (MODE != kNearOnly) {
            if (active && ylev) {
                // the low-rank part is already summed per row (columns c0 .. c0+nc)
                if (sg == 0)
#pragma unroll
                    for (int c = 0; c < NR; ++c)
                        if (c < nc) acc[c] += ylev[(int64_t)c * N + i];
            } else if (active) {
                const int64_t off = i - it.leaf0;
                for (int l = 0; l < kappa; ++l) {
                    const SegRef sr = lseg[(int64_t)it.leaf * kappa + l];
                    const C* seg = contrib + sr.base + off;
#pragma unroll 4
                    for (int64_t e = sg; e < sr.ne; e += SG)
#pragma unroll
                        for (int c = 0; c < NR; ++c)
                            if (c < nc) acc[c] += ldc(seg + (int64_t)c * CT + e * sr.len);
                }
            }
        }
        for (int o = mp; o < 64; o <<= 1)
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
#pragma unroll
        for (int c = 0; c < NR; ++c) red[wv][c][lane] = acc[c];
        __syncthreads();
        if (wv == 0 && active && lane < mp) {
            for (int c = 0; c < nc; ++c) {
                C v = red[0][c][lane];
                for (int w = 1; w < TG / 64; ++w) v += red[w][c][lane];
                if constexpr (MODE == kNearOnly)
                    stv<CO>(yn + (int64_t)c * N + i, v);
                else
                    Y[(int64_t)(c0 + c) * ldy + perm[i]] = (XT)v;
            }
        }
        __syncthreads();   // LDS is reused by the next item
    }
}

template <typename XT, typename C, int NR, int KIND = -1, int MODE = kNearFused>
__global__ __launch_bounds__(TG) void k_gather_near(
    const NearItem* __restrict__ items, int64_t nitems, const SegRef* __restrict__ lseg,
    const int2* __restrict__ nrng, int kappa, const double* __restrict__ pts, int64_t N, int d,
    KParams kp, const C* __restrict__ x, const C* __restrict__ contrib, int64_t CT,
    const int32_t* __restrict__ perm, int nrhs, int c0, XT* __restrict__ Y, int64_t ldy,
    const C* __restrict__ ylev, C* __restrict__ yn) {
    __shared__ C red[TG / 64][NR][64];
    __shared__ NearLds<C, NR> lds;
    // a grid smaller than the item count loops over the items: a capped grid
    // keeps the kernel to a share of every CU while it runs beside others
    for (int64_t bi = blockIdx.x; bi < nitems; bi += gridDim.x)
        gather_near_item<XT, C, NR, KIND, MODE>(items[bi], lseg, nrng, kappa, pts, N, d, kp, x,
                                                contrib, CT, perm, nrhs, c0, Y, ldy, ylev, yn,
                                                red, lds);
}

// Skeleton form (eqs. keq1/keq2): a stored block is its ACA pivots sigma
// (rows of A), tau (columns of B) and the LU of K(sigma, tau) (L on and below
// the diagonal, unit upper above), and
//   K~(A,B) x_B = K(A, tau) U^-1 L^-1 K(sigma, B) x_B,
//   K~(A,B)^T x_A = K(B, sigma) L^-T U^-T K(tau, A) x_A   (symmetric kernel).
// Three launches over all stored blocks: the skeleton projections
// w = K(sigma, B) x_B and w' = K(tau, A) x_A in source segments of up to
// kSkelSeg points (many workgroups per large block, partial sums), one
// workgroup per block summing the partials and solving the two triangular
// pairs in panels of 32 (panel updates by the whole workgroup, the 32 x 32
// diagonal blocks from LDS by one wave each), then the expansions
// K(A, tau) z and K(B, sigma) s in 256-row chunks.  The kernel matrices are
// evaluated on the fly in every launch.
constexpr int kSkelMaxR = 1024;   // largest rank of a block in the skeleton form

// out[k] = sum_j K(p_k, q_j) w_j for k < nt, targets p_k = pts[tidx(k)],
// sources q_j = pts[sidx(j)] with weights wfn(j).  Targets and sources are
// points of two different boxes (a stored block is never a box with itself),
// so no pair is a diagonal entry.  The sources are staged through LDS 256 at
// a time by the whole workgroup, for d <= 3 as one 32-byte record (three
// coordinates, zero beyond d, and the weight: two LDS reads a pair), else
// coordinate by coordinate; g threads share a target and split each tile,
// their partial sums reduced in the group.  Every thread of the workgroup
// must call it.
constexpr int kSkelTile = 256;

template <bool P3>
struct SkelLds {                        // d <= 3: x, y, z, weight per source
    alignas(16) double rec[kSkelTile][4];
};
template <>
struct SkelLds<false> {                 // d > 3: coordinates and weights
    double q[kMaxD][kSkelTile];
    double w[kSkelTile];
};

template <typename C, int KIND, bool P3, typename TI, typename SI, typename WF, typename OF>
__device__ __forceinline__ void skel_products(const double* __restrict__ pts, int64_t N, int d,
                                              const KParams& kp, int nt, TI tidx, int ns,
                                              SI sidx, WF wfn, OF ofn, SkelLds<P3>& L) {
    int g = 1;
    while (g < 64 && g * 2 * nt <= (int)blockDim.x) g *= 2;
    const int per = blockDim.x / g;
    const int sub = threadIdx.x & (g - 1);
    for (int k0 = 0; k0 < nt; k0 += per) {
        const int k = k0 + (int)threadIdx.x / g;
        const bool act = k < nt;
        double xt[kMaxD];
        for (int a = 0; a < kMaxD; ++a) xt[a] = 0.0;
        if (act) {
            const int64_t tp = tidx(k);
            for (int a = 0; a < d; ++a) xt[a] = pts[a * N + tp];
        }
        C acc = 0;
        for (int j0 = 0; j0 < ns; j0 += kSkelTile) {
            const int tn = min(kSkelTile, ns - j0);
            __syncthreads();   // the previous tile is no longer read
            for (int q = threadIdx.x; q < tn; q += blockDim.x) {
                const int64_t sp = sidx(j0 + q);
                if constexpr (P3) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) L.rec[q][a] = a < d ? pts[a * N + sp] : 0.0;
                    L.rec[q][3] = (double)wfn(j0 + q);
                } else {
                    for (int a = 0; a < d; ++a) L.q[a][q] = pts[a * N + sp];
                    L.w[q] = (double)wfn(j0 + q);
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll 4
                for (int q = sub; q < tn; q += g) {
                    C r2 = 0, wq;
                    if constexpr (P3) {
                        const double4 R = *reinterpret_cast<const double4*>(L.rec[q]);
                        const C dx = (C)(xt[0] - R.x), dy = (C)(xt[1] - R.y),
                                dz = (C)(xt[2] - R.z);
                        r2 = dx * dx + dy * dy + dz * dz;
                        wq = (C)R.w;
                    } else {
                        for (int a = 0; a < d; ++a) {
                            const C dx = (C)(xt[a] - L.q[a][q]);
                            r2 += dx * dx;
                        }
                        wq = (C)L.w[q];
                    }
                    acc += kfun_k<KIND>(kp, r2) * wq;
                }
            }
        }
        for (int o = g / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (act && sub == 0) ofn(k, acc);
    }
}

constexpr int kSkelSeg = 4096;      // sources per projection item
constexpr int kSkelRows = 256;      // rows per expansion item

template <typename S, typename C, int KIND, bool P3>
__global__ __launch_bounds__(256) void k_skel_proj(const BlockDesc* __restrict__ blocks,
                                                   const SkelProj* __restrict__ items,
                                                   const double* __restrict__ pts, int64_t N,
                                                   int d, KParams kp, const C* __restrict__ x,
                                                   C* __restrict__ part) {
    __shared__ SkelLds<P3> L;
    const SkelProj it = items[blockIdx.x];
    const BlockDesc b = blocks[it.blk];
    const int32_t* __restrict__ sig = reinterpret_cast<const int32_t*>(b.V);
    const int32_t* __restrict__ tau = sig + b.rank;
    C* out = part + it.dst;
    if (it.side == 0)   // w += K(sigma, B[lo, lo + cnt)) x_B
        skel_products<C, KIND, P3>(
            pts, N, d, kp, b.rank, [&](int k) { return (int64_t)b.a0 + sig[k]; }, it.cnt,
            [&](int j) { return (int64_t)b.b0 + it.lo + j; },
            [&](int j) { return x[b.b0 + it.lo + j]; }, [&](int k, C v) { out[k] = v; }, L);
    else                // w' += K(tau, A[lo, lo + cnt)) x_A
        skel_products<C, KIND, P3>(
            pts, N, d, kp, b.rank, [&](int k) { return (int64_t)b.b0 + tau[k]; }, it.cnt,
            [&](int i) { return (int64_t)b.a0 + it.lo + i; },
            [&](int i) { return x[b.a0 + it.lo + i]; }, [&](int k, C v) { out[k] = v; }, L);
}

constexpr int kSkelPanel = 32;   // rows of a triangular panel (lanes of one wave)
constexpr int kSkelSolveThreads = 128;

// s[i] -= sum_{k0 <= k < k1} M[i][k] s[k] for i0 <= i < i1 (rows of the
// row-major r x r array M): a wave per row, lanes over k; each wave takes
// four rows at a time so that their loads are in flight together (the
// solve is a chain of such steps: their latency is its cost)
template <typename S, typename C>
__device__ __forceinline__ void skel_row_update(gptr_t<S> M, int r, C* s, int i0, int i1,
                                                int k0, int k1) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = i0 + wv; i < i1; i += 4 * nw) {
        C a[4] = {0, 0, 0, 0};
        for (int k = k0 + lane; k < k1; k += 64) {
            const C sk = s[k];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + u * nw < i1) a[u] += ldf<C>(M, (int64_t)(i + u * nw) * r + k) * sk;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const C v = wsum(a[u]);
            if (lane == 0 && i + u * nw < i1) s[i + u * nw] -= v;
        }
    }
    __syncthreads();
}

// s[i0 + t] -= sum_{k0 <= k < k1} M[k][i0 + t] s[k] for t < pb (columns of
// M): lanes over t, the waves split k, partials met in LDS
template <typename S, typename C>
__device__ __forceinline__ void skel_col_update(gptr_t<S> M, int r, C* s, int i0, int pb,
                                                int k0, int k1, C (*red)[64]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    C a = 0;
    if (lane < pb) {
#pragma unroll 8
        for (int k = k0 + wv; k < k1; k += nw) a += ldf<C>(M, (int64_t)k * r + i0 + lane) * s[k];
    }
    red[wv][lane] = a;
    __syncthreads();
    if (wv == 0 && lane < pb) {
        C t = 0;
        for (int w = 0; w < nw; ++w) t += red[w][lane];
        s[i0 + lane] -= t;
    }
    __syncthreads();
}

// the diagonal block M[p .. p+pb)^2 into LDS (D[i][k], rows padded, zero
// past pb) and the reciprocals of its diagonal
template <typename S, typename C>
__device__ __forceinline__ void skel_stage_diag(gptr_t<S> M, int r, int p, int pb, C (*D)[kSkelPanel + 1],
                                                C* rd) {
    // every load issued before the first store (a loop would wait for each)
    constexpr int kU = kSkelPanel * kSkelPanel / kSkelSolveThreads;
    C v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int e = threadIdx.x + u * kSkelSolveThreads;
        const int i = e / kSkelPanel, k = e % kSkelPanel;
        v[u] = (i < pb && k < pb) ? ldf<C>(M, (int64_t)(p + i) * r + p + k) : (C)0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int e = threadIdx.x + u * kSkelSolveThreads;
        D[e / kSkelPanel][e % kSkelPanel] = v[u];
    }
    __syncthreads();
    if (threadIdx.x < kSkelPanel)
        rd[threadIdx.x] = threadIdx.x < pb ? (C)1 / D[threadIdx.x][threadIdx.x] : (C)0;
    __syncthreads();
}

// lane k's value, as a scalar
__device__ __forceinline__ double lane_value(double v, int k) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_value(float v, int k) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

// Solve of one diagonal block by the calling wave, lane t holding entry
// p + t of s.  TR: the block is used transposed; LOWER: forward elimination
// (else backward); UNIT: unit diagonal (else the reciprocals rd).
template <typename C, bool TR, bool LOWER, bool UNIT>
__device__ __forceinline__ void skel_diag_solve(C* s, int p, int pb, const C (*D)[kSkelPanel + 1],
                                                const C* rd) {
    const int lane = threadIdx.x & 63;
    C w = lane < pb ? s[p + lane] : (C)0;
    for (int t = 0; t < pb; ++t) {
        const int k = LOWER ? t : pb - 1 - t;
        C zk = lane_value(w, k);
        if (!UNIT) zk *= rd[k];
        const bool later = LOWER ? lane > k : lane < k;
        if (lane == k)
            w = zk;
        else if (later && lane < pb)
            w -= (TR ? D[k][lane] : D[lane][k]) * zk;
    }
    if (lane < pb) s[p + lane] = w;
}

// one workgroup per stored block: the skeleton projections summed over their
// segments, then z = U^-1 L^-1 w and (symmetric kernel) s = L^-T U^-T w', in
// panels of kSkelPanel: the panel updates by the whole workgroup (two
// waves, so that many blocks are solved on a CU at once), then the diagonal
// block (staged once for both systems, which use its two triangles) solved
// by wave 0 for z and wave 1 for s at the same time; written to the block's
// terms of tb (and sb).  LDS: z and s of maxr values each (dynamic).
template <typename S, typename C>
__global__ __launch_bounds__(kSkelSolveThreads) void k_skel_solve(const BlockDesc* __restrict__ blocks,
                                                    const SkelSolve* __restrict__ solves, int sym,
                                                    const C* __restrict__ part,
                                                    C* __restrict__ tb, C* __restrict__ sb) {
    extern __shared__ double dyn_lds[];
    __shared__ C D[kSkelPanel][kSkelPanel + 1];
    __shared__ C rd[kSkelPanel];
    __shared__ C red[kSkelSolveThreads / 64][64];
    const BlockDesc b = blocks[blockIdx.x];
    const int r = b.rank;
    if (r <= 0) return;
    C* s_f = reinterpret_cast<C*>(dyn_lds);
    C* s_t = s_f + r;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const SkelSolve q = solves[blockIdx.x];
    const gptr_t<S> M = as_global<S>(b.U);
    for (int k = threadIdx.x; k < r; k += blockDim.x) {
        C a = 0, a2 = 0;
        for (int g = 0; g < q.nsf; ++g) a += part[q.pf + (int64_t)g * r + k];
        s_f[k] = a;
        if (sym) {
            for (int g = 0; g < q.nsb; ++g) a2 += part[q.pb + (int64_t)g * r + k];
            s_t[k] = a2;
        }
    }
    __syncthreads();
    // forward: L z1 = w and U^T s1 = w'
    int staged = -1;
    for (int p = 0; p < r; p += kSkelPanel) {
        const int pb = min(kSkelPanel, r - p);
        if (p) {
            skel_row_update<S, C>(M, r, s_f, p, p + pb, 0, p);
            if (sym) skel_col_update<S, C>(M, r, s_t, p, pb, 0, p, red);
        }
        skel_stage_diag<S, C>(M, r, p, pb, D, rd);
        staged = p;
        if (wv == 0) skel_diag_solve<C, false, true, false>(s_f, p, pb, D, rd);
        if (wv == 1 && sym) skel_diag_solve<C, true, true, true>(s_t, p, pb, D, rd);
        __syncthreads();
    }
    // backward: U z = z1 and L^T s = s1
    for (int p = ((r - 1) / kSkelPanel) * kSkelPanel; p >= 0; p -= kSkelPanel) {
        const int pb = min(kSkelPanel, r - p);
        if (p + pb < r) {
            skel_row_update<S, C>(M, r, s_f, p, p + pb, p + pb, r);
            if (sym) skel_col_update<S, C>(M, r, s_t, p, pb, p + pb, r, red);
        }
        if (p != staged) {
            skel_stage_diag<S, C>(M, r, p, pb, D, rd);
            staged = p;
        }
        if (wv == 0) skel_diag_solve<C, false, false, true>(s_f, p, pb, D, rd);
        if (wv == 1 && sym) skel_diag_solve<C, true, false, false>(s_t, p, pb, D, rd);
        __syncthreads();
    }
    for (int k = threadIdx.x; k < r; k += blockDim.x) {
        tb[b.toff + k] = s_f[k];
        if (sym) sb[b.toff + k] = s_t[k];
    }
}

// c_A = K(A, tau) z (side 0) or c_B = K(B, sigma) s (side 1) on rows
// [lo, lo + cnt) of the block's target box
template <typename S, typename C, int KIND, bool P3>
__global__ __launch_bounds__(256) void k_skel_exp(const BlockDesc* __restrict__ blocks,
                                                  const WorkItem* __restrict__ items,
                                                  const double* __restrict__ pts, int64_t N,
                                                  int d, KParams kp, const C* __restrict__ tb,
                                                  const C* __restrict__ sb,
                                                  C* __restrict__ contrib) {
    __shared__ SkelLds<P3> L;
    const WorkItem it = items[blockIdx.x];
    const BlockDesc b = blocks[it.id];
    const int32_t* __restrict__ sig = reinterpret_cast<const int32_t*>(b.V);
    const int32_t* __restrict__ tau = sig + b.rank;
    if (it.level == 0)
        skel_products<C, KIND, P3>(
            pts, N, d, kp, it.cnt, [&](int i) { return (int64_t)b.a0 + it.lo + i; }, b.rank,
            [&](int k) { return (int64_t)b.b0 + tau[k]; }, [&](int k) { return tb[b.toff + k]; },
            [&](int i, C v) { contrib[b.cfwd + it.lo + i] = v; }, L);
    else
        skel_products<C, KIND, P3>(
            pts, N, d, kp, it.cnt, [&](int j) { return (int64_t)b.b0 + it.lo + j; }, b.rank,
            [&](int k) { return (int64_t)b.a0 + sig[k]; }, [&](int k) { return sb[b.toff + k]; },
            [&](int j, C v) { contrib[b.cbwd + it.lo + j] = v; }, L);
}

// Near field on matrix cores (BF16 factors, several right-hand sides):
// y_A += K(A, near(A)) x, K evaluated on the fly in FP32 and rounded to BF16,
// times x in BF16, FP32 accumulation.  One workgroup of 4 waves per 64-row
// chunk of a leaf; the sources are staged through LDS 128 at a time
// (coordinates, and x rows in the operand layout) and each wave multiplies
// all 64 targets by 32 of them: 4 x CT 16x16x32 products per wave and tile.
// The waves' partial sums meet in LDS in wave order and are written to the
// near sums yn (tree order): the kernel needs nothing from the low-rank
// passes and runs beside them.  The kernel function (KIND) and the number of coordinates (DC = 3 for d <= 3,
// 4 for d = 4) are fixed at compile time; padded sources sit at a far
// sentinel point with x = 0 (finite kernel values times zero) and padded
// target rows are computed but never written, so the pair loop carries no
// masks; K rounds to BF16 with the hardware conversion (nearest even).
constexpr int kNmTile = 128;
constexpr float kNmFar = 1e18f;   // sentinel coordinate of padded sources

template <int CT, int KIND, int DC>
__global__ __launch_bounds__(256) void k_near_mfma(
    const NearItem* __restrict__ items, int64_t nitems, const int2* __restrict__ nrng,
    const double* __restrict__ pts, int64_t N, int d, KParams kp,
    const uint16_t* __restrict__ xr, int nc, float* __restrict__ yn) {
    constexpr int NRP = 16 * CT;
    __shared__ int s_pre[kNearTileRanges + 1], s_rs[kNearTileRanges];
    __shared__ __attribute__((aligned(16))) int s_j[kNmTile];
    __shared__ __attribute__((aligned(16))) float s_pt[4][kNmTile];
    __shared__ __attribute__((aligned(16))) uint16_t s_x[kNmTile / 8][NRP][8];
    __shared__ f32x4_t red[4][4][CT][64];
    // a grid smaller than the item count loops over the items: a capped grid
    // keeps the kernel to a share of every CU while it runs beside others
    for (int64_t bi = blockIdx.x; bi < nitems; bi += gridDim.x) {
        const NearItem it = items[bi];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int a = lane & 15, q = lane >> 4;
        // target coordinates (d <= 4, zero padded): target tile tm, row
        // it.lo + 16 tm + a
        float xt[4][4];
        int ti[4];
#pragma unroll
        for (int tm = 0; tm < 4; ++tm) {
            const int o = 16 * tm + a;
            ti[tm] = o < it.cnt ? it.lo + o : -1;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                xt[tm][c] = (ti[tm] >= 0 && c < d) ? (float)pts[c * N + ti[tm]] : 0.f;
        }
        for (int e = threadIdx.x; e < it.nn; e += 256) {
            const int2 rg = nrng[it.nb0 + e];
            s_rs[e] = rg.x;
            s_pre[e] = rg.y - rg.x;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int e = 0; e < it.nn; ++e) {
                const int len = s_pre[e];
                s_pre[e] = acc;
                acc += len;
            }
            s_pre[it.nn] = acc;
        }
        __syncthreads();
        const int total = s_pre[it.nn];
        f32x4_t acc[4][CT];
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[tm][ct] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        for (int t0 = 0; t0 < total; t0 += kNmTile) {
            const int tn = min(kNmTile, total - t0);
            // stage the tile: source index, coordinates, x rows (zero past tn)
            for (int sI = threadIdx.x; sI < kNmTile; sI += 256) {
                int j = -1;
                if (sI < tn) {
                    const int sidx = t0 + sI;
                    int lo = 0, hi = it.nn - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= sidx)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    j = s_rs[lo] + (sidx - s_pre[lo]);
                }
                s_j[sI] = j;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    s_pt[c][sI] = j < 0 ? kNmFar : c < d ? (float)pts[c * N + j] : 0.f;
            }
            __syncthreads();
            for (int f = threadIdx.x; f < kNmTile * NRP; f += 256) {
                const int sI = f / NRP, c = f - sI * NRP;
                const int j = s_j[sI];
                s_x[sI >> 3][c][sI & 7] = j >= 0 ? xr[(int64_t)j * NRP + c] : (uint16_t)0;
            }
            __syncthreads();
            // this wave: sources 32 wv + 8 q + e of the tile
            bf16x8_t xb[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                xb[ct] = __builtin_bit_cast(bf16x8_t,
                                            *reinterpret_cast<const u16x8_t*>(&s_x[4 * wv + q][16 * ct + a][0]));
            // this lane's 8 sources: indices and coordinates, read once per tile
            const int sb0 = 32 * wv + 8 * q;
            int sj[8];
            float sp[4][8];
            {
                const int4 j0 = *reinterpret_cast<const int4*>(&s_j[sb0]);
                const int4 j1 = *reinterpret_cast<const int4*>(&s_j[sb0 + 4]);
                sj[0] = j0.x; sj[1] = j0.y; sj[2] = j0.z; sj[3] = j0.w;
                sj[4] = j1.x; sj[5] = j1.y; sj[6] = j1.z; sj[7] = j1.w;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float4 p0 = *reinterpret_cast<const float4*>(&s_pt[c][sb0]);
                    const float4 p1 = *reinterpret_cast<const float4*>(&s_pt[c][sb0 + 4]);
                    sp[c][0] = p0.x; sp[c][1] = p0.y; sp[c][2] = p0.z; sp[c][3] = p0.w;
                    sp[c][4] = p1.x; sp[c][5] = p1.y; sp[c][6] = p1.z; sp[c][7] = p1.w;
                }
            }
#pragma unroll
            for (int tm = 0; tm < 4; ++tm) {
                if (16 * tm >= it.cnt) break;   // 16-row target tiles past the chunk's rows
                bf16x8_t ka;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float r2 = 0.f;
#pragma unroll
                    for (int c = 0; c < DC; ++c) {
                        const float dx = xt[tm][c] - sp[c][e];
                        r2 += dx * dx;
                    }
                    const float kij = sj[e] == ti[tm] ? (float)kp.diag : kfun_k<KIND>(kp, r2);
                    ka[e] = (__bf16)kij;
                }
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
                    acc[tm][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka, xb[ct], acc[tm][ct], 0, 0, 0);
            }
            __syncthreads();
        }
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) red[wv][tm][ct][lane] = acc[tm][ct];
        __syncthreads();
        // wave tm writes target tile tm: lane (a, q) holds rows 16 tm + 4 q + e,
        // right-hand side 16 ct + a
        {
            const int tm = wv;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                f32x4_t v = red[0][tm][ct][lane];
#pragma unroll
                for (int w2 = 1; w2 < 4; ++w2) v += red[w2][tm][ct][lane];
                const int c = 16 * ct + a;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int o = 16 * tm + 4 * q + e;
                    if (o < it.cnt && c < nc) {
                        const int64_t i = it.lo + o;
                        yn[(int64_t)c * N + i] = v[e];
                    }
                }
            }
        }
        __syncthreads();   // LDS is reused by the next item
    }
}

// ---------------------------------------------------------------------------
// Persistent product: one launch runs every stage of the products of one or
// more handles ("slots") by walking an ordered queue of claims.
//
// The host lists segments in stage order: the permutation into tree order,
// then per batch of NR columns the low-rank blocks of every class with the
// segmented projections and the near field, the sums of the segmented
// projections, their expansions, and the gather to Y.  A workgroup claims
// the next claim index with one atomic add; the claim names a segment and a
// few items in it.  Before working on it the workgroup waits until every
// claim of the earlier stages has completed, counted by a single completion
// counter: claims are handed out in order and a claim of stage p completes
// only after all claims of earlier stages did, so "completed claims >= first
// claim of stage p" holds exactly when the earlier stages are done.  A
// waiting workgroup only waits on claims handed out before its own, which
// running workgroups hold, so the queue drains whatever the grid.  The wait
// is bounded (an error flag instead of a hang).  Writes are released at
// device scope before a claim is counted and acquired after a wait, and
// values written inside the launch are read back through device-coherent
// loads.  The last workgroup to leave resets the counters for the next
// launch, so no clearing launch precedes it.
// ---------------------------------------------------------------------------
enum PKind : int32_t {
    PK_PERM = 0,   // x = X[perm], 256 rows of every column per item
    PK_G8,         // class 0: 32 blocks per claim (groups of 8 lanes)
    PK_G16,        // class 1: 16 blocks per claim
    PK_S2,         // class 2: one block per wave
    PK_S3,         // class 3: one block per wave
    PK_S4,         // class 4: one block per claim
    PK_S5,         // (unused: class-5 blocks take the segmented route)
    PK_FUSED,      // NR > 1: any class, one block per wave
    PK_PROJ,       // segmented projections
    PK_NEAR,       // near field of a 64-row leaf chunk, into the near sums
    PK_PSUM,       // sums of the segmented projections, 256 per claim
    PK_EXP,        // 64-row expansion of a segmented block
    PK_GATHER,     // near sums plus contributions of a leaf chunk, to Y
};

struct PSlot {
    const BlockDesc* cblk;   // persistent class order
    const BlockDesc* blocks;
    const ProjSeg* proj;
    const ProjSum* psum;
    const WorkItem* ex;
    const NearItem* near;
    const SegRef* lseg;
    const int2* nrng;
    const double* pts;
    const int32_t* perm;
    const void* X;
    void* Y;
    void* x;
    void* contrib;
    void* tb;
    void* sb;
    void* pp;
    void* yn;
    KParams kp;
    int64_t N, ldx, ldy, CT, TT, npsum;
    int32_t d, kappa, sym, nrhs;
};

struct PSeg {
    int64_t claim0;        // first claim index of the segment
    int64_t first, nitems; // items [first, first + nitems) of the slot's table
    int32_t slot, kind, c0, per;
    int32_t stage, ndep;   // its stage; the stages it needs complete
    int32_t dep[3], dcnt[3];   // their ids and claim counts
};
// Launch counters, each group on 128-byte lines of its own (hundreds of
// workgroups poll them, and the polls of one line queue with every other
// access to it): the claim and exit counts; the error flag and three
// diagnostics; one completion count per stage.
constexpr int kPersistLine = 32;   // ints per line
constexpr int kPersistAbort = kPersistLine;
constexpr int kPersistCtrBase = 2 * kPersistLine;
constexpr int kPersistMaxStages = 1024;
constexpr int kPersistCtrInts = kPersistCtrBase + kPersistLine * kPersistMaxStages;
// right-hand sides one persistent launch takes (five stages per batch of
// eight columns, and the permutation)
constexpr int kPersistMaxCols = 8 * ((kPersistMaxStages - 1) / 5);

constexpr int kPersistThreads = 256;
constexpr int kPersistFusedRank = 64;       // projections one wave keeps in LDS at once
// longest wait of one claim for the earlier stages: 1 s of the 100 MHz
// constant-rate clock
constexpr uint64_t kPersistWaitTicks = 100000000ull;

// a value every lane holds alike, as a scalar: the compiler then treats the
// branches that depend on it as uniform, so the barriers inside them are
// executed by every wave alike
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// waves per SIMD the persistent kernel is compiled for: FP64 factors need
// about 250 registers a lane without spilling (two waves), FP32 about 170
// (three)
template <typename S>
constexpr int persist_waves() {
    return sizeof(S) == 8 ? 2 : 3;
}

template <typename XT, typename S, int NR>
__global__ __launch_bounds__(kPersistThreads, persist_waves<S>()) void k_persist(const PSlot* __restrict__ slots,
                                                             const PSeg* __restrict__ segs,
                                                             int nseg, int64_t nclaims,
                                                             int nstages, int* ctr) {
    using C = S;
    // tile shapes (the heaviest body decides every claim's occupancy):
    // classes 1 and 2 one block per wave with batches of 4 terms, class 4
    // batches of two
    constexpr int KB4 = 2;
    __shared__ int64_t s_claim;
    __shared__ C s_part[4][2][4];
    __shared__ C s_red[TG / 64][NR][64];
    __shared__ C s_pred[TP / 64][NR];
    __shared__ C s_tw[NR > 1 ? 4 : 1][NR > 1 ? kPersistFusedRank : 1][NR];
    __shared__ C s_sw[NR > 1 ? 4 : 1][NR > 1 ? kPersistFusedRank : 1][NR];
    __shared__ NearLds<C, NR> s_near;
    const int tid = threadIdx.x, lane = tid & 63;
    // the wave index as a scalar: a branch on it is uniform within each wave
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    // No branch that splits the lanes of a wave may enclose or border the
    // workgroup barriers of this loop (the compiler would give the lanes of a
    // wave separate trips through them): wave 0 as a whole claims, waits
    // and counts, with lane-dependent values instead of lane conditions.
    // Every vector one stage hands to another is written and read with
    // device-coherent accesses (ldv / stv with CO), everything else the launch
    // reads stays constant during it: so no cache needs writing back or
    // invalidating between stages (on this chip either would act on a whole
    // XCD's L2).  A stage's results are complete once every wave's stores
    // have completed, which each wave waits for before its workgroup counts
    // them; a workgroup reads them only after it saw the count.
    // Claims finished but not yet counted, all of stage `cur`: a workgroup
    // waits for a stage's dependencies once, on its first claim of the stage,
    // and counts its claims of a stage when it moves on (before it waits for
    // another stage) or leaves.
    int pending = 0;
    int cur = -1;
    auto flush = [&] {
        if (pending == 0) return;
        __builtin_amdgcn_s_waitcnt(0);   // this wave's stores are complete
        __syncthreads();
        if (wv == 0)
            __hip_atomic_fetch_add(ctr + kPersistCtrBase + kPersistLine * cur,
                                   lane == 0 ? pending : 0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        pending = 0;
    };
    for (;;) {
        if (wv == 0) {
            const int old = atomicAdd(ctr + 0, lane == 0 ? 1 : 0);
            s_claim = (int64_t)__builtin_amdgcn_readfirstlane(old);
        }
        __syncthreads();
        // the claim, and everything decided from it below, is uniform
        const int64_t g = uniform64(s_claim);
        __syncthreads();
        if (g >= nclaims) break;
        // the segment holding claim g
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].claim0 <= g)
                lo = mid;
            else
                hi = mid - 1;
        }
        const PSeg sg = segs[lo];
        const PSlot& sl = slots[sg.slot];
        const int64_t i0 = sg.first + (g - sg.claim0) * sg.per;
        const int64_t i1 = min(i0 + sg.per, sg.first + sg.nitems);
        // the stages this one needs complete?
        if (sg.stage != cur) {
            flush();
            cur = sg.stage;
            if (wv == 0) {
                // wave 0 polls; the wait is bounded by the wall clock, and a
                // timed-out wait anywhere ends every wait (wrong results and a
                // flag the host reads, instead of a hang)
                const long long t0 = wall_clock64();
                for (int dd = 0; dd < sg.ndep; ++dd) {
                    const int* cnt = ctr + kPersistCtrBase + kPersistLine * sg.dep[dd];
                    int nap = 1;   // polls back off from 0.1 to 3.4 us
                    for (;;) {
                        const int done = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                            cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (done >= sg.dcnt[dd]) break;
                        // the error flag, once backed off
                        const int abort =
                            nap < 32 ? 0
                                     : __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                           ctr + kPersistAbort, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
                        const bool late = (uint64_t)(wall_clock64() - t0) > kPersistWaitTicks;
                        if (abort || late) {
                            const int prev = __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_or(
                                ctr + kPersistAbort, lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT));
                            if (prev == 0) {
                                // the first timeout: which claim waited for which stage
                                ctr[kPersistAbort + 1] = (int)g;
                                ctr[kPersistAbort + 2] = sg.dep[dd];
                                ctr[kPersistAbort + 3] = done;
                            }
                            dd = sg.ndep;
                            break;
                        }
                        for (int z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(4);
                        nap = min(2 * nap, 32);
                    }
                }
            }
            __syncthreads();
        }
        const C* x = (const C*)sl.x;
        C* contrib = (C*)sl.contrib;
        switch (sg.kind) {
        case PK_PERM: {
            const XT* X = (const XT*)sl.X;
            C* xw = (C*)sl.x;
            const int64_t p = i0 * 256 + tid;
            if (p < sl.N) {
                const int64_t u = sl.perm[p];
                for (int c = 0; c < sl.nrhs; ++c) stv<true>(xw + c * sl.N + p, (C)X[c * sl.ldx + u]);
            }
            break;
        }
        case PK_G8:
            lr_group_body<S, C, 8, true>(sl.cblk, i0, i1, sl.sym, x, contrib);
            break;
        case PK_G16:   // class 1 as class 2
        case PK_S2:
            if (i0 + wv < i1)
                lr_stream_body<S, C, 1, 1, 4, true>(sl.cblk[i0 + wv], sl.sym, x, contrib, nullptr,
                                                    0);
            break;
        case PK_S3:
            if (i0 + wv < i1)
                lr_stream_body<S, C, 1, 2, 4, true>(sl.cblk[i0 + wv], sl.sym, x, contrib, nullptr,
                                                    0);
            break;
        case PK_S4:
            lr_stream_body<S, C, 4, 4, KB4, true>(sl.cblk[i0], sl.sym, x, contrib,
                                            reinterpret_cast<C(*)[2][KB4]>(s_part), wv);
            break;
        case PK_FUSED:
            if constexpr (NR > 1) {
                if (i0 + wv < i1)
                    lr_fused_body<S, C, NR, kPersistFusedRank, true>(sl.cblk[i0 + wv], sl.sym, x, sl.N,
                                                               sl.nrhs, sg.c0, sl.CT, contrib,
                                                               s_tw[wv], s_sw[wv]);
            }
            break;
        case PK_PROJ:
            project_body<S, C, NR, true>(sl.blocks, sl.proj[i0], sl.sym, x, sl.N, sl.nrhs, sg.c0,
                                   (C*)sl.pp, s_pred);
            break;
        case PK_PSUM: {
            const C* pp = (const C*)sl.pp;
            proj_sum_body<C, NR, true>(i0 * 256 + tid, sl.psum, sl.npsum, sl.sym,
                                 min(NR, sl.nrhs - sg.c0),
                                 [pp](int64_t i) { return ldv<true>(pp + i); }, sl.TT, (C*)sl.tb,
                                 (C*)sl.sb);
            break;
        }
        case PK_EXP: {
            const C* tb = (const C*)sl.tb;
            const C* sb = (const C*)sl.sb;
            expand_split_body<S, C, NR, true>(
                sl.blocks, sl.ex[i0], sl.nrhs, sg.c0, sl.TT,
                [tb, sb](int side, int64_t i) { return ldv<true>((side ? sb : tb) + i); }, sl.CT,
                contrib, s_red);
            break;
        }
        case PK_NEAR:
            switch (sl.kp.kind) {
#define HODLR_PNEAR(K)                                                                          \
    case K:                                                                                     \
        gather_near_item<XT, C, NR, K, kNearOnly, true>(                                        \
            sl.near[i0], sl.lseg, sl.nrng, sl.kappa, sl.pts, sl.N, sl.d, sl.kp, x, contrib,     \
            sl.CT, sl.perm, sl.nrhs, sg.c0, (XT*)sl.Y, sl.ldy, nullptr, (C*)sl.yn, s_red,       \
            s_near);                                                                            \
        break;
                HODLR_PNEAR(HODLR_K_LOG)
                HODLR_PNEAR(HODLR_K_INV_R)
                HODLR_PNEAR(HODLR_K_INV_R2)
                HODLR_PNEAR(HODLR_K_GAUSS)
                HODLR_PNEAR(HODLR_K_EXP)
                HODLR_PNEAR(HODLR_K_R)
                HODLR_PNEAR(HODLR_K_SIN)
                default:
                HODLR_PNEAR(HODLR_K_INV_SQRT1P)
#undef HODLR_PNEAR
            }
            break;
        case PK_GATHER:
            gather_near_item<XT, C, NR, -1, kGatherOnly, true>(
                sl.near[i0], sl.lseg, sl.nrng, sl.kappa, sl.pts, sl.N, sl.d, sl.kp, x, contrib,
                sl.CT, sl.perm, sl.nrhs, sg.c0, (XT*)sl.Y, sl.ldy, nullptr, (C*)sl.yn, s_red,
                s_near);
            break;
        default:
            break;
        }
        // LDS and the claim slot are reused by the next claim
        __syncthreads();
        ++pending;
    }
    flush();
    // the last workgroup out resets the counters (claim, stages, exit); a
    // workgroup's counts are complete before it counts itself out
    __builtin_amdgcn_s_waitcnt(0);
    if (tid == 0) {
        if (__hip_atomic_fetch_add(ctr + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
            (int)gridDim.x - 1) {
            __hip_atomic_store(ctr + 0, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int t = 0; t < nstages; ++t)
                __hip_atomic_store(ctr + kPersistCtrBase + kPersistLine * t, 0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ctr + 2, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

// Factor words: the projection pass reads terms up to r16(r) + 15 (the
// prefetch after the last chunk) and columns up to len + 512 (the last wave
// of a 512-column panel); the expansion pass terms up to r16(r) + 15 and
// rows up to len + 512 (a tile of four 128-row waves); both read 16-byte
// words.  x rows (projection pass) up to len + 576 of the slice, nrp BF16
// each.  The bounds use len + 1024 and one term chunk more.
int64_t mcore_extent(int64_t r, int64_t len, int nrp) {
    const int64_t ld = fstride<bf16>(len);
    const int64_t terms = ((r + 15) & ~(int64_t)15) + 32;
    const int64_t f = 2 * (terms * ld + len + 1024) + 16;
    const int64_t x = 2 * (len + 1024) * (int64_t)nrp + 16;
    return std::max(f, x);
}

// The segmented route of block b: projections per term and row segment
// (segments of at least 4096 rows so that enough workgroups stream the few
// large blocks at once), their per-term sums, 64-row expansions.
void split_route(hodlr_t h, int64_t b, std::vector<ProjSeg>& pj, std::vector<ProjSum>& ps,
                 std::vector<WorkItem>& xe) {
    const BlockDesc& bd = h->hblocks[b];
    const int nseg = std::max(1, std::min(kProjSegMax, std::max(bd.m, bd.n) / 4096));
    for (int k = 0; k < bd.rank; ++k) {
        const int64_t pidx = (int64_t)ps.size();
        ps.push_back(ProjSum{bd.toff + k, pidx, nseg, 0});
        for (int g = 0; g < nseg; ++g) pj.push_back(ProjSeg{(int32_t)b, k, g, nseg, pidx});
    }
    for (int32_t i = 0; i < bd.m; i += 64)
        xe.push_back(WorkItem{(int32_t)b, i, std::min(64, bd.m - i), 0});
    if (h->opts.symmetric)
        for (int32_t j = 0; j < bd.n; j += 64)
            xe.push_back(WorkItem{(int32_t)b, j, std::min(64, bd.n - j), 1});
}

// The persistent plan: the per-class plan's classes in the same order,
// except that class-4 blocks wider than seg_side and every class-5 block
// join the segmented route (their terms projected by many workgroups at
// once instead of streamed by one).  Replaces the persistent tables; the
// next persistent launch rebuilds its claim queue.
void plan_persistent(hodlr_t h, int seg_side) {
    std::vector<int32_t> pgrp;
    std::vector<ProjSeg> pproj;
    std::vector<ProjSum> ppsum;
    std::vector<WorkItem> pex;
    h->p_class_off.assign(kNumClasses + 1, 0);
    for (int c = 0; c < kNumClasses; ++c) {
        h->p_class_off[c] = (int64_t)pgrp.size();
        for (int64_t t = h->class_off[c]; t < h->class_off[c + 1]; ++t) {
            const int32_t b = h->cls_ids[t];
            const BlockDesc& bd = h->hblocks[b];
            const int side = std::max(bd.m, bd.n);
            if (c == kNumClasses - 1 || (c == kNumClasses - 2 && side > seg_side))
                split_route(h, b, pproj, ppsum, pex);
            else
                pgrp.push_back(b);
        }
    }
    h->p_class_off[kNumClasses] = (int64_t)pgrp.size();
    for (int64_t b : h->split_ids) split_route(h, b, pproj, ppsum, pex);
    auto upload = [&](const void* src, size_t bytes, void** dst) {
        if (*dst) dfree(h, *dst);
        *dst = dalloc(h, std::max<size_t>(bytes, 16));
        if (bytes) HIP_CHECK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    };
    std::vector<BlockDesc> pbd(pgrp.size());
    for (size_t t = 0; t < pgrp.size(); ++t) pbd[t] = h->hblocks[pgrp[t]];
    upload(pbd.data(), sizeof(BlockDesc) * pbd.size(), (void**)&h->p_class_blocks);
    upload(pproj.data(), sizeof(ProjSeg) * pproj.size(), (void**)&h->p_proj);
    upload(ppsum.data(), sizeof(ProjSum) * ppsum.size(), (void**)&h->p_psum);
    upload(pex.data(), sizeof(WorkItem) * pex.size(), (void**)&h->p_exp);
    h->p_n_proj = (int64_t)pproj.size();
    h->p_n_psum = (int64_t)ppsum.size();
    h->p_n_exp = (int64_t)pex.size();
    h->p_seg_side = seg_side;
    h->p_key.clear();
}

// Launch planning (host): which blocks one wave applies, how the others are
// split, where every block writes its contributions, and the per-level tables
// the gather needs.  Integer bookkeeping only.
void plan_apply(hodlr_t h) {
    const int kappa = h->kappa;
    std::vector<int32_t> fused;
    std::vector<ProjSeg> proj;
    std::vector<ProjSum> psum;
    std::vector<WorkItem> ex;
    // contribution offsets: per level, per box, the box's IL entries in order,
    // |A| values each
    std::vector<std::vector<int64_t>> cbase(kappa + 1);
    int64_t ct = 0;
    for (int l = 1; l <= kappa; ++l) {
        LevelData& Lv = h->lev[l];
        std::vector<int64_t> ptr(Lv.nb + 1), eref(std::max<int64_t>(Lv.nnz, 1));
        HIP_CHECK(hipMemcpy(ptr.data(), Lv.il_ptr, sizeof(int64_t) * (Lv.nb + 1),
                            hipMemcpyDeviceToHost));
        if (Lv.nnz)
            HIP_CHECK(hipMemcpy(eref.data(), Lv.eref, sizeof(int64_t) * Lv.nnz,
                                hipMemcpyDeviceToHost));
        cbase[l].resize(Lv.nb);
        for (int64_t A = 0; A < Lv.nb; ++A) {
            const int64_t len = Lv.hstart[A + 1] - Lv.hstart[A];
            cbase[l][A] = ct;
            for (int64_t e = ptr[A]; e < ptr[A + 1]; ++e) {
                BlockDesc& bd = h->hblocks[eref[e] >> 1];
                if (eref[e] & 1)
                    bd.cbwd = ct;
                else
                    bd.cfwd = ct;
                ct += len;
            }
        }
    }
    h->contrib_total = ct;
    // block classes by size: 0, 1: at most 8 / 16 rows, columns and terms
    // (a lane group each); 2..5: one workgroup streams the block (|A|, |B|
    // up to 64, 128, 1024, 4608); larger blocks are split over many
    // workgroups
    std::vector<std::vector<std::pair<int64_t, int32_t>>> cls(kNumClasses);
    for (int c = 0; c < 8; ++c) h->cls_felems[c] = h->cls_velems[c] = 0;
    h->split_blocks = h->split_felems = 0;
    auto add_split = [&](int64_t b, std::vector<ProjSeg>& pj, std::vector<ProjSum>& ps,
                         std::vector<WorkItem>& xe) { split_route(h, b, pj, ps, xe); };
    std::vector<int64_t> split_ids;
    for (int64_t b = 0; b < h->nblocks; ++b) {
        const BlockDesc& bd = h->hblocks[b];
        const int64_t el = (int64_t)std::max(bd.rank, 0) * (bd.m + bd.n);
        const int side = std::max(bd.m, bd.n);
        const int big = std::max(side, bd.rank);
        int c = -1;
        if (big <= 8) c = 0;
        else if (big <= 16) c = 1;
        else if (side <= 64) c = 2;
        else if (side <= 128) c = 3;
        else if (side <= 1024) c = 4;
        else if (side <= 4608) c = 5;
        const int64_t vel = 2 * (int64_t)(bd.m + bd.n) / (h->opts.symmetric ? 1 : 2);
        if (c >= 0) {
            cls[c].push_back({el, (int32_t)b});
            h->cls_felems[c] += el;
            h->cls_velems[c] += vel;
        } else {
            ++h->split_blocks;
            h->split_felems += el;
            split_ids.push_back(b);
            add_split(b, proj, psum, ex);
        }
    }
    // largest first inside a class so the long workgroups start early
    std::vector<int32_t> grp;
    h->class_off.assign(kNumClasses + 1, 0);
    for (int c = 0; c < kNumClasses; ++c) {
        std::stable_sort(cls[c].begin(), cls[c].end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        h->class_off[c] = (int64_t)grp.size();
        for (auto& p : cls[c]) grp.push_back(p.second);
    }
    h->class_off[kNumClasses] = (int64_t)grp.size();
    h->cls_ids = grp;
    h->split_ids = split_ids;
    // leaves: 64-row chunks, their near-field source ranges and, per level,
    // the contribution segments of the box containing them.  A leaf is a
    // leaf box of any level (in a uniform tree: the boxes of level kappa);
    // its rows take the dense pairs of every box containing them, from the
    // root down to the leaf itself.
    std::vector<std::vector<int64_t>> nptr(kappa + 1);
    std::vector<std::vector<int32_t>> ncol(kappa + 1);
    for (int l = 0; l <= kappa; ++l) {
        const LevelData& Lv = h->lev[l];
        if (!Lv.near_nnz) continue;
        nptr[l].resize(Lv.nb + 1);
        ncol[l].resize(Lv.near_nnz);
        HIP_CHECK(hipMemcpy(nptr[l].data(), Lv.near_ptr, sizeof(int64_t) * (Lv.nb + 1),
                            hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(ncol[l].data(), Lv.near_col, sizeof(int32_t) * Lv.near_nnz,
                            hipMemcpyDeviceToHost));
    }
    struct LeafRef {
        int32_t a0, a1;
        int level;
    };
    std::vector<LeafRef> leaves;
    for (int l = 0; l <= kappa; ++l) {
        const LevelData& Lv = h->lev[l];
        for (int64_t A = 0; A < Lv.nb; ++A)
            if (Lv.hflags[A] & 2) leaves.push_back(LeafRef{Lv.hstart[A], Lv.hstart[A + 1], l});
    }
    std::sort(leaves.begin(), leaves.end(),
              [](const LeafRef& x, const LeafRef& y) { return x.a0 < y.a0; });
    const int64_t nleaf = (int64_t)leaves.size();
    std::vector<NearItem> nr;
    std::vector<int2> rng;
    h->near_max_ranges = 0;
    {
        std::vector<int64_t> box(kappa + 1, 0);   // box of each level containing the leaf
        for (int64_t t = 0; t < nleaf; ++t) {
            const LeafRef& lf = leaves[t];
            const int64_t nb0 = (int64_t)rng.size();
            for (int l = 0; l <= lf.level; ++l) {
                const auto& sl = h->lev[l].hstart;
                while (sl[box[l] + 1] <= lf.a0) ++box[l];
                if (nptr[l].empty()) continue;
                const int64_t A = box[l];
                for (int64_t e = nptr[l][A]; e < nptr[l][A + 1]; ++e)
                    rng.push_back(make_int2(sl[ncol[l][e]], sl[ncol[l][e] + 1]));
            }
            const int32_t nn = (int32_t)((int64_t)rng.size() - nb0);
            h->near_max_ranges = std::max<int64_t>(h->near_max_ranges, nn);
            for (int32_t i = lf.a0; i < lf.a1; i += 64)
                nr.push_back(NearItem{(int32_t)t, i, std::min(64, lf.a1 - i), lf.a0, nb0, nn, 0});
        }
    }
    if (rng.empty()) rng.push_back(make_int2(0, 0));
    std::vector<SegRef> seg((size_t)std::max(kappa, 1) * std::max<int64_t>(nleaf, 1));
    for (int l = 1; l <= kappa; ++l) {
        const auto& sl = h->lev[l].hstart;
        std::vector<int64_t> ptr(h->lev[l].nb + 1);
        HIP_CHECK(hipMemcpy(ptr.data(), h->lev[l].il_ptr, sizeof(int64_t) * (h->lev[l].nb + 1),
                            hipMemcpyDeviceToHost));
        int64_t A = 0;
        for (int64_t leafb = 0; leafb < nleaf; ++leafb) {
            const int32_t a0 = leaves[leafb].a0;
            while (sl[A + 1] <= a0) ++A;
            SegRef& r = seg[(size_t)leafb * kappa + (l - 1)];
            // below the leaf's own level the box holding its first row is
            // inactive and has no entries
            r.base = cbase[l][A] + (a0 - sl[A]);
            r.len = sl[A + 1] - sl[A];
            r.ne = l <= leaves[leafb].level ? (int32_t)(ptr[A + 1] - ptr[A]) : 0;
        }
    }
    auto upload = [&](const void* src, size_t bytes, void** dst) {
        if (*dst) dfree(h, *dst);
        *dst = dalloc(h, std::max<size_t>(bytes, 16));
        if (bytes) HIP_CHECK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    };
    // descriptors copied in class order: the kernels index them directly
    std::vector<BlockDesc> cbd(grp.size());
    for (size_t t = 0; t < grp.size(); ++t) cbd[t] = h->hblocks[grp[t]];
    upload(cbd.data(), sizeof(BlockDesc) * cbd.size(), (void**)&h->class_blocks);
    upload(proj.data(), sizeof(ProjSeg) * proj.size(), (void**)&h->proj_items);
    h->n_proj_items = (int64_t)proj.size();
    upload(psum.data(), sizeof(ProjSum) * psum.size(), (void**)&h->proj_sums);
    h->n_proj_sums = (int64_t)psum.size();
    upload(ex.data(), sizeof(WorkItem) * ex.size(), (void**)&h->exp_items);
    h->n_exp_items = (int64_t)ex.size();
    upload(nr.data(), sizeof(NearItem) * nr.size(), (void**)&h->near_items);
    h->n_near_items = (int64_t)nr.size();
    upload(rng.data(), sizeof(int2) * rng.size(), (void**)&h->near_rng);
    plan_persistent(h, h->p_seg_side);
    upload(seg.data(), sizeof(SegRef) * seg.size(), (void**)&h->leaf_seg);
    // skeleton form: projection segments, per-block partial offsets, 256-row
    // expansion chunks (every block, rank 0 included: its rows get zeros)
    if (h->opts.skeleton) {
        std::vector<SkelProj> sp;
        std::vector<SkelSolve> ss(h->nblocks);
        std::vector<WorkItem> se;
        int64_t pt = 0;
        const bool sym = h->opts.symmetric != 0;
        for (int64_t b = 0; b < h->nblocks; ++b) {
            const BlockDesc& bd = h->hblocks[b];
            SkelSolve q{};
            if (bd.rank > 0) {
                q.pf = pt;
                for (int32_t lo = 0; lo < bd.n; lo += kSkelSeg, pt += bd.rank, ++q.nsf)
                    sp.push_back(SkelProj{(int32_t)b, 0, lo, std::min(kSkelSeg, bd.n - lo), pt});
                if (sym) {
                    q.pb = pt;
                    for (int32_t lo = 0; lo < bd.m; lo += kSkelSeg, pt += bd.rank, ++q.nsb)
                        sp.push_back(
                            SkelProj{(int32_t)b, 1, lo, std::min(kSkelSeg, bd.m - lo), pt});
                }
            }
            ss[b] = q;
            for (int32_t i = 0; i < bd.m; i += kSkelRows)
                se.push_back(WorkItem{(int32_t)b, i, std::min(kSkelRows, bd.m - i), 0});
            if (sym)
                for (int32_t j = 0; j < bd.n; j += kSkelRows)
                    se.push_back(WorkItem{(int32_t)b, j, std::min(kSkelRows, bd.n - j), 1});
        }
        upload(sp.data(), sizeof(SkelProj) * sp.size(), (void**)&h->skel_proj);
        upload(ss.data(), sizeof(SkelSolve) * ss.size(), (void**)&h->skel_solve);
        upload(se.data(), sizeof(WorkItem) * se.size(), (void**)&h->skel_exp);
        h->n_skel_proj = (int64_t)sp.size();
        h->n_skel_exp = (int64_t)se.size();
        h->skel_part_total = pt;
        h->skel_max_rank = 0;
        for (int64_t b = 0; b < h->nblocks; ++b)
            h->skel_max_rank = std::max<int64_t>(h->skel_max_rank, h->hblocks[b].rank);
        if (h->skel_max_rank > kSkelMaxR)
            fail(HODLR_EUNSUPPORTED, "skeleton form: a rank above " + std::to_string(kSkelMaxR) +
                                         " (the solves keep both vectors in LDS)");
    }
    h->nleaf = nleaf;
    // matrix-core plan for BF16 factors (several right-hand sides)
    if (h->opts.storage == HODLR_BF16) {
        const bool sym = h->opts.symmetric != 0;
        auto r16 = [](int r) { return (int64_t)((r + 15) & ~15); };
        // projection term offsets: t of every stored block, then s
        std::vector<int64_t> toff(h->nblocks), soff(h->nblocks);
        int64_t tt = 0;
        for (int64_t b = 0; b < h->nblocks; ++b) {
            toff[b] = tt;
            tt += r16(h->hblocks[b].rank);
        }
        if (sym)
            for (int64_t b = 0; b < h->nblocks; ++b) {
                soff[b] = tt;
                tt += r16(h->hblocks[b].rank);
            }
        h->mt_total = tt;
        std::vector<std::vector<std::pair<int64_t, MJob>>> jobs(4);
        std::vector<MRed> reds;
        int64_t pt = 0;
        for (int c = 0; c < 4; ++c) h->mjob_felems[c] = h->mjob_velems[c] = h->mjob_count[c] = 0;
        auto wclass = [](int len) { return len <= 64 ? 0 : len <= 128 ? 1 : len <= 256 ? 2 : 3; };
        auto add_side = [&](uint64_t F, int len, int x0, int r, int64_t out) {
            const int np = (len + MPANEL - 1) / MPANEL;
            if (np <= 1) {
                const int w = wclass(len);
                jobs[w].push_back({(int64_t)r * len, MJob{F, out, r, len, x0, 0, len, 1}});
            } else {
                reds.push_back(MRed{out, pt, (int32_t)r16(r), np});
                for (int p = 0; p < np; ++p) {
                    const int p0 = p * MPANEL, pl = std::min(MPANEL, len - p0);
                    const int w = wclass(pl);
                    jobs[w].push_back({(int64_t)r * pl,
                                       MJob{F, pt + p * r16(r), r, len, x0, p0, pl, 0}});
                }
                pt += np * r16(r);
            }
        };
        // every offset the passes form must stay below 2^31 (see mcore_extent)
        for (int64_t b = 0; b < h->nblocks; ++b) {
            const BlockDesc& bd = h->hblocks[b];
            if (bd.rank <= 0) continue;
            if (mcore_extent(bd.rank, bd.m, 32) >= kMcoreRange ||
                mcore_extent(bd.rank, bd.n, 32) >= kMcoreRange)
                fail(HODLR_EUNSUPPORTED,
                     "a BF16 factor is too large for the matrix-core product's 2^31-byte "
                     "buffer range (rank " + std::to_string(bd.rank) + ", sides " +
                         std::to_string(bd.m) + " x " + std::to_string(bd.n) +
                         "); use FP32 or FP64 storage, or set max_rank");
        }
        for (int64_t b = 0; b < h->nblocks; ++b) {
            const BlockDesc& bd = h->hblocks[b];
            if (bd.rank <= 0) continue;
            add_side(bd.V, bd.n, bd.b0, bd.rank, toff[b]);
            if (sym) add_side(bd.U, bd.m, bd.a0, bd.rank, soff[b]);
        }
        h->mpart_total = pt;
        std::vector<MJob> mj;
        h->mjob_off.assign(5, 0);
        for (int c = 0; c < 4; ++c) {
            // by the x slice they read (first row, then panel), larger first
            // among equals: an XCD's contiguous range of jobs reuses x in its L2
            std::stable_sort(jobs[c].begin(), jobs[c].end(), [](const auto& a, const auto& b) {
                if (a.second.x0 != b.second.x0) return a.second.x0 < b.second.x0;
                if (a.second.p0 != b.second.p0) return a.second.p0 < b.second.p0;
                return a.first > b.first;
            });
            h->mjob_off[c] = (int64_t)mj.size();
            for (auto& p : jobs[c]) {
                mj.push_back(p.second);
                h->mjob_felems[c] += p.first;
                h->mjob_velems[c] += p.second.plen;
            }
            h->mjob_count[c] = (int64_t)jobs[c].size();
        }
        h->mjob_off[4] = (int64_t)mj.size();
        // expansion: per level, every box's interaction-list entries in order
        // and its 128-row tiles
        std::vector<MEnt> ents;
        std::vector<MTile> tiles, small, big;
        h->mtile_off.assign(1, 0);
        h->mexp_felems = 0;
        for (int l = 1; l <= kappa; ++l) {
            LevelData& Lv = h->lev[l];
            std::vector<int64_t> ptr(Lv.nb + 1), eref(std::max<int64_t>(Lv.nnz, 1));
            HIP_CHECK(hipMemcpy(ptr.data(), Lv.il_ptr, sizeof(int64_t) * (Lv.nb + 1),
                                hipMemcpyDeviceToHost));
            if (Lv.nnz)
                HIP_CHECK(hipMemcpy(eref.data(), Lv.eref, sizeof(int64_t) * Lv.nnz,
                                    hipMemcpyDeviceToHost));
            for (int64_t A = 0; A < Lv.nb; ++A) {
                const int32_t len = Lv.hstart[A + 1] - Lv.hstart[A];
                const int64_t e0 = (int64_t)ents.size();
                for (int64_t e = ptr[A]; e < ptr[A + 1]; ++e) {
                    const int64_t blk = eref[e] >> 1;
                    const BlockDesc& bd = h->hblocks[blk];
                    if (eref[e] & 1)
                        ents.push_back(MEnt{bd.V, soff[blk], bd.rank, 0});
                    else
                        ents.push_back(MEnt{bd.U, toff[blk], bd.rank, 0});
                    h->mexp_felems += (int64_t)std::max(bd.rank, 0) * len;
                }
                const int32_t ne = (int32_t)((int64_t)ents.size() - e0);
                if (len <= MSMALL) {
                    small.push_back(MTile{Lv.hstart[A], len, len, 0, e0, ne, 0});
                } else {
                    const int32_t span = MBIGW * 128;
                    for (int32_t r0 = 0; r0 < len; r0 += span)
                        big.push_back(MTile{Lv.hstart[A] + r0, std::min(span, len - r0), len, r0, e0,
                                            ne, 0});
                }
            }
            // level l: small-box tiles, then big-box tiles
            tiles.insert(tiles.end(), small.begin(), small.end());
            h->mtile_off.push_back((int64_t)tiles.size());
            tiles.insert(tiles.end(), big.begin(), big.end());
            h->mtile_off.push_back((int64_t)tiles.size());
            small.clear();
            big.clear();
        }
        upload(mj.data(), sizeof(MJob) * mj.size(), (void**)&h->mjobs);
        upload(reds.data(), sizeof(MRed) * reds.size(), (void**)&h->mreds);
        h->n_mreds = (int64_t)reds.size();
        upload(ents.data(), sizeof(MEnt) * ents.size(), (void**)&h->ments);
        upload(tiles.data(), sizeof(MTile) * tiles.size(), (void**)&h->mtiles);
    }
    if (h->nblocks)
        HIP_CHECK(hipMemcpy(h->blocks, h->hblocks.data(), sizeof(BlockDesc) * h->nblocks,
                            hipMemcpyHostToDevice));
}

namespace {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Grid of the on-the-fly near kernel beside the low-rank stages.  When the
// near field is light next to the factor bytes the stages stream (at most
// kNearCapPairsPerByte dense pairs per column and byte), one workgroup per CU
// looping over the items: the kernel then ends well inside the streams while
// holding only a small share of every CU.  Otherwise one workgroup per item,
// so that a near-heavy product (crowded leaves) gets the whole chip.
constexpr int64_t kNearGridCap = 256;
constexpr double kNearCapPairsPerByte = 0.05;
inline unsigned near_grid(hodlr_t h, int nc, size_t factor_elem_bytes) {
    int64_t fe = h->split_felems;
    for (int c = 0; c < kNumClasses; ++c) fe += h->cls_felems[c];
    const double light = kNearCapPairsPerByte * (double)fe * (double)factor_elem_bytes;
    const int64_t n = h->n_near_items;
    return (unsigned)((double)h->near_pairs * nc <= light ? std::min(n, kNearGridCap) : n);
}

// Candidate tile shapes <W, CH, KB> of the single-RHS block classes (W waves
// per block, CH rows per lane, KB terms per register batch); candidate 0 is
// the default, the autotuner may pick another per handle.  Classes 0 and 1
// (a lane group per block) have one shape.
constexpr int kTuneCands = 3;
inline int class_candidates(int c) { return c <= 1 ? 1 : (c == 5 ? 2 : 3); }

template <typename S, typename C>
void launch_class(int c, int cand, const BlockDesc* it, int64_t cnt, int sym, const C* x,
                  C* contrib, hipStream_t s) {
    const unsigned g = (unsigned)cnt;
    constexpr int K4 = sizeof(C) == 8 ? 2 : 4, K5 = sizeof(C) == 8 ? 1 : 2;
    switch (c * kTuneCands + cand) {
    case 0 * kTuneCands + 0:
        k_lr_group<S, C, 8><<<nblk(cnt * 8, 256), 256, 0, s>>>(it, cnt, sym, x, contrib);
        break;
    case 1 * kTuneCands + 0:
        k_lr_group<S, C, 16><<<nblk(cnt * 16, 256), 256, 0, s>>>(it, cnt, sym, x, contrib);
        break;
    case 2 * kTuneCands + 0: k_lr_stream<S, C, 1, 1, 8><<<g, 64, 0, s>>>(it, sym, x, contrib); break;
    case 2 * kTuneCands + 1: k_lr_stream<S, C, 1, 1, 4><<<g, 64, 0, s>>>(it, sym, x, contrib); break;
    case 2 * kTuneCands + 2: k_lr_stream<S, C, 1, 1, 16><<<g, 64, 0, s>>>(it, sym, x, contrib); break;
    case 3 * kTuneCands + 0: k_lr_stream<S, C, 1, 2, 4><<<g, 64, 0, s>>>(it, sym, x, contrib); break;
    case 3 * kTuneCands + 1: k_lr_stream<S, C, 1, 2, 8><<<g, 64, 0, s>>>(it, sym, x, contrib); break;
    case 3 * kTuneCands + 2: k_lr_stream<S, C, 2, 1, 8><<<g, 128, 0, s>>>(it, sym, x, contrib); break;
    case 4 * kTuneCands + 0: k_lr_stream<S, C, 4, 4, K4><<<g, 256, 0, s>>>(it, sym, x, contrib); break;
    case 4 * kTuneCands + 1:
        k_lr_stream<S, C, 4, 4, 2 * K4><<<g, 256, 0, s>>>(it, sym, x, contrib);
        break;
    case 4 * kTuneCands + 2: k_lr_stream<S, C, 8, 2, K4><<<g, 512, 0, s>>>(it, sym, x, contrib); break;
    case 5 * kTuneCands + 0: k_lr_stream<S, C, 8, 9, K5><<<g, 512, 0, s>>>(it, sym, x, contrib); break;
    default:
        k_lr_stream<S, C, 8, 9, 2 * K5><<<g, 512, 0, s>>>(it, sym, x, contrib);
        break;
    }
}

// aux: the stream of the near field (the handle's second stream, or s itself
// for a product on one stream)
template <typename XT, typename S, typename C, int NR>
void run_matvec(hodlr_t h, const XT* X, int64_t ldx, int nrhs, XT* Y, int64_t ldy, char* ws,
                hipEvent_t const* ev, int nev, hipStream_t s, hipStream_t aux) {
    const int64_t N = h->N;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    const int64_t CT = std::max<int64_t>(h->contrib_total, 1);
    C* x = (C*)ws;
    C* contrib = x + N * nrhs;
    C* tb = contrib + CT * NR;
    C* sb = tb + TT * NR;
    C* pp = sb + TT * NR;   // partials of the segmented projections
    C* yn = pp + 2 * kProjSegMax * std::max(h->n_proj_sums, h->p_n_psum) * NR;   // near sums
    const int sym = h->opts.symmetric ? 1 : 0;
    // the second stream starts after everything issued so far on s, and s
    // waits for all of its work at the join
    auto fork = [&] {
        if (aux == s) return;
        HIP_CHECK(hipEventRecord(h->ev_fork, s));
        HIP_CHECK(hipStreamWaitEvent(aux, h->ev_fork, 0));
    };
    auto join = [&] {
        if (aux == s) return;
        HIP_CHECK(hipEventRecord(h->ev_join, aux));
        HIP_CHECK(hipStreamWaitEvent(s, h->ev_join, 0));
    };
    if (ev) HIP_CHECK(hipEventRecord(ev[0], s));
    k_permute_in<XT, C><<<nblk(N, 256), 256, 0, s>>>(X, ldx, nrhs, N, h->perm, x);
    HIP_CHECK(hipGetLastError());
    if (ev) HIP_CHECK(hipEventRecord(ev[1], s));
    // the contribution buffer holds NR columns: stages repeat per column batch
    constexpr int RMAX = kFusedMaxRank;
    constexpr bool kMfma = std::is_same<S, bf16>::value && NR >= 16;
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        if constexpr (kMfma) {
            const int nc = std::min(NR, nrhs - c0);
            constexpr int CTn = NR / 16;
            // workspace after x: x rows (BF16), level sums, projections, partials
            char* p = ws + align256(sizeof(C) * (size_t)N * nrhs);
            uint16_t* xr = reinterpret_cast<uint16_t*>(p);
            p += align256(2 * (size_t)N * NR);
            float* yl = reinterpret_cast<float*>(p);
            p += align256(4 * (size_t)N * NR);
            uint16_t* tproj = reinterpret_cast<uint16_t*>(p);
            p += align256(2 * (size_t)std::max<int64_t>(h->mt_total, 1) * NR);
            float* part = reinterpret_cast<float*>(p);
            p += align256(4 * (size_t)std::max<int64_t>(h->mpart_total, 1) * NR);
            float* ynm = reinterpret_cast<float*>(p);   // near sums
            k_rows_bf16<XT><<<nblk(N * NR, 256), 256, 0, s>>>(X, ldx, c0, nc, N, h->perm, NR, xr);
            HIP_CHECK(hipGetLastError());
            // the near field on matrix cores, on the second stream beside both
            // passes, into its own sums
            const bool nm = h->near_max_ranges <= kNearTileRanges && h->d <= 4;
            if (nm) {
                fork();
                switch (h->kp.kind * 2 + (h->d == 4 ? 1 : 0)) {
#define HODLR_NEAR_MFMA(K, DC)                                                                  \
    case K * 2 + (DC == 4 ? 1 : 0):                                                             \
        k_near_mfma<CTn, K, DC><<<(unsigned)h->n_near_items, 256, 0, aux>>>(              \
            h->near_items, h->n_near_items, h->near_rng, h->pts, N, h->d, h->kp, xr, nc, ynm);   \
        break;
#define HODLR_NEAR_MFMA2(K) HODLR_NEAR_MFMA(K, 3) HODLR_NEAR_MFMA(K, 4)
                    HODLR_NEAR_MFMA2(HODLR_K_LOG)
                    HODLR_NEAR_MFMA2(HODLR_K_INV_R)
                    HODLR_NEAR_MFMA2(HODLR_K_INV_R2)
                    HODLR_NEAR_MFMA2(HODLR_K_GAUSS)
                    HODLR_NEAR_MFMA2(HODLR_K_EXP)
                    HODLR_NEAR_MFMA2(HODLR_K_R)
                    HODLR_NEAR_MFMA2(HODLR_K_SIN)
                    HODLR_NEAR_MFMA2(HODLR_K_INV_SQRT1P)
#undef HODLR_NEAR_MFMA2
#undef HODLR_NEAR_MFMA
                    default:
                        join();
                        fail(HODLR_EINVAL, "unknown kernel function");
                }
                HIP_CHECK(hipGetLastError());
            }
            k_fill_zero<float><<<nblk(N * NR, 256), 256, 0, s>>>(yl, N * NR);
            HIP_CHECK(hipGetLastError());
            // pass 1: projections, by workgroup width
            for (int w = 0; w < 4; ++w) {
                const int64_t n0 = h->mjob_off[w], cnt = h->mjob_off[w + 1] - n0;
                if (cnt) {
                    const MJob* jb = h->mjobs + n0;
                    const unsigned g = xcd_grid(cnt);
                    // 32 columns: fewer waves per job, two or four column
                    // groups each; 16 columns: one group per wave (its
                    // near field runs beside this pass and takes more of
                    // the chip when the pass holds fewer, fuller waves)
                    if constexpr (CTn == 2) {
                        switch (w) {
                        case 0: k_mproj<1, CTn><<<g, 64, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        case 1: k_mproj<1, CTn, 2><<<g, 64, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        case 2: k_mproj<2, CTn, 2><<<g, 128, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        default: k_mproj<2, CTn, 4><<<g, 128, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        }
                    } else {
                        switch (w) {
                        case 0: k_mproj<1, CTn><<<g, 64, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        case 1: k_mproj<2, CTn><<<g, 128, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        case 2: k_mproj<4, CTn><<<g, 256, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        default: k_mproj<8, CTn><<<g, 512, 0, s>>>(jb, cnt, xr, tproj, part); break;
                        }
                    }
                    HIP_CHECK(hipGetLastError());
                }
                if (ev && nev > 5 && c0 == 0) HIP_CHECK(hipEventRecord(ev[5 + w], s));
            }
            if (h->n_mreds)
                k_mreduce<<<(unsigned)h->n_mreds, 256, 0, s>>>(h->mreds, part, NR, tproj);
            HIP_CHECK(hipGetLastError());
            if (ev && nev > 5 && c0 == 0)
                for (int c = 4; c < kNumClasses; ++c) HIP_CHECK(hipEventRecord(ev[5 + c], s));
            if (ev && c0 == 0) HIP_CHECK(hipEventRecord(ev[2], s));
            // pass 2: expansions, one level at a time (tiles of a level own
            // disjoint rows of the level sum)
            for (int l = 1; l <= h->kappa; ++l) {
                const int64_t t0 = h->mtile_off[2 * l - 2], n0 = h->mtile_off[2 * l - 1] - t0;
                const int64_t t1 = h->mtile_off[2 * l - 1], n1 = h->mtile_off[2 * l] - t1;
                if (n0)
                    k_mexp<CTn, MSMALL / 16, 1><<<(unsigned)n0, 64, 0, s>>>(
                        h->mtiles + t0, h->ments, tproj, N, nc, yl);
                if (n1)
                    k_mexp<CTn, 8, MBIGW><<<(unsigned)n1, 64 * MBIGW, 0, s>>>(
                        h->mtiles + t1, h->ments, tproj, N, nc, yl);
                HIP_CHECK(hipGetLastError());
            }
            if (ev && c0 == 0) HIP_CHECK(hipEventRecord(ev[3], s));
            if (nm) {
                join();
                k_permute_out<XT><<<nblk(N, 256), 256, 0, s>>>(yl, ynm, N, nc, c0, h->perm, Y,
                                                               ldy);
            } else
                k_gather_near<XT, C, NR><<<(unsigned)h->n_near_items, TG, 0, s>>>(
                    h->near_items, h->n_near_items, h->leaf_seg, h->near_rng, h->kappa, h->pts, N,
                    h->d, h->kp, x, contrib, CT, h->perm, nrhs, c0, Y, ldy, yl, nullptr);
            HIP_CHECK(hipGetLastError());
            continue;
        } else {
        // the near field on the second stream, beside the low-rank stages
        fork();
        const unsigned gnear = near_grid(h, std::min(NR, nrhs - c0), sizeof(S));
        {
            // the kernel function fixed at compile time
            switch (h->kp.kind) {
#define HODLR_NEAR(K)                                                                           \
    case K:                                                                                     \
        k_gather_near<XT, C, NR, K, kNearOnly><<<gnear, TG, 0, aux>>>(                         \
            h->near_items, h->n_near_items, h->leaf_seg, h->near_rng, h->kappa, h->pts, N, h->d, \
            h->kp, x, contrib, CT, h->perm, nrhs, c0, Y, ldy, nullptr, yn);                     \
        break;
                HODLR_NEAR(HODLR_K_LOG)
                HODLR_NEAR(HODLR_K_INV_R)
                HODLR_NEAR(HODLR_K_INV_R2)
                HODLR_NEAR(HODLR_K_GAUSS)
                HODLR_NEAR(HODLR_K_EXP)
                HODLR_NEAR(HODLR_K_R)
                HODLR_NEAR(HODLR_K_SIN)
                default:
                HODLR_NEAR(HODLR_K_INV_SQRT1P)
#undef HODLR_NEAR
            }
        }
        HIP_CHECK(hipGetLastError());
        if constexpr (NR == 1 && !std::is_same<S, bf16>::value) {
            if (h->opts.skeleton) {
                // skeleton form: every stored block, the kernel evaluated on the fly
                const C* xc = x + (int64_t)c0 * N;
                if (h->nblocks) {
                    C* skp = yn + (int64_t)N * NR;   // partials of the skeleton projections
                    switch (h->kp.kind) {
#define HODLR_SKEL_P(K, P3)                                                                     \
    if (h->n_skel_proj)                                                                         \
        k_skel_proj<S, C, K, P3><<<(unsigned)h->n_skel_proj, 256, 0, s>>>(                      \
            h->blocks, h->skel_proj, h->pts, N, h->d, h->kp, xc, skp);                          \
    k_skel_solve<S, C><<<(unsigned)h->nblocks, kSkelSolveThreads,                               \
                         2 * sizeof(C) * h->skel_max_rank, s>>>(h->blocks, h->skel_solve, sym,  \
                                                                 skp, tb, sb);                  \
    k_skel_exp<S, C, K, P3><<<(unsigned)h->n_skel_exp, 256, 0, s>>>(                            \
        h->blocks, h->skel_exp, h->pts, N, h->d, h->kp, tb, sb, contrib);
#define HODLR_SKEL(K)                                                                           \
    case K:                                                                                     \
        if (h->d <= 3) {                                                                        \
            HODLR_SKEL_P(K, true)                                                               \
        } else {                                                                                \
            HODLR_SKEL_P(K, false)                                                              \
        }                                                                                       \
        break;
                        HODLR_SKEL(HODLR_K_LOG)
                        HODLR_SKEL(HODLR_K_INV_R)
                        HODLR_SKEL(HODLR_K_INV_R2)
                        HODLR_SKEL(HODLR_K_GAUSS)
                        HODLR_SKEL(HODLR_K_EXP)
                        HODLR_SKEL(HODLR_K_R)
                        HODLR_SKEL(HODLR_K_SIN)
                        default:
                        HODLR_SKEL(HODLR_K_INV_SQRT1P)
#undef HODLR_SKEL
#undef HODLR_SKEL_P
                    }
                    HIP_CHECK(hipGetLastError());
                }
                if (ev && c0 == 0) {
                    for (int c = 0; c < kNumClasses; ++c) HIP_CHECK(hipEventRecord(ev[5 + c], s));
                    HIP_CHECK(hipEventRecord(ev[2], s));
                    HIP_CHECK(hipEventRecord(ev[3], s));
                }
                goto gather;
            }
        }
        if (NR == 1) {
            // one launch per size class
            for (int c = 0; c < kNumClasses; ++c) {
                const int64_t n0 = h->class_off[c], cnt = h->class_off[c + 1] - n0;
                if (!cnt) {
                    if (ev && nev > 5 && c0 == 0) HIP_CHECK(hipEventRecord(ev[5 + c], s));
                    continue;
                }
                launch_class<S, C>(c, h->tune_cls[c], h->class_blocks + n0, cnt, sym, x, contrib,
                                   s);
                if (ev && nev > 5 && c0 == 0) HIP_CHECK(hipEventRecord(ev[5 + c], s));
            }
        } else {
            const int64_t cnt = h->class_off[kNumClasses];
            if (cnt)
                k_lr_fused<S, C, NR, RMAX><<<(unsigned)cnt, 64, 0, s>>>(
                    h->class_blocks, sym, x, N, nrhs, c0, CT, contrib);
        }
        if (h->n_proj_items) {
            k_project<S, C, NR><<<(unsigned)h->n_proj_items, TP, 0, s>>>(
                h->blocks, h->proj_items, sym, x, N, nrhs, c0, pp);
            k_proj_sum<C, NR><<<nblk(h->n_proj_sums * 2 * NR, 256), 256, 0, s>>>(
                h->proj_sums, h->n_proj_sums, sym, std::min(NR, nrhs - c0), pp, TT, tb, sb);
        }
        HIP_CHECK(hipGetLastError());
        if (ev && c0 == 0) HIP_CHECK(hipEventRecord(ev[2], s));
        if (h->n_exp_items)
            k_expand_split<S, C, NR><<<(unsigned)h->n_exp_items, TE, 0, s>>>(
                h->blocks, h->exp_items, nrhs, c0, TT, tb, sb, CT, contrib);
        HIP_CHECK(hipGetLastError());
        if (ev && c0 == 0) HIP_CHECK(hipEventRecord(ev[3], s));
        }
    gather:
        // near-field sums plus the contributions of every level, to Y
        join();
        k_gather_near<XT, C, NR, -1, kGatherOnly><<<(unsigned)h->n_near_items, TG, 0, s>>>(
            h->near_items, h->n_near_items, h->leaf_seg, h->near_rng, h->kappa, h->pts, N, h->d,
            h->kp, x, contrib, CT, h->perm, nrhs, c0, Y, ldy, nullptr, yn);
        HIP_CHECK(hipGetLastError());
    }
    if (ev) HIP_CHECK(hipEventRecord(ev[4], s));
}

template <typename XT, typename S, typename C>
void dispatch_nr(hodlr_t h, const XT* X, int64_t ldx, int nrhs, XT* Y, int64_t ldy, char* ws,
                 hipEvent_t const* ev, int nev, hipStream_t s, hipStream_t aux) {
    if constexpr (std::is_same<S, bf16>::value) {
        // BF16 factors: matrix cores for several right-hand sides
        if (nrhs == 1)
            run_matvec<XT, S, C, 1>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s, aux);
        else if (nrhs <= 16)
            run_matvec<XT, S, C, 16>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s, aux);
        else
            run_matvec<XT, S, C, 32>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s, aux);
        return;
    }
    if (nrhs == 1 || h->opts.skeleton)   // the skeleton form takes one column per pass
        run_matvec<XT, S, C, 1>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s, aux);
    else if (nrhs <= 4)
        run_matvec<XT, S, C, 4>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s, aux);
    else
        run_matvec<XT, S, C, 8>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s, aux);
}

// ---- persistent product: host side -------------------------------------
// One slot: a handle's product of nrhs columns, X -> Y, with the workspace
// carved as in run_matvec.
struct PSlotHost {
    hodlr_t h;
    const void* X;
    int64_t ldx;
    void* Y;
    int64_t ldy;
    int nrhs;
    char* ws;
};

// The claim queue of a persistent launch.  Stages and what they need:
//   P     the permutation into tree order
//   A_b   column batch b: the blocks of every class and the segmented
//         projections (needs P, and G_{b-1}, which last read the buffers)
//   S_b   sums of the segmented projections (needs A_b)
//   N_b   the near field (needs P and G_{b-1}; queued between the largest
//         blocks of A_b and the rest, so that it runs beside them)
//   E_b   expansions of the segmented blocks (needs S_b)
//   G_b   the gather (needs A_b, N_b, E_b)
// Every stage is queued after the stages it needs.
void persist_segments(const std::vector<PSlotHost>& sl, int NR, std::vector<PSeg>& segs,
                      int64_t& nclaims, int& nstages) {
    segs.clear();
    int64_t claim = 0;
    std::vector<int64_t> scnt;   // claims per stage
    auto stage = [&] {
        scnt.push_back(0);
        return (int)scnt.size() - 1;
    };
    std::vector<int> deps;
    auto add = [&](int st, int slot, int kind, int c0, int64_t first, int64_t n, int per) {
        if (n <= 0) return;
        PSeg q{};
        q.claim0 = claim;
        q.first = first;
        q.nitems = n;
        q.slot = slot;
        q.kind = kind;
        q.c0 = c0;
        q.per = per;
        q.stage = st;
        q.ndep = 0;
        segs.push_back(q);
        const int64_t c = (n + per - 1) / per;
        claim += c;
        scnt[st] += c;
    };
    // stage ids each segment depends on, set after all claims are known
    std::vector<std::vector<int>> sdeps;
    auto need = [&](int st, std::initializer_list<int> d) {
        if ((int)sdeps.size() <= st) sdeps.resize(st + 1);
        for (int x : d)
            if (x >= 0) sdeps[st].push_back(x);
    };
    int maxcb = 0;
    for (auto& q : sl) maxcb = std::max(maxcb, (q.nrhs + NR - 1) / NR);
    const int P = stage();
    need(P, {});
    for (int t = 0; t < (int)sl.size(); ++t)
        add(P, t, PK_PERM, 0, 0, (sl[t].h->N + 255) / 256, 1);
    int Gprev = -1;
    for (int cb = 0; cb < maxcb; ++cb) {
        const int c0 = cb * NR;
        const int A = stage(), Sx = stage(), Nr = stage(), E = stage(), G = stage();
        need(A, {P, Gprev});
        need(Sx, {A});
        need(Nr, {P, Gprev});
        need(E, {Sx});
        need(G, {A, Nr, E});
        for (int t = 0; t < (int)sl.size(); ++t) {
            hodlr_t h = sl[t].h;
            if (sl[t].nrhs <= c0) continue;
            const std::vector<int64_t>& o = h->p_class_off;
            add(A, t, PK_PROJ, c0, 0, h->p_n_proj, 1);
            if (NR == 1) {
                add(A, t, PK_S4, c0, o[4], o[5] - o[4], 1);
                add(Nr, t, PK_NEAR, c0, 0, h->n_near_items, 1);
                add(A, t, PK_S3, c0, o[3], o[4] - o[3], 4);
                add(A, t, PK_S2, c0, o[2], o[3] - o[2], 4);
                add(A, t, PK_G16, c0, o[1], o[2] - o[1], 4);
                add(A, t, PK_G8, c0, o[0], o[1] - o[0], 32);
            } else {
                add(A, t, PK_FUSED, c0, o[0], o[6] - o[0], 4);
                add(Nr, t, PK_NEAR, c0, 0, h->n_near_items, 1);
            }
        }
        for (int t = 0; t < (int)sl.size(); ++t)
            if (sl[t].nrhs > c0)
                add(Sx, t, PK_PSUM, c0, 0, (sl[t].h->p_n_psum * 2 * NR + 255) / 256, 1);
        for (int t = 0; t < (int)sl.size(); ++t)
            if (sl[t].nrhs > c0) add(E, t, PK_EXP, c0, 0, sl[t].h->p_n_exp, 1);
        for (int t = 0; t < (int)sl.size(); ++t)
            if (sl[t].nrhs > c0) add(G, t, PK_GATHER, c0, 0, sl[t].h->n_near_items, 1);
        Gprev = G;
    }
    nstages = (int)scnt.size();
    if (nstages > kPersistMaxStages)
        fail(HODLR_EUNSUPPORTED, "more right-hand sides than one persistent launch takes");
    sdeps.resize(nstages);
    for (auto& q : segs) {
        // a dependency with no claims is complete from the start
        for (int x : sdeps[q.stage])
            if (scnt[x] > 0) {
                q.dep[q.ndep] = x;
                q.dcnt[q.ndep] = (int32_t)scnt[x];
                ++q.ndep;
            }
    }
    nclaims = claim;
}

template <typename C>
PSlot persist_slot(const PSlotHost& q, int NR) {
    hodlr_t h = q.h;
    const int64_t N = h->N;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    const int64_t CT = std::max<int64_t>(h->contrib_total, 1);
    C* x = (C*)q.ws;
    C* contrib = x + N * q.nrhs;
    C* tb = contrib + CT * NR;
    C* sb = tb + TT * NR;
    C* pp = sb + TT * NR;
    C* yn = pp + 2 * kProjSegMax * std::max(h->n_proj_sums, h->p_n_psum) * NR;
    PSlot p{};
    p.cblk = h->p_class_blocks;
    p.blocks = h->blocks;
    p.proj = h->p_proj;
    p.psum = h->p_psum;
    p.ex = h->p_exp;
    p.near = h->near_items;
    p.lseg = h->leaf_seg;
    p.nrng = h->near_rng;
    p.pts = h->pts;
    p.perm = h->perm;
    p.X = q.X;
    p.Y = q.Y;
    p.x = x;
    p.contrib = contrib;
    p.tb = tb;
    p.sb = sb;
    p.pp = pp;
    p.yn = yn;
    p.kp = h->kp;
    p.N = N;
    p.ldx = q.ldx;
    p.ldy = q.ldy;
    p.CT = CT;
    p.TT = TT;
    p.npsum = h->p_n_psum;
    p.d = h->d;
    p.kappa = h->kappa;
    p.sym = h->opts.symmetric ? 1 : 0;
    p.nrhs = q.nrhs;
    return p;
}

template <typename XT, typename S, int NR>
unsigned persist_grid(int64_t nclaims) {
    static int cap = -1;
    static std::mutex mu;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (cap < 0) {
            int per_cu = 0, dev = 0, cus = 0;
            HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<XT, S, NR>,
                                                                   kPersistThreads, 0));
            HIP_CHECK(hipGetDevice(&dev));
            HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            cap = std::max(1, per_cu) * std::max(1, cus);
        }
    }
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nclaims, cap));
}

// the error flag of a finished persistent launch (a wait that timed out)
void persist_check(int* ctr, hipStream_t s) {
    int v[4] = {0};
    HIP_CHECK(hipMemcpyAsync(v, ctr + kPersistAbort, sizeof(v), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (v[0]) {
        // the flag is cleared for the next launch (every other count was
        // reset by the launch's last workgroup)
        HIP_CHECK(hipMemsetAsync(ctr + kPersistAbort, 0, sizeof(v), s));
        HIP_CHECK(hipStreamSynchronize(s));
        fail(HODLR_EDEVICE, "persistent product: a stage wait timed out (claim " +
                                std::to_string(v[1]) + " waited for stage " +
                                std::to_string(v[2]) + ", which had " + std::to_string(v[3]) +
                                " completed claims)");
    }
}

// Launches the persistent product of the slots on s.  dslots / dsegs: device
// tables of at least slots.size() / segs.size() entries, written here when
// `upload` is set; ctr: kPersistCtrInts zeroed ints (left zeroed by the launch).
template <typename XT, typename S, int NR>
void persist_launch(const std::vector<PSlotHost>& slots, const std::vector<PSeg>& segs,
                    int64_t nclaims, int nstages, PSlot* dslots, PSeg* dsegs, bool upload,
                    int* ctr, hipStream_t s) {
    if (upload) {
        std::vector<PSlot> ps(slots.size());
        for (size_t t = 0; t < slots.size(); ++t) ps[t] = persist_slot<S>(slots[t], NR);
        HIP_CHECK(hipMemcpyAsync(dslots, ps.data(), sizeof(PSlot) * ps.size(),
                                 hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(dsegs, segs.data(), sizeof(PSeg) * segs.size(),
                                 hipMemcpyHostToDevice, s));
    }
    if (nclaims <= 0) return;
    k_persist<XT, S, NR><<<persist_grid<XT, S, NR>(nclaims), kPersistThreads, 0, s>>>(
        dslots, dsegs, (int)segs.size(), nclaims, nstages, ctr);
    HIP_CHECK(hipGetLastError());
}

// Workspace (per product, device memory) for nrhs columns in compute_prec.
size_t workspace_need(hodlr_t h, int nrhs, int compute_prec) {
    const int64_t N = h->N;
    const size_t cs = compute_prec == HODLR_FP32 ? 4 : 8;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    const int64_t CT = std::max<int64_t>(h->contrib_total, 1);
    const bool b16 = h->opts.storage == HODLR_BF16;
    const int nr = (nrhs == 1 || h->opts.skeleton) ? 1
                   : b16 ? (nrhs <= 16 ? 16 : 32) : (nrhs <= 4 ? 4 : 8);
    if (b16 && nr >= 16)   // x, x rows, level sums, projections, panel partials, near sums
        return align256(cs * (size_t)N * nrhs) + align256(2 * (size_t)N * nr) +
               align256(4 * (size_t)N * nr) +
               align256(2 * (size_t)std::max<int64_t>(h->mt_total, 1) * nr) +
               align256(4 * (size_t)std::max<int64_t>(h->mpart_total, 1) * nr) +
               align256(4 * (size_t)N * nr) + 4096;
    // x, contributions, projections, partials, near-field sums (and the
    // skeleton projections' partials)
    return cs * ((size_t)N * nrhs + (size_t)CT * nr + 2 * (size_t)TT * nr +
                 2 * (size_t)kProjSegMax * (size_t)std::max(h->n_proj_sums, h->p_n_psum) * nr +
                 (size_t)N * nr + (h->opts.skeleton ? (size_t)h->skel_part_total : 0)) +
           4096;
}

void run_product(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y,
                 int64_t ldy, int compute_prec, char* ws, hipEvent_t const* ev, int nev,
                 hipStream_t s, hipStream_t aux) {
    const bool b16 = h->opts.storage == HODLR_BF16;
    const bool s32 = h->opts.storage == HODLR_FP32;
    const bool c32 = compute_prec == HODLR_FP32;
    if (b16) {
        // BF16 factors are applied in FP32 (checked by the caller)
        if (x_prec == HODLR_FP64)
            dispatch_nr<double, bf16, float>(h, (const double*)X, ldx, nrhs, (double*)Y, ldy, ws,
                                             ev, nev, s, aux);
        else
            dispatch_nr<float, bf16, float>(h, (const float*)X, ldx, nrhs, (float*)Y, ldy, ws, ev,
                                            nev, s, aux);
        return;
    }
    if (x_prec == HODLR_FP64) {
        const double* Xd = (const double*)X;
        double* Yd = (double*)Y;
        if (!s32 && !c32) dispatch_nr<double, double, double>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s, aux);
        else if (!s32 && c32) dispatch_nr<double, double, float>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s, aux);
        else if (s32 && !c32) dispatch_nr<double, float, double>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s, aux);
        else dispatch_nr<double, float, float>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s, aux);
    } else {
        const float* Xf = (const float*)X;
        float* Yf = (float*)Y;
        if (!s32 && !c32) dispatch_nr<float, double, double>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s, aux);
        else if (!s32 && c32) dispatch_nr<float, double, float>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s, aux);
        else if (s32 && !c32) dispatch_nr<float, float, double>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s, aux);
        else dispatch_nr<float, float, float>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s, aux);
    }
}

// Static workspace of the product for callers that cannot allocate: one copy
// per GPU, held until the process ends.  Host code uses it only through the
// device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[kScratchBytes];

char* scratch_address(int device) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static void* addr[kMaxDev] = {};
    if (device < 0 || device >= kMaxDev) fail(HODLR_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(HODLR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[device] = p;
    }
    return (char*)addr[device];
}

}  // namespace

void reserve_workspace(hodlr_t h, int nrhs, int compute_prec, hipStream_t s) {
    const size_t need = workspace_need(h, nrhs, compute_prec);
    // growing allocates and synchronises, and creating the second stream is
    // no stream operation: neither is allowed inside a graph capture
    auto capturing = [&] {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        return s && hipStreamIsCapturing(s, &cap) == hipSuccess &&
               cap != hipStreamCaptureStatusNone;
    };
    if (h->ws_bytes < need || !h->aux) {
        if (capturing())
            fail(HODLR_EINVAL, "workspace not reserved before stream capture "
                               "(call hodlr_reserve_workspace first)");
    }
    if (!h->aux) {
        HIP_CHECK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    if (!h->p_ctr) {
        // the persistent launch's counters start at zero and each launch
        // leaves them at zero
        h->p_ctr = (int*)dalloc(h, kPersistCtrInts * sizeof(int));
        HIP_CHECK(hipMemset(h->p_ctr, 0, kPersistCtrInts * sizeof(int)));
    }
    if (h->ws_bytes < need) {
        if (h->ws) {
            HIP_CHECK(hipStreamSynchronize(s));
            dfree(h, h->ws);
            h->ws = nullptr;
            h->ws_bytes = 0;
        }
        h->ws = dalloc(h, need);
        h->ws_bytes = need;
    }
}

bool persistent_route(hodlr_t h, int x_prec, int compute_prec) {
    (void)x_prec;
    const bool supported = !h->opts.skeleton && h->opts.storage != HODLR_BF16 &&
                           ((h->opts.storage == HODLR_FP64) == (compute_prec == HODLR_FP64));
    if (!supported) return false;
    return h->use_persistent == 1;
}

namespace {
template <typename XT, typename S, int NR>
void persist_single(hodlr_t h, const void* X, int64_t ldx, int nrhs, void* Y, int64_t ldy,
                    hipStream_t s) {
    const std::vector<int64_t> key = {(int64_t)(uintptr_t)X, ldx, nrhs, (int64_t)(uintptr_t)Y,
                                      ldy, (int64_t)(uintptr_t)h->ws, (int64_t)sizeof(XT),
                                      (int64_t)sizeof(S), NR};
    if (key != h->p_key) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (s && hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
            fail(HODLR_EINVAL, "a persistent product captured with new arguments: run it once "
                               "with the same X, Y and nrhs before the capture");
        std::vector<PSlotHost> sl = {PSlotHost{h, X, ldx, Y, ldy, nrhs, (char*)h->ws}};
        std::vector<PSeg> segs;
        int64_t nclaims = 0;
        int nstages = 0;
        persist_segments(sl, NR, segs, nclaims, nstages);
        if (!h->p_dslot) h->p_dslot = dalloc(h, sizeof(PSlot));
        if (h->p_segcap < segs.size()) {
            HIP_CHECK(hipStreamSynchronize(s));
            dfree(h, h->p_dsegs);
            h->p_segcap = segs.size() + 16;
            h->p_dsegs = dalloc(h, sizeof(PSeg) * h->p_segcap);
        }
        persist_launch<XT, S, NR>(sl, segs, nclaims, nstages, (PSlot*)h->p_dslot,
                                  (PSeg*)h->p_dsegs, true, h->p_ctr, s);
        persist_check(h->p_ctr, s);   // synchronises: the host tables may go
        h->p_key = key;
        h->p_nclaims = nclaims;
        h->p_nseg = segs.size();
        h->p_nstages = nstages;
        return;
    }
    std::vector<PSlotHost> none;
    std::vector<PSeg> segs(h->p_nseg);   // only the count is used without upload
    persist_launch<XT, S, NR>(none, segs, h->p_nclaims, h->p_nstages, (PSlot*)h->p_dslot,
                              (PSeg*)h->p_dsegs, false, h->p_ctr, s);
}

template <typename XT, typename S>
void persist_dispatch(hodlr_t h, const void* X, int64_t ldx, int nrhs, void* Y, int64_t ldy,
                      hipStream_t s) {
    if (nrhs == 1)
        persist_single<XT, S, 1>(h, X, ldx, nrhs, Y, ldy, s);
    else if (nrhs <= 4)
        persist_single<XT, S, 4>(h, X, ldx, nrhs, Y, ldy, s);
    else
        persist_single<XT, S, 8>(h, X, ldx, nrhs, Y, ldy, s);
}
}  // namespace

void matvec(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y, int64_t ldy,
            int compute_prec, hipEvent_t const* ev, int nev, hipStream_t s) {
    reserve_workspace(h, nrhs, compute_prec, s);
    if (!ev && nrhs <= kPersistMaxCols && persistent_route(h, x_prec, compute_prec)) {
        const bool s64 = h->opts.storage == HODLR_FP64;
        if (x_prec == HODLR_FP64) {
            if (s64) persist_dispatch<double, double>(h, X, ldx, nrhs, Y, ldy, s);
            else persist_dispatch<double, float>(h, X, ldx, nrhs, Y, ldy, s);
        } else {
            if (s64) persist_dispatch<float, double>(h, X, ldx, nrhs, Y, ldy, s);
            else persist_dispatch<float, float>(h, X, ldx, nrhs, Y, ldy, s);
        }
        return;
    }
    // route 2: the near field on the caller's stream too
    run_product(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec, (char*)h->ws, ev, nev, s,
                h->use_persistent == 2 ? s : h->aux);
}

namespace {
template <typename XT, typename S, int NR>
void batch_launch(const std::vector<PSlotHost>& sl, int* ctr, hodlr_t h0, hipStream_t s) {
    std::vector<PSeg> segs;
    int64_t nclaims = 0;
    int nstages = 0;
    persist_segments(sl, NR, segs, nclaims, nstages);
    PSlot* dslot = (PSlot*)dalloc(h0, sizeof(PSlot) * sl.size());
    PSeg* dsegs = (PSeg*)dalloc(h0, sizeof(PSeg) * std::max<size_t>(segs.size(), 1));
    persist_launch<XT, S, NR>(sl, segs, nclaims, nstages, dslot, dsegs, true, ctr, s);
    persist_check(ctr, s);
    dfree(h0, dslot);
    dfree(h0, dsegs);
}
}  // namespace

// Device tables of asynchronous batched launches (one set per server slot).
struct BatchTables {
    PSlot* dslot = nullptr;
    PSeg* dsegs = nullptr;
    int* ctr = nullptr;
    int max_slots = 0;
    size_t segcap = 0;
};

void* batch_tables_create(int max_slots, size_t segcap) {
    auto* t = new BatchTables();
    t->max_slots = max_slots;
    t->segcap = segcap;
    if (hipMalloc(&t->dslot, sizeof(PSlot) * max_slots) != hipSuccess ||
        hipMalloc(&t->dsegs, sizeof(PSeg) * segcap) != hipSuccess ||
        hipMalloc(&t->ctr, kPersistCtrInts * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(t->dslot);
        (void)hipFree(t->dsegs);
        delete t;
        fail(HODLR_ENOMEM, "batch tables");
    }
    HIP_CHECK(hipMemset(t->ctr, 0, kPersistCtrInts * sizeof(int)));
    return t;
}

void batch_tables_destroy(void* p) {
    auto* t = (BatchTables*)p;
    if (!t) return;
    (void)hipFree(t->dslot);
    (void)hipFree(t->dsegs);
    (void)hipFree(t->ctr);
    delete t;
}

namespace {
template <typename XT, typename S, int NR>
void batch_async(const std::vector<PSlotHost>& sl, BatchTables* t, hipStream_t s) {
    std::vector<PSeg> segs;
    int64_t nclaims = 0;
    int nstages = 0;
    persist_segments(sl, NR, segs, nclaims, nstages);
    if ((int)sl.size() > t->max_slots || segs.size() > t->segcap)
        fail(HODLR_EINVAL, "batch larger than its tables");
    persist_launch<XT, S, NR>(sl, segs, nclaims, nstages, t->dslot, t->dsegs, true, t->ctr, s);
}
}  // namespace

void matvec_batch_async(int nslots, hodlr_t const* hs, const void* const* X, const int64_t* ldx,
                        const int* nrhs, int x_prec, void* const* Y, const int64_t* ldy,
                        void* tables, hipStream_t s) {
    if (nslots <= 0) return;
    auto* t = (BatchTables*)tables;
    const int st = hs[0]->opts.storage;
    const int comp = st == HODLR_FP64 ? HODLR_FP64 : HODLR_FP32;
    int maxr = 1;
    for (int i = 0; i < nslots; ++i) {
        if (hs[i]->opts.storage != st || hs[i]->opts.skeleton || st == HODLR_BF16)
            fail(HODLR_EINVAL, "a batch needs FP64 or FP32 factors of one storage precision");
        maxr = std::max(maxr, nrhs[i]);
    }
    const int NR = maxr == 1 ? 1 : (maxr <= 4 ? 4 : 8);
    std::vector<PSlotHost> sl;
    for (int i = 0; i < nslots; ++i) {
        const int sizing = NR == 1 ? 1 : std::max(nrhs[i], NR == 4 ? 2 : 5);
        reserve_workspace(hs[i], sizing, comp, s);
        sl.push_back(PSlotHost{hs[i], X[i], ldx[i], Y[i], ldy[i], nrhs[i], (char*)hs[i]->ws});
    }
    const bool s64 = st == HODLR_FP64;
#define HODLR_BATCH(XT, S)                                                                      \
    do {                                                                                        \
        if (NR == 1) batch_async<XT, S, 1>(sl, t, s);                                           \
        else if (NR == 4) batch_async<XT, S, 4>(sl, t, s);                                      \
        else batch_async<XT, S, 8>(sl, t, s);                                                   \
    } while (0)
    if (x_prec == HODLR_FP64) {
        if (s64) HODLR_BATCH(double, double);
        else HODLR_BATCH(double, float);
    } else {
        if (s64) HODLR_BATCH(float, double);
        else HODLR_BATCH(float, float);
    }
#undef HODLR_BATCH
}

namespace {
// mean time of `reps` calls of fn on s after one untimed call, in ms
template <typename F>
double time_ms(F&& fn, hipStream_t s, int reps) {
    hipEvent_t a, b;
    HIP_CHECK(hipEventCreate(&a));
    HIP_CHECK(hipEventCreate(&b));
    fn();
    HIP_CHECK(hipEventRecord(a, s));
    for (int i = 0; i < reps; ++i) fn();
    HIP_CHECK(hipEventRecord(b, s));
    HIP_CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return (double)ms / reps;
}

// the least of three such timings (a one-off stall in one of them, from
// whatever else the GPU or the runtime does, would decide the choice)
template <typename F>
double time_ms_best(F&& fn, hipStream_t s, int reps) {
    double best = 1e300;
    for (int t = 0; t < 3; ++t) best = std::min(best, time_ms(fn, s, reps));
    return best;
}

// every tile-shape candidate of every single-RHS block class, timed alone on
// the handle's own blocks (inputs: the workspace's x; outputs: its
// contribution segments), the fastest kept
template <typename S, typename C>
void tune_classes(hodlr_t h, hodlr_tuning* out, hipStream_t s, int reps) {
    C* x = (C*)h->ws;
    C* contrib = x + h->N;
    const int sym = h->opts.symmetric ? 1 : 0;
    for (int c = 0; c < kNumClasses; ++c) {
        const int64_t n0 = h->class_off[c], cnt = h->class_off[c + 1] - n0;
        h->tune_cls[c] = 0;
        out->class_choice[c] = 0;
        out->class_ms[c] = 0.0;
        if (!cnt) continue;
        double best = 1e300;
        for (int cand = 0; cand < class_candidates(c); ++cand) {
            const double ms = time_ms_best(
                [&] {
                    launch_class<S, C>(c, cand, h->class_blocks + n0, cnt, sym, x, contrib, s);
                    HIP_CHECK(hipGetLastError());
                },
                s, reps);
            if (ms < best) {
                best = ms;
                h->tune_cls[c] = cand;
            }
        }
        out->class_choice[c] = h->tune_cls[c];
        out->class_ms[c] = best;
    }
}
}  // namespace

void autotune(hodlr_t h, int nrhs, int x_prec, int compute_prec, hodlr_tuning* out,
              hipStream_t s) {
    const int64_t N = h->N;
    const size_t xs = x_prec == HODLR_FP64 ? 8 : 4;
    std::memset(out, 0, sizeof(*out));
    void* X = dalloc(h, xs * (size_t)N * nrhs);
    void* Y = dalloc(h, xs * (size_t)N * nrhs);
    HIP_CHECK(hipMemsetAsync(X, 0, xs * (size_t)N * nrhs, s));
    reserve_workspace(h, nrhs, compute_prec, s);
    const int reps = 5;
    const int saved = h->use_persistent;
    try {
        if (nrhs == 1 && !h->opts.skeleton) {
            const bool c32 = compute_prec == HODLR_FP32;
            switch (h->opts.storage) {
            case HODLR_FP64:
                if (c32) tune_classes<double, float>(h, out, s, reps);
                else tune_classes<double, double>(h, out, s, reps);
                break;
            case HODLR_FP32:
                if (c32) tune_classes<float, float>(h, out, s, reps);
                else tune_classes<float, double>(h, out, s, reps);
                break;
            default:
                tune_classes<bf16, float>(h, out, s, reps);
                break;
            }
        }
        auto product = [&] { matvec(h, X, N, nrhs, x_prec, Y, N, compute_prec, nullptr, 0, s); };
        h->use_persistent = 0;
        out->class_route_ms = time_ms_best(product, s, reps);
        h->use_persistent = 2;
        out->one_stream_ms = time_ms_best(product, s, reps);
        const int per_class = out->one_stream_ms < out->class_route_ms ? 2 : 0;
        const double per_class_ms = std::min(out->one_stream_ms, out->class_route_ms);
        h->use_persistent = 1;
        if (persistent_route(h, x_prec, compute_prec)) {
            // the persistent plan's widest block a workgroup streams alone:
            // every class-4 block (1024), or only those up to 512 or 256 rows
            // (the wider ones segmented over many workgroups)
            const int sides[3] = {1024, 512, 256};
            double best = 1e300;
            int keep = sides[0];
            for (int side : sides) {
                plan_persistent(h, side);
                product();   // builds the claim queue outside the timing
                const double ms = time_ms_best(product, s, reps);
                if (ms < best) {
                    best = ms;
                    keep = side;
                }
            }
            if (keep != h->p_seg_side) plan_persistent(h, keep);
            out->persistent_ms = best;
            out->seg_side = keep;
            out->route = out->persistent_ms < per_class_ms ? 1 : per_class;
        } else {
            out->persistent_ms = 0.0;
            out->route = per_class;
        }
        h->use_persistent = out->route;
    } catch (...) {
        h->use_persistent = saved;
        (void)hipStreamSynchronize(s);
        dfree(h, X);
        dfree(h, Y);
        throw;
    }
    HIP_CHECK(hipStreamSynchronize(s));
    dfree(h, X);
    dfree(h, Y);
}

void matvec_batch(int nslots, hodlr_t const* hs, const void* const* X, const int64_t* ldx,
                  const int* nrhs, int x_prec, void* const* Y, const int64_t* ldy, int* ctr,
                  hipStream_t s) {
    if (nslots <= 0) return;
    if (!ctr) {
        // the first handle's counters (reserved with its workspace below)
        reserve_workspace(hs[0], nrhs[0], hs[0]->opts.storage == HODLR_FP64 ? HODLR_FP64
                                                                            : HODLR_FP32, s);
        ctr = hs[0]->p_ctr;
    }
    const int st = hs[0]->opts.storage;
    const int comp = st == HODLR_FP64 ? HODLR_FP64 : HODLR_FP32;
    int maxr = 1;
    std::vector<PSlotHost> sl;
    for (int t = 0; t < nslots; ++t) {
        hodlr_t h = hs[t];
        if (h->opts.storage != st || h->opts.skeleton || st == HODLR_BF16)
            fail(HODLR_EINVAL, "a batch needs FP64 or FP32 factors of one storage precision");
        maxr = std::max(maxr, nrhs[t]);
    }
    const int NR = maxr == 1 ? 1 : (maxr <= 4 ? 4 : 8);
    for (int t = 0; t < nslots; ++t) {
        // every slot's workspace sized for the batch's column block NR (a
        // column count that the sizing maps to NR)
        const int sizing = NR == 1 ? 1 : std::max(nrhs[t], NR == 4 ? 2 : 5);
        reserve_workspace(hs[t], sizing, comp, s);
        sl.push_back(PSlotHost{hs[t], X[t], ldx[t], Y[t], ldy[t], nrhs[t], (char*)hs[t]->ws});
    }
    const bool s64 = st == HODLR_FP64;
#define HODLR_BATCH(XT, S)                                                                          do {                                                                                                if (NR == 1) batch_launch<XT, S, 1>(sl, ctr, hs[0], s);                                         else if (NR == 4) batch_launch<XT, S, 4>(sl, ctr, hs[0], s);                                    else batch_launch<XT, S, 8>(sl, ctr, hs[0], s);                                             } while (0)
    if (x_prec == HODLR_FP64) {
        if (s64) HODLR_BATCH(double, double);
        else HODLR_BATCH(double, float);
    } else {
        if (s64) HODLR_BATCH(float, double);
        else HODLR_BATCH(float, float);
    }
#undef HODLR_BATCH
}

void matvec_noalloc(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y,
                    int64_t ldy, int compute_prec, hipStream_t s) {
    const size_t need = workspace_need(h, nrhs, compute_prec);
    if (need > (size_t)kScratchBytes)
        fail(HODLR_EINVAL, "this product needs " + std::to_string(need) +
                               " bytes of workspace, more than the static scratch of " +
                               std::to_string((size_t)kScratchBytes) +
                               " bytes (fewer right-hand sides, or hodlr_matvec)");
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev != h->device) fail(HODLR_EINVAL, "the handle's device is not the current device");
    // no second stream: the near field runs on s between the other stages
    run_product(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec, scratch_address(dev), nullptr, 0,
                s, s);
}

}  // namespace hodlr
