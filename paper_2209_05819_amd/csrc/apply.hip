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

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int TP = 256;   // split projection workgroup (4 waves)
constexpr int TE = 256;   // split expansion workgroup (4 waves share 64 rows)
constexpr int KB = 16;    // rows reduced together in the fused projection
constexpr int kFusedMaxRank = 256;  // projections a fused wave keeps in LDS at once
constexpr int kNumClasses = kApplyClasses;  // block size classes of the one-workgroup kernels

template <typename C>
__device__ __forceinline__ C wsum(C v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduce KB = 2^q partial sums per lane over the 64 lanes at once: at each
// halving step a lane keeps half of its values and sends the other half to
// its partner, so KB sums cost KB-1 exchanges plus 6-q plain steps (instead
// of 6 KB).  On return lane L holds the full sum of row (L >> (6 - q)).
template <typename C, int K>
__device__ __forceinline__ C multi_reduce(C (&p)[K]) {
    const int lane = threadIdx.x & 63;
    int width = K;
    int off = 32;
#pragma unroll
    for (int step = 0; (1 << step) < K; ++step) {
        const int half = width >> 1;
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int kk = 0; kk < K / 2; ++kk) {
            if (kk < half) {
                const C keep = upper ? p[half + kk] : p[kk];
                const C give = upper ? p[kk] : p[half + kk];
                p[kk] = keep + __shfl_xor(give, off, 64);
            }
        }
        width = half;
        off >>= 1;
    }
    C v = p[0];
    for (; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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

// One wave applies one stored block with NR right-hand sides: the
// projections of up to RMAX terms (multi-row reductions in batches of K),
// then their expansion re-reading the factors (cache hits); repeated over
// chunks of RMAX terms, accumulating into the contribution segments.
template <typename S, typename C, int NR, int RMAX>
__global__ __launch_bounds__(64) void k_lr_fused(const BlockDesc* __restrict__ blocks, int sym,
                                                 const C* __restrict__ x, int64_t N, int nrhs,
                                                 int c0, int64_t CT, C* __restrict__ contrib) {
    constexpr int K = NR == 1 ? KB : 4;
    constexpr int Q = Log2<K>::v;
    __shared__ C tw[RMAX][NR], sw[RMAX][NR];
    const BlockDesc b = blocks[blockIdx.x];
    const int lane = threadIdx.x;
    const gptr_t<S> U = as_global<S>(b.U);
    const gptr_t<S> V = as_global<S>(b.V);
    const int nc = min(NR, nrhs - c0);
    const int r = b.rank, m = b.m, n = b.n;
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
                for (int c = 0; c < NR; ++c) xv[c] = c < nc ? xB[(int64_t)c * N + j] : (C)0;
#pragma unroll
                for (int kk = 0; kk < K; ++kk)
                    if (kk < kr) {
                        const C v = (C)V[(int64_t)(kc + k0 + kk) * n + j];
#pragma unroll
                        for (int c = 0; c < NR; ++c) pv[c][kk] += v * xv[c];
                    }
            }
            if (sym) {
                for (int i = lane; i < m; i += 64) {
                    C xu[NR];
#pragma unroll
                    for (int c = 0; c < NR; ++c) xu[c] = c < nc ? xA[(int64_t)c * N + i] : (C)0;
#pragma unroll
                    for (int kk = 0; kk < K; ++kk)
                        if (kk < kr) {
                            const C u = (C)U[(int64_t)(kc + k0 + kk) * m + i];
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
        __syncthreads();
        // expansion of this chunk: c_A += U t (and c_B += V^T s)
        for (int i = lane; i < m; i += 64) {
            C acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = (kc > 0 && c < nc) ? contrib[(int64_t)c * CT + b.cfwd + i] : (C)0;
#pragma unroll 4
            for (int k = 0; k < rc; ++k) {
                const C u = (C)U[(int64_t)(kc + k) * m + i];
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += u * tw[k][c];
            }
            for (int c = 0; c < nc; ++c) contrib[(int64_t)c * CT + b.cfwd + i] = acc[c];
        }
        if (sym) {
            for (int j = lane; j < n; j += 64) {
                C acc[NR];
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    acc[c] = (kc > 0 && c < nc) ? contrib[(int64_t)c * CT + b.cbwd + j] : (C)0;
#pragma unroll 4
                for (int k = 0; k < rc; ++k) {
                    const C v = (C)V[(int64_t)(kc + k) * n + j];
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += v * sw[k][c];
                }
                for (int c = 0; c < nc; ++c) contrib[(int64_t)c * CT + b.cbwd + j] = acc[c];
            }
        }
        __syncthreads();
    }
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
    gptr_t<S> Vk = V + k0 * n;
    gptr_t<S> Uk = U + k0 * m;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + c * 64;
            bt.v[kk][c] = (kk < kr && i < n) ? (C)Vk[kk * n + i] : (C)0;
            bt.u[kk][c] = (kk < kr && i < m) ? (C)Uk[kk * m + i] : (C)0;
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
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            tk[kk] = __shfl(tv, kk << (6 - Q), 64);
            sk[kk] = __shfl(sv, kk << (6 - Q), 64);
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

template <typename S, typename C, int W, int CH, int KB>
__global__ __launch_bounds__(64 * W) void k_lr_stream(const BlockDesc* __restrict__ blocks, int sym,
                                                      const C* __restrict__ x,
                                                      C* __restrict__ contrib) {
    __shared__ C part[W][2][KB];
    const BlockDesc b = blocks[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = b.rank, m = b.m, n = b.n;
    const gptr_t<S> U = as_global<S>(b.U);
    const gptr_t<S> V = as_global<S>(b.V);
    const int base = wv * 64 * CH + lane;
    C xa[CH], xb[CH], ca[CH], cb[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int i = base + c * 64;
        xa[c] = i < m ? x[b.a0 + i] : (C)0;
        xb[c] = i < n ? x[b.b0 + i] : (C)0;
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
        if (i < m) contrib[b.cfwd + i] = ca[c];
        if (sym && i < n) contrib[b.cbwd + i] = cb[c];
    }
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
template <typename S, typename C, int G>
__global__ __launch_bounds__(256) void k_lr_group(const BlockDesc* __restrict__ blocks,
                                                  int64_t nitems, int sym,
                                                  const C* __restrict__ x,
                                                  C* __restrict__ contrib) {
    const int g = threadIdx.x & (G - 1);
    const int base = (threadIdx.x & 63) & ~(G - 1);   // first lane of the group
    const int64_t item = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
    const bool valid = item < nitems;
    BlockDesc b{};
    if (valid) b = blocks[item];
    const int r = valid ? b.rank : 0, m = b.m, n = b.n;
    const gptr_t<S> U = as_global<S>(b.U);
    const gptr_t<S> V = as_global<S>(b.V);
    C u[G], v[G], p[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        u[k] = (k < r && g < m) ? (C)U[(int64_t)k * m + g] : (C)0;
        v[k] = (k < r && g < n) ? (C)V[(int64_t)k * n + g] : (C)0;
    }
    const C xa = (valid && g < m) ? x[b.a0 + g] : (C)0;
    const C xb = (valid && g < n) ? x[b.b0 + g] : (C)0;
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
    if (valid && g < m) contrib[b.cfwd + g] = ca;
    if (valid && sym && g < n) contrib[b.cbwd + g] = cb;
}

// One term (row of V, column of U) of a large block per workgroup: the 256
// threads stride over the row with four independent partial sums, then a
// workgroup reduction gives t_k (and s_k).
template <typename C, int NR>
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
            out[(int64_t)c * stride] = v;
        }
    __syncthreads();
}

template <typename S, typename C, int NR>
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
            const C v = (C)row[j + u * TP];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nc) a[u][c] += v * xs[(int64_t)c * N + j + u * TP];
        }
    }
    for (; j < len; j += TP) {
        const C v = (C)row[j];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            if (c < nc) a[0][c] += v * xs[(int64_t)c * N + j];
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = (a[0][c] + a[1][c]) + (a[2][c] + a[3][c]);
}

template <typename S, typename C, int NR>
__global__ __launch_bounds__(TP) void k_project(const BlockDesc* __restrict__ blocks,
                                                const WorkItem* __restrict__ items, int sym,
                                                const C* __restrict__ x, int64_t N, int nrhs,
                                                int c0, int64_t TT, C* __restrict__ tb,
                                                C* __restrict__ sb) {
    __shared__ C red[TP / 64][NR];
    const WorkItem it = items[blockIdx.x];
    const BlockDesc b = blocks[it.id];
    const gptr_t<S> Ub = as_global<S>(b.U);
    const gptr_t<S> Vb = as_global<S>(b.V);
    const int nc = min(NR, nrhs - c0);
    const C* __restrict__ xB = x + (int64_t)c0 * N + b.b0;
    const C* __restrict__ xA = x + (int64_t)c0 * N + b.a0;
    for (int k = it.lo; k < it.lo + it.cnt; ++k) {
        C acc[NR];
        row_dot<S, C, NR>(Vb + (int64_t)k * b.n, b.n, xB, N, nc, acc);
        wg_reduce_store<C, NR>(acc, red, nc, tb + b.toff + k, TT);
        if (sym) {
            row_dot<S, C, NR>(Ub + (int64_t)k * b.m, b.m, xA, N, nc, acc);
            wg_reduce_store<C, NR>(acc, red, nc, sb + b.toff + k, TT);
        }
    }
}

// 64-row chunk of one side of a large block: side 0 writes U t into the rows
// of A, side 1 writes V^T s into the rows of B; the 4 waves split the terms
template <typename S, typename C, int NR>
__global__ __launch_bounds__(TE) void k_expand_split(const BlockDesc* __restrict__ blocks,
                                                     const WorkItem* __restrict__ items, int nrhs,
                                                     int c0, int64_t TT, const C* __restrict__ tb,
                                                     const C* __restrict__ sb, int64_t CT,
                                                     C* __restrict__ contrib) {
    __shared__ C part[TE / 64][NR][64];
    const WorkItem it = items[blockIdx.x];
    const BlockDesc b = blocks[it.id];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool tr = it.level != 0;
    const gptr_t<S> W = as_global<S>(tr ? b.V : b.U);
    const int len = tr ? b.n : b.m;
    const C* __restrict__ coef = (tr ? sb : tb) + b.toff;
    const int o = it.lo + lane;
    const bool active = lane < it.cnt;
    const int nc = min(NR, nrhs - c0);
    C acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0;
    if (active) {
        for (int k = wv; k < b.rank; k += TE / 64) {
            const C w = (C)W[(int64_t)k * len + o];
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] += w * coef[(int64_t)c * TT + k];
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
            contrib[(int64_t)c * CT + seg + o] = s;
        }
    }
}

// rows [lo, lo+cnt) of one leaf: near field on the fly plus the low-rank
// contributions of every level, written to Y in user order.  The 4 waves of
// the workgroup and, when cnt < 64, slices of lanes inside a wave split the
// sources and the contribution segments; partial sums meet in a fixed order.
// The leaf's source ranges and per-level segments are precomputed, so its
// loads do not depend on each other.
constexpr int TG = 256;
constexpr int kNearTile = 256;         // sources per LDS tile
constexpr int kNearTileRanges = 1024;  // near boxes a tiled leaf may have

template <typename XT, typename C, int NR>
__global__ __launch_bounds__(TG) void k_gather_near(
    const NearItem* __restrict__ items, const SegRef* __restrict__ lseg,
    const int2* __restrict__ nrng, int kappa, const double* __restrict__ pts, int64_t N, int d,
    KParams kp, const C* __restrict__ x, const C* __restrict__ contrib, int64_t CT,
    const int32_t* __restrict__ perm, int nrhs, int c0, XT* __restrict__ Y, int64_t ldy) {
    __shared__ C red[TG / 64][NR][64];
    const NearItem it = items[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
    if (active)
        for (int a = 0; a < d; ++a) xi[a] = pts[a * N + i];
    if (d <= 4 && it.nn <= kNearTileRanges) {
        // sources staged through LDS in tiles: coalesced cooperative loads,
        // then every lane reads them as broadcasts
        __shared__ int s_pre[kNearTileRanges + 1], s_rs[kNearTileRanges];
        __shared__ int s_j[kNearTile];
        __shared__ double s_pt[4][kNearTile];
        __shared__ C s_x[NR][kNearTile];
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
                s_j[q] = j;
                for (int a = 0; a < d; ++a) s_pt[a][q] = pts[a * N + j];
#pragma unroll
                for (int c = 0; c < NR; ++c) s_x[c][q] = c < nc ? x[(int64_t)(c0 + c) * N + j] : (C)0;
            }
            __syncthreads();
            if (active) {
#pragma unroll 4
                for (int q = sg; q < tn; q += SG) {
                    C kij;
                    if (s_j[q] == i) {
                        kij = (C)kp.diag;
                    } else {
                        C r2 = 0;
                        for (int a = 0; a < d; ++a) {
                            const C dx = (C)(xi[a] - s_pt[a][q]);
                            r2 += dx * dx;
                        }
                        kij = kfun(kp, r2);
                    }
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += kij * s_x[c][q];
                }
            }
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
                    kij = kfun(kp, r2);
                }
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nc) acc[c] += kij * x[(int64_t)(c0 + c) * N + j];
            }
        }
    }
    if (active) {
        const int64_t off = i - it.leaf0;
        for (int l = 0; l < kappa; ++l) {
            const SegRef sr = lseg[(int64_t)it.leaf * kappa + l];
            const C* __restrict__ seg = contrib + sr.base + off;
#pragma unroll 4
            for (int64_t e = sg; e < sr.ne; e += SG)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nc) acc[c] += seg[(int64_t)c * CT + e * sr.len];
        }
    }
    for (int o = mp; o < 64; o <<= 1)
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
#pragma unroll
    for (int c = 0; c < NR; ++c) red[wv][c][lane] = acc[c];
    __syncthreads();
    if (wv == 0 && active && lane < mp) {
        const int64_t u = perm[i];
        for (int c = 0; c < nc; ++c) {
            C v = red[0][c][lane];
            for (int w = 1; w < TG / 64; ++w) v += red[w][c][lane];
            Y[(int64_t)(c0 + c) * ldy + u] = (XT)v;
        }
    }
}

}  // namespace

// Launch planning (host): which blocks one wave applies, how the others are
// split, where every block writes its contributions, and the per-level tables
// the gather needs.  Integer bookkeeping only.
void plan_apply(hodlr_t h) {
    const int kappa = h->kappa;
    std::vector<int32_t> fused;
    std::vector<WorkItem> proj, ex;
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
            const int per = 1;
            for (int k = 0; k < bd.rank; k += per)
                proj.push_back(WorkItem{(int32_t)b, k, std::min(per, bd.rank - k), bd.level});
            for (int32_t i = 0; i < bd.m; i += 64)
                ex.push_back(WorkItem{(int32_t)b, i, std::min(64, bd.m - i), 0});
            if (h->opts.symmetric)
                for (int32_t j = 0; j < bd.n; j += 64)
                    ex.push_back(WorkItem{(int32_t)b, j, std::min(64, bd.n - j), 1});
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
    // leaves: 64-row chunks, their near-field source ranges and, per level,
    // the contribution segments of the box containing them
    const auto& st = h->lev[kappa].hstart;
    const int64_t nleaf = h->lev[kappa].nb;
    std::vector<int64_t> nptr(nleaf + 1);
    std::vector<int32_t> ncol(std::max<int64_t>(h->near_nnz, 1));
    HIP_CHECK(hipMemcpy(nptr.data(), h->near_ptr, sizeof(int64_t) * (nleaf + 1),
                        hipMemcpyDeviceToHost));
    if (h->near_nnz)
        HIP_CHECK(hipMemcpy(ncol.data(), h->near_col, sizeof(int32_t) * h->near_nnz,
                            hipMemcpyDeviceToHost));
    std::vector<NearItem> nr;
    for (int64_t A = 0; A < nleaf; ++A)
        for (int32_t i = st[A]; i < st[A + 1]; i += 64)
            nr.push_back(NearItem{(int32_t)A, i, std::min(64, st[A + 1] - i), st[A], nptr[A],
                                  (int32_t)(nptr[A + 1] - nptr[A]), 0});
    std::vector<int2> rng(std::max<int64_t>(h->near_nnz, 1));
    for (int64_t e = 0; e < h->near_nnz; ++e) rng[e] = make_int2(st[ncol[e]], st[ncol[e] + 1]);
    std::vector<SegRef> seg((size_t)std::max(kappa, 1) * nleaf);
    for (int l = 1; l <= kappa; ++l) {
        const auto& sl = h->lev[l].hstart;
        std::vector<int64_t> ptr(h->lev[l].nb + 1);
        HIP_CHECK(hipMemcpy(ptr.data(), h->lev[l].il_ptr, sizeof(int64_t) * (h->lev[l].nb + 1),
                            hipMemcpyDeviceToHost));
        int64_t A = 0;
        for (int64_t leafb = 0; leafb < nleaf; ++leafb) {
            while (sl[A + 1] <= st[leafb]) ++A;
            SegRef& r = seg[(size_t)leafb * kappa + (l - 1)];
            r.base = cbase[l][A] + (st[leafb] - sl[A]);
            r.len = sl[A + 1] - sl[A];
            r.ne = (int32_t)(ptr[A + 1] - ptr[A]);
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
    upload(proj.data(), sizeof(WorkItem) * proj.size(), (void**)&h->proj_items);
    h->n_proj_items = (int64_t)proj.size();
    upload(ex.data(), sizeof(WorkItem) * ex.size(), (void**)&h->exp_items);
    h->n_exp_items = (int64_t)ex.size();
    upload(nr.data(), sizeof(NearItem) * nr.size(), (void**)&h->near_items);
    h->n_near_items = (int64_t)nr.size();
    upload(rng.data(), sizeof(int2) * rng.size(), (void**)&h->near_rng);
    upload(seg.data(), sizeof(SegRef) * seg.size(), (void**)&h->leaf_seg);
    h->nleaf = nleaf;
    if (h->nblocks)
        HIP_CHECK(hipMemcpy(h->blocks, h->hblocks.data(), sizeof(BlockDesc) * h->nblocks,
                            hipMemcpyHostToDevice));
}

namespace {

template <typename XT, typename S, typename C, int NR>
void run_matvec(hodlr_t h, const XT* X, int64_t ldx, int nrhs, XT* Y, int64_t ldy, char* ws,
                hipEvent_t const* ev, int nev, hipStream_t s) {
    const int64_t N = h->N;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    const int64_t CT = std::max<int64_t>(h->contrib_total, 1);
    C* x = (C*)ws;
    C* contrib = x + N * nrhs;
    C* tb = contrib + CT * NR;
    C* sb = tb + TT * NR;
    const int sym = h->opts.symmetric ? 1 : 0;
    if (ev) HIP_CHECK(hipEventRecord(ev[0], s));
    k_permute_in<XT, C><<<nblk(N, 256), 256, 0, s>>>(X, ldx, nrhs, N, h->perm, x);
    HIP_CHECK(hipGetLastError());
    if (ev) HIP_CHECK(hipEventRecord(ev[1], s));
    // the contribution buffer holds NR columns: stages repeat per column batch
    constexpr int RMAX = kFusedMaxRank;
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        if (NR == 1) {
            // one launch per size class
            for (int c = 0; c < kNumClasses; ++c) {
                const int64_t n0 = h->class_off[c], cnt = h->class_off[c + 1] - n0;
                if (!cnt) {
                    if (ev && nev > 5 && c0 == 0) HIP_CHECK(hipEventRecord(ev[5 + c], s));
                    continue;
                }
                const BlockDesc* it = h->class_blocks + n0;
                const unsigned g = (unsigned)cnt;
                switch (c) {
                case 0:
                    k_lr_group<S, C, 8><<<nblk(cnt * 8, 256), 256, 0, s>>>(it, cnt, sym, x, contrib);
                    break;
                case 1:
                    k_lr_group<S, C, 16><<<nblk(cnt * 16, 256), 256, 0, s>>>(it, cnt, sym, x, contrib);
                    break;
                case 2:
                    k_lr_stream<S, C, 1, 1, 8><<<g, 64, 0, s>>>(it, sym, x, contrib);
                    break;
                case 3:
                    k_lr_stream<S, C, 1, 2, 4><<<g, 64, 0, s>>>(it, sym, x, contrib);
                    break;
                case 4:
                    k_lr_stream<S, C, 4, 4, sizeof(C) == 8 ? 2 : 4><<<g, 256, 0, s>>>(it, sym, x,
                                                                                   contrib);
                    break;
                default:
                    k_lr_stream<S, C, 8, 9, sizeof(C) == 8 ? 1 : 2><<<g, 512, 0, s>>>(it, sym, x,
                                                                                   contrib);
                    break;
                }
                if (ev && nev > 5 && c0 == 0) HIP_CHECK(hipEventRecord(ev[5 + c], s));
            }
        } else {
            const int64_t cnt = h->class_off[kNumClasses];
            if (cnt)
                k_lr_fused<S, C, NR, RMAX><<<(unsigned)cnt, 64, 0, s>>>(
                    h->class_blocks, sym, x, N, nrhs, c0, CT, contrib);
        }
        if (h->n_proj_items)
            k_project<S, C, NR><<<(unsigned)h->n_proj_items, TP, 0, s>>>(
                h->blocks, h->proj_items, sym, x, N, nrhs, c0, TT, tb, sb);
        HIP_CHECK(hipGetLastError());
        if (ev && c0 == 0) HIP_CHECK(hipEventRecord(ev[2], s));
        if (h->n_exp_items)
            k_expand_split<S, C, NR><<<(unsigned)h->n_exp_items, TE, 0, s>>>(
                h->blocks, h->exp_items, nrhs, c0, TT, tb, sb, CT, contrib);
        HIP_CHECK(hipGetLastError());
        if (ev && c0 == 0) HIP_CHECK(hipEventRecord(ev[3], s));
        k_gather_near<XT, C, NR><<<(unsigned)h->n_near_items, TG, 0, s>>>(
            h->near_items, h->leaf_seg, h->near_rng, h->kappa, h->pts, N, h->d, h->kp, x,
            contrib, CT, h->perm, nrhs, c0, Y, ldy);
        HIP_CHECK(hipGetLastError());
    }
    if (ev) HIP_CHECK(hipEventRecord(ev[4], s));
}

template <typename XT, typename S, typename C>
void dispatch_nr(hodlr_t h, const XT* X, int64_t ldx, int nrhs, XT* Y, int64_t ldy, char* ws,
                 hipEvent_t const* ev, int nev, hipStream_t s) {
    if (nrhs == 1)
        run_matvec<XT, S, C, 1>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s);
    else if (nrhs <= 4)
        run_matvec<XT, S, C, 4>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s);
    else
        run_matvec<XT, S, C, 8>(h, X, ldx, nrhs, Y, ldy, ws, ev, nev, s);
}

}  // namespace

void matvec(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y, int64_t ldy,
            int compute_prec, hipEvent_t const* ev, int nev, hipStream_t s) {
    const int64_t N = h->N;
    const size_t cs = compute_prec == HODLR_FP32 ? 4 : 8;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    const int64_t CT = std::max<int64_t>(h->contrib_total, 1);
    const int nr = nrhs == 1 ? 1 : (nrhs <= 4 ? 4 : 8);
    const size_t need = cs * ((size_t)N * nrhs + (size_t)CT * nr + 2 * (size_t)TT * nr) + 4096;
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
    char* ws = (char*)h->ws;
    const bool s32 = h->opts.storage == HODLR_FP32;
    const bool c32 = compute_prec == HODLR_FP32;
    if (x_prec == HODLR_FP64) {
        const double* Xd = (const double*)X;
        double* Yd = (double*)Y;
        if (!s32 && !c32) dispatch_nr<double, double, double>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s);
        else if (!s32 && c32) dispatch_nr<double, double, float>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s);
        else if (s32 && !c32) dispatch_nr<double, float, double>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s);
        else dispatch_nr<double, float, float>(h, Xd, ldx, nrhs, Yd, ldy, ws, ev, nev, s);
    } else {
        const float* Xf = (const float*)X;
        float* Yf = (float*)Y;
        if (!s32 && !c32) dispatch_nr<float, double, double>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s);
        else if (!s32 && c32) dispatch_nr<float, double, float>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s);
        else if (s32 && !c32) dispatch_nr<float, float, double>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s);
        else dispatch_nr<float, float, float>(h, Xf, ldx, nrhs, Yf, ldy, ws, ev, nev, s);
    }
}

}  // namespace hodlr
