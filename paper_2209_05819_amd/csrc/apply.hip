// The HODLRdD matrix-vector product (paper Alg. "HODLRdD matrix-vector
// Product") on the device:
//   1. permute-in: x = X in tree order (compute precision);
//   2. projection: for every stored block b, t_b = V_b x_B and, when the
//      block also stands for its transpose, s_b = U_b^T x_A;
//   3. expansion: for every box A of every level, y_l(A) = sum over IL(A) of
//      U_b t_b (entry stored as (A,B)) or V_b^T s_b (entry stored as (B,A));
//   4. near field + permute-out: Y(perm) = sum_l y_l + sum over near(A) of
//      K(A,B) x_B, the kernel evaluated on the fly.
// Every output element is produced by one thread in a fixed order, so the
// result is bitwise reproducible; no floating-point atomics are used.
#include <algorithm>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int TP = 256;   // projection workgroup
constexpr int TE = 256;   // expansion workgroup (4 waves share 64 rows)
constexpr int TN = 64;    // near-field workgroup (one wave)

template <typename C>
__device__ __forceinline__ C wsum(C v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename XT, typename C>
__global__ void k_permute_in(const XT* __restrict__ X, int64_t ldx, int nrhs, int64_t N,
                             const int32_t* __restrict__ perm, C* __restrict__ x) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t u = perm[p];
    for (int c = 0; c < nrhs; ++c) x[c * N + p] = (C)X[c * ldx + u];
}

// rows [lo, lo+cnt) of one stored block; wave w takes rows lo+w, lo+w+4, ...
template <typename S, typename C, int NR>
__global__ __launch_bounds__(TP) void k_project(const BlockDesc* __restrict__ blocks,
                                                const WorkItem* __restrict__ items, int sym,
                                                const C* __restrict__ x, int64_t N, int nrhs,
                                                int c0, int64_t TT, C* __restrict__ tb,
                                                C* __restrict__ sb) {
    const WorkItem it = items[blockIdx.x];
    const BlockDesc b = blocks[it.id];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const S* __restrict__ Ub = reinterpret_cast<const S*>(b.U);
    const S* __restrict__ Vb = reinterpret_cast<const S*>(b.V);
    const int nc = min(NR, nrhs - c0);
    for (int k = it.lo + wv; k < it.lo + it.cnt; k += TP / 64) {
        C acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = 0;
        const S* __restrict__ row = Vb + (int64_t)k * b.n;
        for (int j = lane; j < b.n; j += 64) {
            const C v = (C)row[j];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nc) acc[c] += v * x[(int64_t)(c0 + c) * N + b.b0 + j];
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = wsum(acc[c]);
        if (lane == 0)
            for (int c = 0; c < nc; ++c) tb[(int64_t)(c0 + c) * TT + b.toff + k] = acc[c];
        if (sym) {
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = 0;
            const S* __restrict__ col = Ub + (int64_t)k * b.m;
            for (int i = lane; i < b.m; i += 64) {
                const C u = (C)col[i];
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nc) acc[c] += u * x[(int64_t)(c0 + c) * N + b.a0 + i];
            }
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = wsum(acc[c]);
            if (lane == 0)
                for (int c = 0; c < nc; ++c) sb[(int64_t)(c0 + c) * TT + b.toff + k] = acc[c];
        }
    }
}

// rows [lo, lo+cnt) (cnt <= 64) of box id of level `level`; the four waves
// split the (entry, term) pairs and are summed through LDS in a fixed order
template <typename S, typename C, int NR>
__global__ __launch_bounds__(TE) void k_expand(const BlockDesc* __restrict__ blocks,
                                               const WorkItem* __restrict__ items,
                                               const int32_t* const* __restrict__ lstart,
                                               const int64_t* const* __restrict__ lptr,
                                               const int64_t* const* __restrict__ lref,
                                               int64_t N, int nrhs, int c0, int64_t TT,
                                               const C* __restrict__ tb, const C* __restrict__ sb,
                                               C* __restrict__ ylev) {
    __shared__ C part[TE / 64][NR][64];
    const WorkItem it = items[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int level = it.level;
    const int32_t a0 = lstart[level][it.id];
    const int o = it.lo - a0 + lane;          // row offset inside box A
    const bool active = lane < it.cnt;
    const int nc = min(NR, nrhs - c0);
    C acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0;
    const int64_t e0 = lptr[level][it.id], e1 = lptr[level][it.id + 1];
    const int64_t* __restrict__ ref = lref[level];
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t rf = ref[e];
        const BlockDesc b = blocks[rf >> 1];
        const bool tr = (rf & 1) != 0;
        const S* __restrict__ W = reinterpret_cast<const S*>(tr ? b.V : b.U);
        const int len = tr ? b.n : b.m;       // == |A|
        const C* __restrict__ coef = (tr ? sb : tb) + b.toff;
        if (active) {
            for (int k = wv; k < b.rank; k += TE / 64) {
                const C w = (C)W[(int64_t)k * len + o];
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nc) acc[c] += w * coef[(int64_t)(c0 + c) * TT + k];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) part[wv][c][lane] = acc[c];
    __syncthreads();
    if (wv == 0 && active) {
        for (int c = 0; c < nc; ++c) {
            C s = part[0][c][lane];
            for (int w = 1; w < TE / 64; ++w) s += part[w][c][lane];
            ylev[((int64_t)(level - 1) * nrhs + c0 + c) * N + it.lo + lane] = s;
        }
    }
}

template <typename C>
__device__ __forceinline__ C pair_r2(const double* __restrict__ pts, int64_t N, int d, int64_t i,
                                     int64_t j) {
    C r2 = 0;
    for (int a = 0; a < d; ++a) {
        const C t = (C)(pts[a * N + i] - pts[a * N + j]);
        r2 += t * t;
    }
    return r2;
}

// near field of rows [lo, lo+cnt) of leaf box id, plus the low-rank sums of
// every level, written to Y in user order.  Lanes are split into S slices
// over the sources when the box has fewer than 64 rows.
template <typename XT, typename C, int NR>
__global__ __launch_bounds__(TN) void k_near_out(
    const WorkItem* __restrict__ items, const int32_t* __restrict__ start,
    const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
    const double* __restrict__ pts, int64_t N, int d, KParams kp, const C* __restrict__ x,
    const C* __restrict__ ylev, int kappa, const int32_t* __restrict__ perm, int nrhs, int c0,
    XT* __restrict__ Y, int64_t ldy) {
    const WorkItem it = items[blockIdx.x];
    const int lane = threadIdx.x;
    int mp = 1;
    while (mp < it.cnt) mp <<= 1;
    const int S = 64 / mp;
    const int t = lane % mp, sl = lane / mp;
    const bool active = t < it.cnt;
    const int64_t i = it.lo + t;
    const int nc = min(NR, nrhs - c0);
    C acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0;
    if (active) {
        for (int64_t e = nptr[it.id]; e < nptr[it.id + 1]; ++e) {
            const int32_t B = ncol[e];
            for (int64_t j = start[B] + sl; j < start[B + 1]; j += S) {
                C kij;
                if (j == i)
                    kij = (C)kp.diag;
                else
                    kij = kfun(kp, pair_r2<C>(pts, N, d, i, j));
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nc) acc[c] += kij * x[(int64_t)(c0 + c) * N + j];
            }
        }
    }
    for (int o = mp; o < 64; o <<= 1)
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
    if (active && sl == 0) {
        const int64_t u = perm[i];
        for (int c = 0; c < nc; ++c) {
            C s = 0;
            for (int l = 0; l < kappa; ++l) s += ylev[((int64_t)l * nrhs + c0 + c) * N + i];
            Y[(int64_t)(c0 + c) * ldy + u] = (XT)(s + acc[c]);
        }
    }
}

template <typename T>
T* as(void* p) {
    return reinterpret_cast<T*>(p);
}

}  // namespace

void plan_apply(hodlr_t h) {
    // projection: rows of each stored block, 16 per workgroup for short rows
    std::vector<WorkItem> proj;
    for (int64_t b = 0; b < h->nblocks; ++b) {
        const BlockDesc& bd = h->hblocks[b];
        const int per = std::max(bd.m, bd.n) <= 1024 ? 16 : 4;
        for (int k = 0; k < bd.rank; k += per)
            proj.push_back(WorkItem{(int32_t)b, k, std::min(per, bd.rank - k), bd.level});
    }
    // expansion: 64-row chunks of every box of every level
    std::vector<WorkItem> ex;
    for (int l = 1; l <= h->kappa; ++l) {
        const auto& st = h->lev[l].hstart;
        for (int64_t A = 0; A < h->lev[l].nb; ++A)
            for (int32_t i = st[A]; i < st[A + 1]; i += 64)
                ex.push_back(WorkItem{(int32_t)A, i, std::min(64, st[A + 1] - i), l});
    }
    std::vector<WorkItem> nr;
    {
        const auto& st = h->lev[h->kappa].hstart;
        for (int64_t A = 0; A < h->lev[h->kappa].nb; ++A)
            for (int32_t i = st[A]; i < st[A + 1]; i += 64)
                nr.push_back(WorkItem{(int32_t)A, i, std::min(64, st[A + 1] - i), h->kappa});
    }
    auto upload = [&](std::vector<WorkItem>& v, WorkItem** dst) {
        if (*dst) dfree(h, *dst);
        *dst = (WorkItem*)dalloc(h, sizeof(WorkItem) * std::max<size_t>(v.size(), 1));
        if (!v.empty())
            HIP_CHECK(hipMemcpy(*dst, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice));
    };
    upload(proj, &h->proj_items);
    h->n_proj_items = (int64_t)proj.size();
    upload(ex, &h->exp_items);
    h->exp_lvl_off.assign(1, (int64_t)ex.size());
    upload(nr, &h->near_items);
    h->n_near_items = (int64_t)nr.size();
}

namespace {

struct LevelPtrs {
    const int32_t** start;
    const int64_t** ptr;
    const int64_t** ref;
};

template <typename XT, typename S, typename C, int NR>
void run_matvec(hodlr_t h, const XT* X, int64_t ldx, int nrhs, XT* Y, int64_t ldy, char* ws,
                LevelPtrs lp, hipStream_t s) {
    const int64_t N = h->N;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    C* x = (C*)ws;
    C* ylev = x + N * nrhs;
    C* tb = ylev + std::max(h->kappa, 1) * N * nrhs;
    C* sb = tb + TT * nrhs;
    k_permute_in<XT, C><<<nblk(N, 256), 256, 0, s>>>(X, ldx, nrhs, N, h->perm, x);
    HIP_CHECK(hipGetLastError());
    const int sym = h->opts.symmetric ? 1 : 0;
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        if (h->n_proj_items)
            k_project<S, C, NR><<<(unsigned)h->n_proj_items, TP, 0, s>>>(
                h->blocks, h->proj_items, sym, x, N, nrhs, c0, TT, tb, sb);
        const int64_t nex = h->exp_lvl_off[0];
        if (nex)
            k_expand<S, C, NR><<<(unsigned)nex, TE, 0, s>>>(h->blocks, h->exp_items, lp.start,
                                                           lp.ptr, lp.ref, N, nrhs, c0, TT, tb,
                                                           sb, ylev);
        k_near_out<XT, C, NR><<<(unsigned)h->n_near_items, TN, 0, s>>>(
            h->near_items, h->lev[h->kappa].start, h->near_ptr, h->near_col, h->pts, N, h->d,
            h->kp, x, ylev, h->kappa, h->perm, nrhs, c0, Y, ldy);
        HIP_CHECK(hipGetLastError());
    }
}

template <typename XT, typename S, typename C>
void dispatch_nr(hodlr_t h, const XT* X, int64_t ldx, int nrhs, XT* Y, int64_t ldy, char* ws,
                 LevelPtrs lp, hipStream_t s) {
    if (nrhs == 1)
        run_matvec<XT, S, C, 1>(h, X, ldx, nrhs, Y, ldy, ws, lp, s);
    else if (nrhs <= 4)
        run_matvec<XT, S, C, 4>(h, X, ldx, nrhs, Y, ldy, ws, lp, s);
    else
        run_matvec<XT, S, C, 8>(h, X, ldx, nrhs, Y, ldy, ws, lp, s);
}

}  // namespace

void matvec(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y, int64_t ldy,
            int compute_prec, hipStream_t s) {
    const int64_t N = h->N;
    const size_t cs = compute_prec == HODLR_FP32 ? 4 : 8;
    const int64_t TT = std::max<int64_t>(h->t_total, 1);
    const size_t need =
        cs * ((size_t)N * nrhs * (1 + std::max(h->kappa, 1)) + 2 * (size_t)TT * nrhs) + 4096;
    // level tables (device arrays of per-level device pointers) live at the end
    const size_t tbl = 3 * sizeof(void*) * kMaxLevels;
    if (h->ws_bytes < need + tbl) {
        if (h->ws) {
            HIP_CHECK(hipStreamSynchronize(s));
            dfree(h, h->ws);
        }
        h->ws = dalloc(h, need + tbl);
        h->ws_bytes = need + tbl;
        const void* ptrs[3 * kMaxLevels] = {nullptr};
        for (int l = 1; l <= h->kappa; ++l) {
            ptrs[l] = h->lev[l].start;
            ptrs[kMaxLevels + l] = h->lev[l].il_ptr;
            ptrs[2 * kMaxLevels + l] = h->lev[l].eref;
        }
        HIP_CHECK(hipMemcpy((char*)h->ws + h->ws_bytes - tbl, ptrs, tbl, hipMemcpyHostToDevice));
    }
    char* tblp = (char*)h->ws + h->ws_bytes - tbl;
    LevelPtrs lp{(const int32_t**)tblp, (const int64_t**)(tblp + sizeof(void*) * kMaxLevels),
                 (const int64_t**)(tblp + 2 * sizeof(void*) * kMaxLevels)};
    char* ws = (char*)h->ws;
    const bool s32 = h->opts.storage == HODLR_FP32;
    const bool c32 = compute_prec == HODLR_FP32;
    if (x_prec == HODLR_FP64) {
        const double* Xd = (const double*)X;
        double* Yd = (double*)Y;
        if (!s32 && !c32) dispatch_nr<double, double, double>(h, Xd, ldx, nrhs, Yd, ldy, ws, lp, s);
        else if (!s32 && c32) dispatch_nr<double, double, float>(h, Xd, ldx, nrhs, Yd, ldy, ws, lp, s);
        else if (s32 && !c32) dispatch_nr<double, float, double>(h, Xd, ldx, nrhs, Yd, ldy, ws, lp, s);
        else dispatch_nr<double, float, float>(h, Xd, ldx, nrhs, Yd, ldy, ws, lp, s);
    } else {
        const float* Xf = (const float*)X;
        float* Yf = (float*)Y;
        if (!s32 && !c32) dispatch_nr<float, double, double>(h, Xf, ldx, nrhs, Yf, ldy, ws, lp, s);
        else if (!s32 && c32) dispatch_nr<float, double, float>(h, Xf, ldx, nrhs, Yf, ldy, ws, lp, s);
        else if (s32 && !c32) dispatch_nr<float, float, double>(h, Xf, ldx, nrhs, Yf, ldy, ws, lp, s);
        else dispatch_nr<float, float, float>(h, Xf, ldx, nrhs, Yf, ldy, ws, lp, s);
    }
}

}  // namespace hodlr
