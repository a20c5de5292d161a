// Interaction lists of every level and near lists of the leaves (paper
// sec. 5.3: table of notations and the HODLRdD admissibility definition),
// plus the table of stored low-rank blocks.
//
// IL(A) at level l: boxes B != A whose parent Q equals A's parent P or shares
// a hyper-surface of dimension >= 1 with P (the parent's vertex-sharing
// neighbours were compressed one level up), and which share at most a vertex
// with A (vertex-sharing) or lie at least one box away (far field).
// near(A) at the leaves: A and the boxes sharing a hyper-surface of dimension
// 1..d-1 with A.  Candidates are enumerated from the parent's 3^d
// neighbourhood; the children of a box are a contiguous key range, found by
// binary search in the level's sorted keys.  Rows are sorted afterwards.
// Adaptive tree (sec. 5.2 names it beside the balanced tree): only active
// boxes (parent subdivided) take part; a pair that is not admissible is a
// dense near-field pair of its level when either box is a leaf, so near
// lists exist on every level that has leaves.
#include <algorithm>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int T = 128;

__device__ __forceinline__ uint64_t interleave(const int32_t* c, int level, int d) {
    uint64_t k = 0;
    for (int bit = level - 1; bit >= 0; --bit)
        for (int a = 0; a < d; ++a) k = (k << 1) | (uint64_t)((c[a] >> bit) & 1);
    return k;
}

__device__ __forceinline__ int64_t lower_bound(const uint64_t* __restrict__ key, int64_t n,
                                               uint64_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (key[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// count (ptr == nullptr: out[A] = count) or fill (out = columns)
__global__ void k_il(int level, int d, int adm, int64_t nb, const uint64_t* __restrict__ key,
                     const int32_t* __restrict__ coord, const uint8_t* __restrict__ flags,
                     const int64_t* __restrict__ ptr, int32_t* __restrict__ out) {
    int64_t A = blockIdx.x * (int64_t)T + threadIdx.x;
    if (A >= nb) return;
    if (!(flags[A] & 1)) {   // below a leaf: no lists
        if (!ptr) out[A] = 0;
        return;
    }
    int32_t a[kMaxD], P[kMaxD], Q[kMaxD];
    for (int k = 0; k < d; ++k) {
        a[k] = coord[A * d + k];
        P[k] = a[k] >> 1;
    }
    const int32_t np = 1 << (level - 1);
    int ncand = 1;
    for (int k = 0; k < d; ++k) ncand *= 3;
    int64_t cnt = 0;
    const int64_t base = ptr ? ptr[A] : 0;
    for (int t = 0; t < ncand; ++t) {
        int tt = t;
        bool ok = true;
        int nzero = 0;
        for (int k = 0; k < d; ++k) {
            int dl = tt % 3 - 1;
            tt /= 3;
            Q[k] = P[k] + dl;
            if (Q[k] < 0 || Q[k] >= np) ok = false;
            if (dl == 0) ++nzero;
        }
        // the parents' pair must not be admissible itself: the same parent,
        // or neighbours sharing a hyper-surface of dimension > adm
        if (!ok || nzero <= adm) continue;
        const uint64_t kq = interleave(Q, level - 1, d);
        const int64_t lo = lower_bound(key, nb, kq << d);
        const int64_t hi = lower_bound(key, nb, (kq + 1) << d);
        for (int64_t B = lo; B < hi; ++B) {
            if (B == A || !(flags[B] & 1)) continue;
            int mx = 0, eq = 0;
            for (int k = 0; k < d; ++k) {
                int dc = abs(coord[B * d + k] - a[k]);
                mx = max(mx, dc);
                if (dc == 0) ++eq;
            }
            // admissible: far apart, or adjacent sharing a hyper-surface of
            // dimension <= adm (adm = 0: vertex sharing)
            if (mx >= 2 || (mx == 1 && eq <= adm)) {
                if (ptr) out[base + cnt] = (int32_t)B;
                ++cnt;
            }
        }
    }
    if (!ptr) out[A] = (int32_t)cnt;
}

__global__ void k_near(int level, int d, int adm, int64_t nb, const uint64_t* __restrict__ key,
                       const int32_t* __restrict__ coord, const uint8_t* __restrict__ flags,
                       const int64_t* __restrict__ ptr, int32_t* __restrict__ out) {
    int64_t A = blockIdx.x * (int64_t)T + threadIdx.x;
    if (A >= nb) return;
    const int fa = flags[A];
    if (!(fa & 1)) {
        if (!ptr) out[A] = 0;
        return;
    }
    int32_t a[kMaxD], B[kMaxD];
    for (int k = 0; k < d; ++k) a[k] = coord[A * d + k];
    const int32_t ns = 1 << level;
    int ncand = 1;
    for (int k = 0; k < d; ++k) ncand *= 3;
    int64_t cnt = 0;
    const int64_t base = ptr ? ptr[A] : 0;
    for (int t = 0; t < ncand; ++t) {
        int tt = t;
        bool ok = true;
        int nzero = 0;
        for (int k = 0; k < d; ++k) {
            int dl = tt % 3 - 1;
            tt /= 3;
            B[k] = a[k] + dl;
            if (B[k] < 0 || B[k] >= ns) ok = false;
            if (dl == 0) ++nzero;
        }
        // the box itself and the adjacent boxes that are not admissible
        if (!ok || nzero <= adm) continue;
        const uint64_t kb = interleave(B, level, d);
        const int64_t pos = lower_bound(key, nb, kb);
        // both active, and not subdivided further: one of them is a leaf
        if (pos < nb && key[pos] == kb && (flags[pos] & 1) && ((fa | flags[pos]) & 2)) {
            if (ptr) out[base + cnt] = (int32_t)pos;
            ++cnt;
        }
    }
    if (!ptr) out[A] = (int32_t)cnt;
}

__global__ void k_widen(const int32_t* __restrict__ in, int64_t* __restrict__ out, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)T + threadIdx.x;
    if (i < n) out[i] = in[i];
}

__global__ void k_set_last(int64_t* ptr, int64_t nb, const int32_t* cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ptr[nb] = nb ? ptr[nb - 1] + cnt[nb - 1] : 0;
}

__global__ void k_row_of_entry(const int64_t* __restrict__ ptr, int64_t nb,
                               int32_t* __restrict__ row) {
    int64_t A = blockIdx.x * (int64_t)T + threadIdx.x;
    if (A >= nb) return;
    for (int64_t e = ptr[A]; e < ptr[A + 1]; ++e) row[e] = (int32_t)A;
}

__global__ void k_mark_stored(const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                              int64_t nnz, int sym, int64_t* __restrict__ flag) {
    int64_t e = blockIdx.x * (int64_t)T + threadIdx.x;
    if (e >= nnz) return;
    flag[e] = (!sym || row[e] < col[e]) ? 1 : 0;
}

__global__ void k_fill_blocks(const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                              const int64_t* __restrict__ flag, const int64_t* __restrict__ bid,
                              int64_t nnz, const int32_t* __restrict__ start, int level,
                              int64_t blk0, BlockDesc* __restrict__ blocks,
                              int64_t* __restrict__ eref) {
    int64_t e = blockIdx.x * (int64_t)T + threadIdx.x;
    if (e >= nnz || !flag[e]) return;
    const int32_t A = row[e], B = col[e];
    BlockDesc b;
    b.a0 = start[A];
    b.m = start[A + 1] - start[A];
    b.b0 = start[B];
    b.n = start[B + 1] - start[B];
    b.rank = -1;
    b.level = level;
    b.toff = 0;
    b.U = 0;
    b.V = 0;
    b.cfwd = -1;
    b.cbwd = -1;
    blocks[blk0 + bid[e]] = b;
    eref[e] = (blk0 + bid[e]) << 1;
}

// entry (A,B) with A > B uses the stored block of (B,A), transposed
__global__ void k_fill_back(const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                            const int64_t* __restrict__ ptr, const int64_t* __restrict__ bid,
                            int64_t nnz, int64_t blk0, int64_t* __restrict__ eref,
                            int* __restrict__ err) {
    int64_t e = blockIdx.x * (int64_t)T + threadIdx.x;
    if (e >= nnz) return;
    const int32_t A = row[e], B = col[e];
    if (A < B) return;
    int64_t lo = ptr[B], hi = ptr[B + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < A)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo >= ptr[B + 1] || col[lo] != A) {
        atomicOr(err, 1);
        return;
    }
    eref[e] = ((blk0 + bid[lo]) << 1) | 1;
}

// CSR rows: count, scan, fill, sort every row
void build_csr(hodlr_t h, int level, bool near, int64_t** ptr_out, int32_t** col_out,
               int64_t* nnz_out, hipStream_t s) {
    LevelData& Lv = h->lev[level];
    const int64_t nb = Lv.nb;
    int32_t* cnt = (int32_t*)dalloc(h, sizeof(int32_t) * (nb + 1));
    int32_t* off32 = (int32_t*)dalloc(h, sizeof(int32_t) * (nb + 1));
    int64_t* ptr = (int64_t*)dalloc(h, sizeof(int64_t) * (nb + 1));
    if (near)
        k_near<<<nblk(nb, T), T, 0, s>>>(level, h->d, h->opts.adm_dim, nb, Lv.key, Lv.coord,
                                         Lv.flags, nullptr, cnt);
    else
        k_il<<<nblk(nb, T), T, 0, s>>>(level, h->d, h->opts.adm_dim, nb, Lv.key, Lv.coord,
                                       Lv.flags, nullptr, cnt);
    HIP_CHECK(hipGetLastError());
    // row counts fit in 32 bits; the offsets are widened before they can overflow
    int64_t* cnt64 = (int64_t*)dalloc(h, sizeof(int64_t) * (nb + 1));
    k_widen<<<nblk(nb, T), T, 0, s>>>(cnt, cnt64, nb);
    HIP_CHECK(hipGetLastError());
    exclusive_scan_i64(cnt64, ptr, nb, s);
    k_set_last<<<1, 1, 0, s>>>(ptr, nb, cnt);
    HIP_CHECK(hipGetLastError());
    int64_t nnz = 0;
    HIP_CHECK(hipMemcpyAsync(&nnz, ptr + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (nnz >= (int64_t)1 << 32) fail(HODLR_EUNSUPPORTED, "interaction list too long");
    int32_t* col = (int32_t*)dalloc(h, sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    int32_t* tmp = (int32_t*)dalloc(h, sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    if (near)
        k_near<<<nblk(nb, T), T, 0, s>>>(level, h->d, h->opts.adm_dim, nb, Lv.key, Lv.coord,
                                         Lv.flags, ptr, tmp);
    else
        k_il<<<nblk(nb, T), T, 0, s>>>(level, h->d, h->opts.adm_dim, nb, Lv.key, Lv.coord,
                                       Lv.flags, ptr, tmp);
    HIP_CHECK(hipGetLastError());
    if (nnz > 0) segmented_sort_i32(tmp, col, nnz, nb, ptr, s);
    dfree(h, tmp);
    dfree(h, cnt);
    dfree(h, cnt64);
    dfree(h, off32);
    *ptr_out = ptr;
    *col_out = col;
    *nnz_out = nnz;
}

}  // namespace

void build_lists(hodlr_t h, hipStream_t s) {
    for (int l = 1; l <= h->kappa; ++l)
        build_csr(h, l, false, &h->lev[l].il_ptr, &h->lev[l].il_col, &h->lev[l].nnz, s);
    // dense pairs: on level kappa only in a uniform tree (the other levels
    // have no leaves, their rows stay empty), on every level in an adaptive one
    int64_t pairs = 0;
    for (int l = 0; l <= h->kappa; ++l) {
        LevelData& Lk = h->lev[l];
        build_csr(h, l, true, &Lk.near_ptr, &Lk.near_col, &Lk.near_nnz, s);
        // number of point pairs of the near field (reported by hodlr_get_info)
        if (!Lk.near_nnz) continue;
        std::vector<int64_t> ptr(Lk.nb + 1);
        std::vector<int32_t> col(Lk.near_nnz);
        HIP_CHECK(hipMemcpyAsync(ptr.data(), Lk.near_ptr, sizeof(int64_t) * (Lk.nb + 1),
                                 hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(col.data(), Lk.near_col, sizeof(int32_t) * Lk.near_nnz,
                                 hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        for (int64_t A = 0; A < Lk.nb; ++A) {
            int64_t m = Lk.hstart[A + 1] - Lk.hstart[A];
            for (int64_t e = ptr[A]; e < ptr[A + 1]; ++e)
                pairs += m * (Lk.hstart[col[e] + 1] - Lk.hstart[col[e]]);
        }
    }
    h->near_ptr = h->lev[h->kappa].near_ptr;
    h->near_col = h->lev[h->kappa].near_col;
    h->near_nnz = h->lev[h->kappa].near_nnz;
    h->near_pairs = pairs;
}

void build_block_table(hodlr_t h, hipStream_t s) {
    const int sym = h->opts.symmetric ? 1 : 0;
    std::vector<int64_t> nstored(h->kappa + 1, 0);
    std::vector<int32_t*> rows(h->kappa + 1, nullptr);
    std::vector<int64_t*> flags(h->kappa + 1, nullptr), bids(h->kappa + 1, nullptr);
    int64_t total = 0;
    for (int l = 1; l <= h->kappa; ++l) {
        LevelData& Lv = h->lev[l];
        const int64_t nnz = Lv.nnz;
        Lv.blk0 = total;
        if (nnz == 0) continue;
        rows[l] = (int32_t*)dalloc(h, sizeof(int32_t) * nnz);
        flags[l] = (int64_t*)dalloc(h, sizeof(int64_t) * nnz);
        bids[l] = (int64_t*)dalloc(h, sizeof(int64_t) * nnz);
        k_row_of_entry<<<nblk(Lv.nb, T), T, 0, s>>>(Lv.il_ptr, Lv.nb, rows[l]);
        k_mark_stored<<<nblk(nnz, T), T, 0, s>>>(rows[l], Lv.il_col, nnz, sym, flags[l]);
        HIP_CHECK(hipGetLastError());
        exclusive_scan_i64(flags[l], bids[l], nnz, s);
        int64_t lastb = 0, lastf = 0;
        HIP_CHECK(hipMemcpyAsync(&lastb, bids[l] + nnz - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(&lastf, flags[l] + nnz - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        nstored[l] = lastb + lastf;
        Lv.nblk = nstored[l];
        total += nstored[l];
    }
    h->nblocks = total;
    h->blocks = (BlockDesc*)dalloc(h, sizeof(BlockDesc) * std::max<int64_t>(total, 1));
    int* err = (int*)dalloc(h, sizeof(int));
    HIP_CHECK(hipMemsetAsync(err, 0, sizeof(int), s));
    for (int l = 1; l <= h->kappa; ++l) {
        LevelData& Lv = h->lev[l];
        const int64_t nnz = Lv.nnz;
        Lv.eref = (int64_t*)dalloc(h, sizeof(int64_t) * std::max<int64_t>(nnz, 1));
        if (nnz == 0) continue;
        k_fill_blocks<<<nblk(nnz, T), T, 0, s>>>(rows[l], Lv.il_col, flags[l], bids[l], nnz,
                                                 Lv.start, l, Lv.blk0, h->blocks, Lv.eref);
        if (sym)
            k_fill_back<<<nblk(nnz, T), T, 0, s>>>(rows[l], Lv.il_col, Lv.il_ptr, bids[l], nnz,
                                                   Lv.blk0, Lv.eref, err);
        HIP_CHECK(hipGetLastError());
    }
    int herr = 0;
    HIP_CHECK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (herr) fail(HODLR_EDEVICE, "interaction list is not symmetric");
    for (int l = 1; l <= h->kappa; ++l) {
        if (rows[l]) dfree(h, rows[l]);
        if (flags[l]) dfree(h, flags[l]);
        if (bids[l]) dfree(h, bids[l]);
    }
    dfree(h, err);
    h->hblocks.resize(total);
    if (total)
        HIP_CHECK(hipMemcpyAsync(h->hblocks.data(), h->blocks, sizeof(BlockDesc) * total,
                                 hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace hodlr
