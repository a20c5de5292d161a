// Computational hyper-cube, Morton keys, sort and per-level boxes of the 2^d
// tree (paper sec. 5.2).  Integer results must equal the oracle's bit for
// bit, so the floating-point steps are exactly one IEEE subtraction, one
// IEEE division, an exact power-of-two scaling and a floor.
#include <algorithm>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int T = 256;

// flags[0]: non-finite coordinate; flags[1]: point outside the explicit cube
__global__ void k_check(const double* __restrict__ P, int64_t n_elem, int d, int has_domain,
                        const double* __restrict__ lo_side, int* flags) {
    for (int64_t e = blockIdx.x * (int64_t)T + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * T) {
        double x = P[e];
        if (!isfinite(x)) atomicOr(&flags[0], 1);
        if (has_domain) {
            int a = (int)(e % d);
            double lo = lo_side[a], side = lo_side[8];
            if (!(x >= lo && x <= lo + side)) atomicOr(&flags[1], 1);
        }
    }
}

// per-workgroup min/max of every coordinate
__global__ void k_bbox_partial(const double* __restrict__ P, int64_t N, int d,
                               double* __restrict__ pmin, double* __restrict__ pmax) {
    __shared__ double smin[T], smax[T];
    for (int a = 0; a < d; ++a) {
        double mn = INFINITY, mx = -INFINITY;
        for (int64_t i = blockIdx.x * (int64_t)T + threadIdx.x; i < N;
             i += (int64_t)gridDim.x * T) {
            double x = P[i * d + a];
            mn = fmin(mn, x);
            mx = fmax(mx, x);
        }
        smin[threadIdx.x] = mn;
        smax[threadIdx.x] = mx;
        __syncthreads();
        for (int s = T / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
                smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            pmin[blockIdx.x * kMaxD + a] = smin[0];
            pmax[blockIdx.x * kMaxD + a] = smax[0];
        }
        __syncthreads();
    }
}

// bounding cube: lo = min per coordinate, side = largest extent (1 if 0)
__global__ void k_bbox_final(const double* __restrict__ pmin, const double* __restrict__ pmax,
                             int nparts, int d, double* lo_side) {
    if (threadIdx.x != 0) return;
    double side = 0.0;
    for (int a = 0; a < d; ++a) {
        double mn = pmin[a], mx = pmax[a];
        for (int b = 1; b < nparts; ++b) {
            mn = fmin(mn, pmin[b * kMaxD + a]);
            mx = fmax(mx, pmax[b * kMaxD + a]);
        }
        lo_side[a] = mn;
        double w = mx - mn;
        if (w > side) side = w;
    }
    lo_side[8] = side > 0.0 ? side : 1.0;
}

__global__ void k_keys(const double* __restrict__ P, int64_t N, int d, int L,
                       const double* __restrict__ lo_side, uint64_t* __restrict__ keys,
                       int32_t* __restrict__ idx) {
    int64_t i = blockIdx.x * (int64_t)T + threadIdx.x;
    if (i >= N) return;
    const int64_t qmax = ((int64_t)1 << L) - 1;
    const double side = lo_side[8];
    int64_t q[kMaxD];
    for (int a = 0; a < d; ++a) {
        double t = (P[i * d + a] - lo_side[a]) / side;
        double f = floor(ldexp(t, L));
        int64_t qi = (int64_t)f;
        qi = qi < 0 ? 0 : (qi > qmax ? qmax : qi);
        q[a] = qi;
    }
    uint64_t key = 0;
    for (int b = L - 1; b >= 0; --b)
        for (int a = 0; a < d; ++a) key = (key << 1) | (uint64_t)((q[a] >> b) & 1);
    keys[i] = key;
    idx[i] = (int32_t)i;
}

// tree-order SoA copy of the points
__global__ void k_gather_pts(const double* __restrict__ P, const int32_t* __restrict__ perm,
                             int64_t N, int d, double* __restrict__ pts) {
    int64_t p = blockIdx.x * (int64_t)T + threadIdx.x;
    if (p >= N) return;
    int64_t i = perm[p];
    for (int a = 0; a < d; ++a) pts[a * N + p] = P[i * d + a];
}

// coincident distinct points: they share their finest cell, hence key runs
__global__ void k_dups(const double* __restrict__ pts, const uint64_t* __restrict__ keys,
                       int64_t N, int d, int* flag) {
    int64_t p = blockIdx.x * (int64_t)T + threadIdx.x;
    if (p >= N) return;
    for (int64_t q = p + 1; q < N && keys[q] == keys[p]; ++q) {
        bool same = true;
        for (int a = 0; a < d; ++a) same = same && (pts[a * N + p] == pts[a * N + q]);
        if (same) {
            atomicOr(flag, 1);
            return;
        }
    }
}

__global__ void k_level_flags(const uint64_t* __restrict__ keys, int64_t N, int shift,
                              int32_t* __restrict__ flag) {
    int64_t p = blockIdx.x * (int64_t)T + threadIdx.x;
    if (p >= N) return;
    flag[p] = (p == 0 || (keys[p] >> shift) != (keys[p - 1] >> shift)) ? 1 : 0;
}

// box b of the level starts at the b-th flagged position; its integer
// coordinates are the de-interleaved bits of its level key
__global__ void k_level_boxes(const uint64_t* __restrict__ keys, const int32_t* __restrict__ flag,
                              const int32_t* __restrict__ pos, int64_t N, int shift, int d,
                              int level, int64_t nb, int32_t* __restrict__ start,
                              uint64_t* __restrict__ bkey, int32_t* __restrict__ coord) {
    int64_t p = blockIdx.x * (int64_t)T + threadIdx.x;
    if (p == 0) start[nb] = (int32_t)N;
    if (p >= N || !flag[p]) return;
    int64_t b = pos[p];
    uint64_t k = keys[p] >> shift;
    start[b] = (int32_t)p;
    bkey[b] = k;
    for (int a = 0; a < d; ++a) {
        int32_t c = 0;
        for (int bit = level - 1; bit >= 0; --bit)
            c = (c << 1) | (int32_t)((k >> (bit * d + (d - 1 - a))) & 1);
        coord[b * d + a] = c;
    }
}

__global__ void k_max_count(const int32_t* __restrict__ start, int64_t nb, int* out) {
    int64_t b = blockIdx.x * (int64_t)T + threadIdx.x;
    if (b >= nb) return;
    atomicMax(out, start[b + 1] - start[b]);
}

}  // namespace

void build_tree(hodlr_t h, const double* points_in, hipStream_t s) {
    const int64_t N = h->N;
    const int d = h->d;
    const int L = std::min(63 / d, 30);
    h->lmax = L;

    double* P = (double*)dalloc(h, sizeof(double) * N * d);
    double* lo_side = (double*)dalloc(h, sizeof(double) * 16);
    int* flags = (int*)dalloc(h, sizeof(int) * 4);
    HIP_CHECK(hipMemcpyAsync(P, points_in, sizeof(double) * N * d, hipMemcpyDefault, s));
    HIP_CHECK(hipMemsetAsync(flags, 0, sizeof(int) * 4, s));
    double ls_host[16] = {0};
    if (h->opts.has_domain) {
        for (int a = 0; a < d; ++a) ls_host[a] = h->opts.domain_lo[a];
        ls_host[8] = h->opts.domain_side;
        HIP_CHECK(hipMemcpyAsync(lo_side, ls_host, sizeof(ls_host), hipMemcpyHostToDevice, s));
    }
    const unsigned gchk = std::min<unsigned>(nblk(N * d, T), 4096u);
    k_check<<<gchk, T, 0, s>>>(P, N * d, d, h->opts.has_domain, lo_side, flags);
    HIP_CHECK(hipGetLastError());
    int fl[4];
    HIP_CHECK(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (fl[0]) fail(HODLR_ENONFINITE, "points contain NaN or Inf");
    if (fl[1]) fail(HODLR_EINVAL, "a point lies outside the given hyper-cube");

    if (!h->opts.has_domain) {
        const int parts = (int)std::min<int64_t>(nblk(N, T), 1024);
        double* pmin = (double*)dalloc(h, sizeof(double) * parts * kMaxD);
        double* pmax = (double*)dalloc(h, sizeof(double) * parts * kMaxD);
        k_bbox_partial<<<parts, T, 0, s>>>(P, N, d, pmin, pmax);
        k_bbox_final<<<1, 64, 0, s>>>(pmin, pmax, parts, d, lo_side);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(ls_host, lo_side, sizeof(ls_host), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        dfree(h, pmin);
        dfree(h, pmax);
    }
    for (int a = 0; a < d; ++a) h->lo[a] = ls_host[a];
    h->side = ls_host[8];

    uint64_t* kraw = (uint64_t*)dalloc(h, sizeof(uint64_t) * N);
    int32_t* iraw = (int32_t*)dalloc(h, sizeof(int32_t) * N);
    h->keys = (uint64_t*)dalloc(h, sizeof(uint64_t) * N);
    h->perm = (int32_t*)dalloc(h, sizeof(int32_t) * N);
    k_keys<<<nblk(N, T), T, 0, s>>>(P, N, d, L, lo_side, kraw, iraw);
    HIP_CHECK(hipGetLastError());
    // LSD radix sort is stable: equal keys keep ascending original index
    sort_pairs_u64(kraw, h->keys, iraw, h->perm, N, d * L, s);
    dfree(h, kraw);
    dfree(h, iraw);

    h->pts = (double*)dalloc(h, sizeof(double) * N * d);
    k_gather_pts<<<nblk(N, T), T, 0, s>>>(P, h->perm, N, d, h->pts);
    HIP_CHECK(hipGetLastError());
    dfree(h, P);

    const int kind = h->kern.kind;
    if (kind == HODLR_K_LOG || kind == HODLR_K_INV_R || kind == HODLR_K_INV_R2) {
        HIP_CHECK(hipMemsetAsync(flags, 0, sizeof(int), s));
        k_dups<<<nblk(N, T), T, 0, s>>>(h->pts, h->keys, N, d, flags);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(fl, flags, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (fl[0]) fail(HODLR_EDUPLICATE, "coincident points under a singular kernel");
    }

    // levels 0, 1, ... until the depth rule is met
    int32_t* flag = (int32_t*)dalloc(h, sizeof(int32_t) * N);
    int32_t* pos = (int32_t*)dalloc(h, sizeof(int32_t) * N);
    int kappa_cf = 0;
    if (h->opts.level_rule == 1) {
        while (kappa_cf < L) {
            int bits = d * kappa_cf;
            if (bits >= 62) break;
            int64_t need = (N + ((int64_t)1 << bits) - 1) >> bits;
            if ((int64_t)h->leaf >= need) break;
            ++kappa_cf;
        }
    }
    int l = 0;
    for (;; ++l) {
        const int shift = d * (L - l);
        k_level_flags<<<nblk(N, T), T, 0, s>>>(h->keys, N, shift, flag);
        HIP_CHECK(hipGetLastError());
        exclusive_scan_i32(flag, pos, N, s);
        int32_t last[2];
        HIP_CHECK(hipMemcpyAsync(&last[0], pos + N - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(&last[1], flag + N - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        const int64_t nb = (int64_t)last[0] + last[1];
        LevelData& Lv = h->lev[l];
        Lv.nb = nb;
        Lv.start = (int32_t*)dalloc(h, sizeof(int32_t) * (nb + 1));
        Lv.key = (uint64_t*)dalloc(h, sizeof(uint64_t) * nb);
        Lv.coord = (int32_t*)dalloc(h, sizeof(int32_t) * nb * d);
        k_level_boxes<<<nblk(N, T), T, 0, s>>>(h->keys, flag, pos, N, shift, d, l, nb, Lv.start,
                                               Lv.key, Lv.coord);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemsetAsync(flags, 0, sizeof(int), s));
        k_max_count<<<nblk(nb, T), T, 0, s>>>(Lv.start, nb, flags);
        HIP_CHECK(hipGetLastError());
        Lv.hstart.resize(nb + 1);
        HIP_CHECK(hipMemcpyAsync(Lv.hstart.data(), Lv.start, sizeof(int32_t) * (nb + 1),
                                 hipMemcpyDeviceToHost, s));
        int maxc = 0;
        HIP_CHECK(hipMemcpyAsync(&maxc, flags, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        bool stop;
        if (h->opts.level_rule == 1)
            stop = (l >= kappa_cf);
        else
            stop = (maxc <= h->leaf) || (l >= L);
        if (stop) break;
        if (l + 1 >= kMaxLevels) fail(HODLR_EUNSUPPORTED, "tree deeper than 31 levels");
    }
    h->kappa = l;
    // active and leaf boxes (uniform rules: all active, leaves on level kappa;
    // adaptive rule: a box is active when its parent holds more than `leaf`
    // points, and an active box is a leaf when it holds at most `leaf` points
    // or lies on level kappa)
    for (int lv = 0; lv <= h->kappa; ++lv) {
        LevelData& Lv = h->lev[lv];
        Lv.hflags.assign((size_t)Lv.nb, 0);
        const std::vector<int32_t>* ps = lv > 0 ? &h->lev[lv - 1].hstart : nullptr;
        int64_t par = 0;
        for (int64_t A = 0; A < Lv.nb; ++A) {
            const int32_t cnt = Lv.hstart[A + 1] - Lv.hstart[A];
            bool act, lf;
            if (h->opts.level_rule != 2) {
                act = true;
                lf = lv == h->kappa;
            } else {
                act = true;
                if (ps) {
                    while ((*ps)[par + 1] <= Lv.hstart[A]) ++par;
                    act = (*ps)[par + 1] - (*ps)[par] > h->leaf;
                }
                lf = act && (cnt <= h->leaf || lv == h->kappa);
            }
            Lv.hflags[A] = (uint8_t)((act ? 1 : 0) | (lf ? 2 : 0));
        }
        Lv.flags = (uint8_t*)dalloc(h, std::max<size_t>((size_t)Lv.nb, 1));
        if (Lv.nb)
            HIP_CHECK(hipMemcpyAsync(Lv.flags, Lv.hflags.data(), (size_t)Lv.nb,
                                     hipMemcpyHostToDevice, s));
    }
    HIP_CHECK(hipStreamSynchronize(s));
    dfree(h, flag);
    dfree(h, pos);
    dfree(h, lo_side);
    dfree(h, flags);
}

}  // namespace hodlr
