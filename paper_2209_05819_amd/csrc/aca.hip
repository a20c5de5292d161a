// ACA compression of every stored interaction-list block (paper eq. keq1,
// Alg. "HODLRdD Initialization"): partial-pivot cross approximation in FP64,
// one workgroup per block.  Small blocks keep their factors in LDS for the
// whole iteration; larger ones iterate in a global FP64 workspace.  Finished
// factors are packed into per-chunk arenas in the storage precision.
//
// The iteration:
//   row residual of pivot row i*, column pivot j* = largest |entry| (lowest
//   index on ties); a zero pivot marks the row tried and restarts from the
//   lowest untried row; otherwise v = row / pivot, u = residual of column j*.
//   The candidate term u v is small when |u||v| <= tol * |S|_F with S the
//   approximation including it.  A small term ends the iteration, dropped,
//   only if sampled residuals of the approximation without it confirm the
//   tolerance: 16 evenly spaced rows and 16 evenly spaced columns (every one
//   in a smaller block; the c-th check of a block shifts them by 997c and
//   991c modulo the spacing), each sum of squares scaled up to an estimate of
//   |K - S|_F^2, both at most (tol/2)^2 |S|_F^2.  Otherwise the term is kept
//   and the next pivot row is the untried row holding the largest sampled
//   residual entry (lowest row on ties).  Without a check the next pivot row
//   is the untried row with the largest |u_i|.  The per-term stop alone
//   underestimates the error of large blocks whose residual gathers near a
//   shared vertex, and the product then misses the tolerance.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <climits>

#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int T = 256;
constexpr int NW = T / 64;
constexpr int kAcaSamples = 16;   // rows and columns sampled to confirm a stop

struct AcaJob {
    int32_t a0, m, b0, n;
    int32_t kmax;   // min(m, n, max_rank)
    int32_t cap;    // columns available in the workspace
    int64_t ws;     // offset (in doubles) of the job's workspace
    int64_t block;  // global block index
    int64_t pv;     // offset of the job's pivot pairs (row, column) per term
};

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// larger |value| wins, ties -> lower index
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(v, o, 64);
        int oi = __shfl_xor(i, o, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

template <bool kLds>
__global__ __launch_bounds__(T) void k_aca(const double* __restrict__ pts, int64_t N, int d,
                                           KParams kp, double tol, const AcaJob* __restrict__ jobs,
                                           double* __restrict__ wsbase, int32_t* __restrict__ ranks,
                                           int32_t* __restrict__ overflow,
                                           int32_t* __restrict__ pivots,
                                           double* __restrict__ tsize,
                                           double* __restrict__ s2out) {
    extern __shared__ double dyn[];
    __shared__ double red_v[NW], red_w[NW], red_x[NW];
    __shared__ int red_i[NW], red_j[NW];
    __shared__ int sh_k, sh_istar, sh_nused, sh_done, sh_jstar, sh_small, sh_ix, sh_next,
        sh_checks;
    __shared__ double sh_S2, sh_piv, sh_S2new, sh_tsize;

    const AcaJob J = jobs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = J.m, n = J.n;
    const int kcap = min(J.kmax, J.cap);
    double* s_a = dyn;            // U[p][i*] then cross products
    double* s_b = dyn + J.cap;    // V[p][j*]
    double* ws = wsbase + J.ws;
    double* U;
    double* V;
    unsigned char* used;
    if (kLds) {
        U = dyn + 2 * J.cap;
        V = U + (int64_t)J.cap * m;
        used = reinterpret_cast<unsigned char*>(V + (int64_t)J.cap * n);
    } else {
        U = ws;
        V = ws + (int64_t)J.cap * m;
        used = reinterpret_cast<unsigned char*>(V + (int64_t)J.cap * n);
    }
    const double* __restrict__ X = pts + J.a0;   // coordinate a of row i: X[a*N + i]
    const double* __restrict__ Y = pts + J.b0;

    for (int i = tid; i < m; i += T) used[i] = 0;
    if (tid == 0) {
        sh_k = 0;
        sh_istar = 0;
        sh_nused = 0;
        sh_done = 0;
        sh_checks = 0;
        sh_S2 = 0.0;
    }
    __syncthreads();
    int ovf = 0;
    for (;;) {
        const int k = sh_k;
        const int istar = sh_istar;
        if (k >= kcap) {
            ovf = (k < J.kmax) ? 1 : 0;
            break;
        }
        for (int p = tid; p < k; p += T) s_a[p] = U[(int64_t)p * m + istar];
        double xi[kMaxD];
        for (int a = 0; a < d; ++a) xi[a] = X[a * N + istar];
        __syncthreads();
        // residual of the pivot row, written as row k of V
        double bv = -1.0;
        int bi = INT_MAX;
        double* Vk = V + (int64_t)k * n;
        for (int j = tid; j < n; j += T) {
            double r2 = 0.0;
            for (int a = 0; a < d; ++a) {
                double t = xi[a] - Y[a * N + j];
                r2 += t * t;
            }
            double v = kfun(kp, r2);
            for (int p = 0; p < k; ++p) v -= s_a[p] * V[(int64_t)p * n + j];
            Vk[j] = v;
            double av = fabs(v);
            if (av > bv) {
                bv = av;
                bi = j;
            }
        }
        wave_argmax(bv, bi);
        if (lane == 0) {
            red_v[wv] = bv;
            red_i[wv] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double b = red_v[0];
            int ix = red_i[0];
            for (int w = 1; w < NW; ++w)
                if (red_v[w] > b || (red_v[w] == b && red_i[w] < ix)) {
                    b = red_v[w];
                    ix = red_i[w];
                }
            // no finite maximum (non-finite entries): treat the row as zero
            if (ix < 0 || ix >= n) {
                sh_jstar = 0;
                sh_piv = 0.0;
            } else {
                sh_jstar = ix;
                sh_piv = Vk[ix];
            }
            if (!used[istar]) {
                used[istar] = 1;
                sh_nused += 1;
            }
        }
        __syncthreads();
        const int jstar = sh_jstar;
        const double piv = sh_piv;
        if (piv == 0.0) {
            if (sh_nused == m) break;
            int mi = INT_MAX;
            for (int i = tid; i < m; i += T)
                if (!used[i]) {
                    mi = i;
                    break;
                }
            mi = wave_min(mi);
            if (lane == 0) red_i[wv] = mi;
            __syncthreads();
            if (tid == 0) {
                int b = red_i[0];
                for (int w = 1; w < NW; ++w) b = min(b, red_i[w]);
                // b < m: nused < m guarantees an untried row
                if (b < 0 || b >= m) sh_done = 1;
                sh_istar = (b < 0 || b >= m) ? 0 : b;
            }
            __syncthreads();
            if (sh_done) break;
            continue;
        }
        double nv2 = 0.0;
        for (int j = tid; j < n; j += T) {
            double v = Vk[j] / piv;
            Vk[j] = v;
            nv2 += v * v;
        }
        for (int p = tid; p < k; p += T) s_b[p] = V[(int64_t)p * n + jstar];
        double yj[kMaxD];
        for (int a = 0; a < d; ++a) yj[a] = Y[a * N + jstar];
        __syncthreads();
        // residual of the pivot column, written as column k of U
        double nu2 = 0.0, bu = -1.0;
        int bui = INT_MAX;
        double* Uk = U + (int64_t)k * m;
        for (int i = tid; i < m; i += T) {
            double r2 = 0.0;
            for (int a = 0; a < d; ++a) {
                double t = X[a * N + i] - yj[a];
                r2 += t * t;
            }
            double u = kfun(kp, r2);
            for (int p = 0; p < k; ++p) u -= U[(int64_t)p * m + i] * s_b[p];
            Uk[i] = u;
            nu2 += u * u;
            if (!used[i] && fabs(u) > bu) {
                bu = fabs(u);
                bui = i;
            }
        }
        nu2 = wave_sum(nu2);
        nv2 = wave_sum(nv2);
        wave_argmax(bu, bui);
        if (lane == 0) {
            red_v[wv] = nu2;
            red_w[wv] = nv2;
            red_x[wv] = bu;
            red_j[wv] = bui;
        }
        __syncthreads();
        // cross terms (U_p . u)(V_p . v), p < k; wave w takes p = w, w + NW, ...
        for (int p = wv; p < k; p += NW) {
            double su = 0.0, sv = 0.0;
            const double* Up = U + (int64_t)p * m;
            const double* Vp = V + (int64_t)p * n;
            for (int i = lane; i < m; i += 64) su += Up[i] * Uk[i];
            for (int j = lane; j < n; j += 64) sv += Vp[j] * Vk[j];
            su = wave_sum(su);
            sv = wave_sum(sv);
            if (lane == 0) s_a[p] = su * sv;
        }
        __syncthreads();
        if (tid == 0) {
            double tnu = 0.0, tnv = 0.0, b = red_x[0];
            int ix = red_j[0];
            for (int w = 0; w < NW; ++w) {
                tnu += red_v[w];
                tnv += red_w[w];
            }
            for (int w = 1; w < NW; ++w)
                if (red_x[w] > b || (red_x[w] == b && red_j[w] < ix)) {
                    b = red_x[w];
                    ix = red_j[w];
                }
            double cross = 0.0;
            for (int p = 0; p < k; ++p) cross += s_a[p];
            const double S2new = sh_S2 + 2.0 * cross + tnu * tnv;
            sh_S2new = S2new;
            sh_tsize = sqrt(tnu * tnv);
            sh_ix = ix;
            sh_next = -1;
            sh_small = (k > 0 && sqrt(tnu * tnv) <= tol * sqrt(S2new)) ? 1 : 0;
        }
        __syncthreads();
        if (sh_small) {
            // residual of the k-term approximation on sampled rows and columns
            const int sr = min(m, kAcaSamples), str = m / sr;
            const int sc = min(n, kAcaSamples), stc = n / sc;
            const int c = sh_checks;
            const int offr = (int)(((int64_t)c * 997) % str);
            const int offc = (int)(((int64_t)c * 991) % stc);
            const int64_t nrow = (int64_t)sr * n, total = nrow + (int64_t)sc * m;
            double er = 0.0, ec = 0.0, bs = 0.0;
            int bsi = INT_MAX;
            for (int64_t t = tid; t < total; t += T) {
                int i, j;
                const bool row = t < nrow;
                if (row) {
                    const int q = (int)(t / n);
                    j = (int)(t - (int64_t)q * n);
                    i = q * str + offr;
                } else {
                    const int64_t t2 = t - nrow;
                    const int q = (int)(t2 / m);
                    i = (int)(t2 - (int64_t)q * m);
                    j = q * stc + offc;
                }
                double r2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    double dx = X[a * N + i] - Y[a * N + j];
                    r2 += dx * dx;
                }
                double v = kfun(kp, r2);
                for (int p = 0; p < k; ++p) v -= U[(int64_t)p * m + i] * V[(int64_t)p * n + j];
                if (row)
                    er += v * v;
                else
                    ec += v * v;
                const double av = fabs(v);
                if (!used[i] && av > 0.0 && (av > bs || (av == bs && i < bsi))) {
                    bs = av;
                    bsi = i;
                }
            }
            er = wave_sum(er);
            ec = wave_sum(ec);
            wave_argmax(bs, bsi);
            if (lane == 0) {
                red_v[wv] = er;
                red_w[wv] = ec;
                red_x[wv] = bs;
                red_i[wv] = bsi;
            }
            __syncthreads();
            if (tid == 0) {
                double ter = 0.0, tec = 0.0, b = red_x[0];
                int bi = red_i[0];
                for (int w = 0; w < NW; ++w) {
                    ter += red_v[w];
                    tec += red_w[w];
                }
                for (int w = 1; w < NW; ++w)
                    if (red_x[w] > b || (red_x[w] == b && red_i[w] < bi)) {
                        b = red_x[w];
                        bi = red_i[w];
                    }
                ter *= (double)m / (double)sr;
                tec *= (double)n / (double)sc;
                const double lim = 0.25 * tol * tol * sh_S2;
                sh_checks = c + 1;
                if (ter <= lim && tec <= lim)
                    sh_done = 1;
                else if (b > 0.0 && bi >= 0 && bi < m)
                    sh_next = bi;
            }
            __syncthreads();
        }
        if (tid == 0 && !sh_done) {
            sh_S2 = sh_S2new;
            sh_k = k + 1;
            // the accepted term's pivots: row istar of A, column jstar of B;
            // its size |u| |v|
            pivots[J.pv + 2 * k] = istar;
            pivots[J.pv + 2 * k + 1] = jstar;
            tsize[J.pv / 2 + k] = sh_tsize;
            const int ix = sh_next >= 0 ? sh_next : sh_ix;
            // ix is out of range only if every untried |u_i| is non-finite
            if (sh_nused == m || ix < 0 || ix >= m)
                sh_done = 1;
            else
                sh_istar = ix;
        }
        __syncthreads();
        if (sh_done) break;
    }
    __syncthreads();
    const int r = sh_k;
    if (kLds) {
        // move the finished factors out of LDS: same layout as the workspace
        double* gU = ws;
        double* gV = ws + (int64_t)J.cap * m;
        for (int64_t e = tid; e < (int64_t)r * m; e += T) gU[e] = U[e];
        for (int64_t e = tid; e < (int64_t)r * n; e += T) gV[e] = V[e];
    }
    if (tid == 0) {
        ranks[blockIdx.x] = r;
        overflow[blockIdx.x] = ovf;
        s2out[blockIdx.x] = sh_S2;
    }
}

// ---------------------------------------------------------------------------
// The same iteration for the few largest blocks, each spread over `wpb`
// workgroups of one cooperative launch (all workgroups resident at once).
// Workgroup wl of a block owns rows [wl m / wpb, (wl + 1) m / wpb) of U and the
// matching slice of V's columns.  Every step is a pass over the owned slices
// followed by a grid-wide barrier; each workgroup then reduces the per-slice
// partial results of its block in slice order and takes the same decision
// (pivot, stop, next row) as every other workgroup of the block, so no
// decision is broadcast.  Values one workgroup reads from another's slice
// (the pivot row's U entries, the pivot column's V entries, the sampled rows
// and columns of a stop check, the partials, the tried-row flags) go through
// device-scope atomic loads and stores.  Blocks of one launch advance in
// lockstep; a finished block idles through the barriers until every block of
// the launch is done, so every workgroup runs the same number of barriers.
// ---------------------------------------------------------------------------
namespace coop {

// per (block, workgroup) record of partial results, in doubles
constexpr int R_ROWABS = 0, R_ROWIDX = 1, R_ROWVAL = 2, R_NU2 = 3, R_NV2 = 4, R_UABS = 5,
              R_UIDX = 6, R_ER = 7, R_EC = 8, R_BABS = 9, R_BIDX = 10, R_CROSS = 16;

__device__ __forceinline__ double ldd(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void std_(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ldi(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sti(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void gsync() {
    __threadfence();
    cooperative_groups::this_grid().sync();
    __threadfence();
}

// workgroup sum of one value per thread (result in every thread)
__device__ __forceinline__ double wg_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    return t;
}

// workgroup argmax of (|value|, index) pairs, larger value then lower index
// (result in every thread); idle threads pass (-1, INT_MAX)
__device__ __forceinline__ void wg_argmax(double& v, int& i, double& sv, double* redv, int* redi,
                                          double* reds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // carry the signed value along with the winning index
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(i, o, 64);
        const double os = __shfl_xor(sv, o, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
            sv = os;
        }
    }
    __syncthreads();
    if (lane == 0) {
        redv[wv] = v;
        redi[wv] = i;
        reds[wv] = sv;
    }
    __syncthreads();
    v = redv[0];
    i = redi[0];
    sv = reds[0];
    for (int w = 1; w < NW; ++w)
        if (redv[w] > v || (redv[w] == v && redi[w] < i)) {
            v = redv[w];
            i = redi[w];
            sv = reds[w];
        }
}

}  // namespace coop

__global__ __launch_bounds__(T) void k_aca_coop(const double* __restrict__ pts, int64_t N, int d,
                                                KParams kp, double tol,
                                                const AcaJob* __restrict__ jobs, int njobs,
                                                int wpb, double* wsbase, int* usedbase,
                                                const int64_t* __restrict__ usedoff, double* recs,
                                                int recstride, int* doneflags,
                                                int32_t* __restrict__ ranks,
                                                int32_t* __restrict__ overflow,
                                                int32_t* __restrict__ pivots,
                                                double* __restrict__ tsize,
                                                double* __restrict__ s2out) {
    using namespace coop;
    extern __shared__ double dyn[];
    __shared__ double redv[NW], reds[NW];
    __shared__ int redi[NW];
    const int b = blockIdx.x / wpb, wl = blockIdx.x - b * wpb;
    const int tid = threadIdx.x;
    const AcaJob J = jobs[b];
    const int m = J.m, n = J.n, cap = J.cap;
    const int kcap = min(J.kmax, cap);
    const int r0 = (int)((int64_t)wl * m / wpb), r1 = (int)((int64_t)(wl + 1) * m / wpb);
    const int c0 = (int)((int64_t)wl * n / wpb), c1 = (int)((int64_t)(wl + 1) * n / wpb);
    double* U = wsbase + J.ws;
    double* V = U + (int64_t)cap * m;
    int* used = usedbase + usedoff[b];
    double* mine = recs + ((int64_t)b * wpb + wl) * recstride;
    const double* brec = recs + (int64_t)b * wpb * recstride;
    double* s_a = dyn;          // U entries of the pivot row (or of a sampled row)
    double* s_b = dyn + cap;    // V entries of the pivot column (or of a sampled column)
    const double* __restrict__ X = pts + J.a0;
    const double* __restrict__ Y = pts + J.b0;

    for (int i = r0 + tid; i < r1; i += T) sti(used + i, 0);
    if (wl == 0 && tid == 0) sti(doneflags + b, 0);
    int k = 0, istar = 0, nused = 0, checks = 0;
    bool done = false, ovf = false;
    double S2 = 0.0;
    gsync();
    for (;;) {
        // ---- row residual of the pivot row over the owned columns
        if (!done && k >= kcap) {
            ovf = k < J.kmax;
            done = true;
        }
        if (!done) {
            if (wl == 0 && tid == 0) sti(used + istar, 1);
            nused += 1;
            for (int p = tid; p < k; p += T) s_a[p] = ldd(U + (int64_t)p * m + istar);
            double xi[kMaxD];
            for (int a = 0; a < d; ++a) xi[a] = X[a * N + istar];
            __syncthreads();
            double* Vk = V + (int64_t)k * n;
            double bv = -1.0, bs = 0.0;
            int bi = INT_MAX;
            for (int j = c0 + tid; j < c1; j += T) {
                double r2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    const double t = xi[a] - Y[a * N + j];
                    r2 += t * t;
                }
                double v = kfun(kp, r2);
                for (int p = 0; p < k; ++p) v -= s_a[p] * V[(int64_t)p * n + j];
                Vk[j] = v;
                const double av = fabs(v);
                if (av > bv) {
                    bv = av;
                    bi = j;
                    bs = v;
                }
            }
            wg_argmax(bv, bi, bs, redv, redi, reds);
            if (tid == 0) {
                std_(mine + R_ROWABS, bv);
                std_(mine + R_ROWIDX, (double)bi);
                std_(mine + R_ROWVAL, bs);
            }
        }
        gsync();
        // ---- pivot; residual of the pivot column over the owned rows
        bool zero = false;
        int jstar = INT_MAX;
        done = __builtin_amdgcn_readfirstlane(done ? 1 : 0) != 0;
        if (!done) {
            double bv = -1.0, piv = 0.0;
            for (int w = 0; w < wpb; ++w) {
                const double v = ldd(brec + (int64_t)w * recstride + R_ROWABS);
                const int ix = (int)ldd(brec + (int64_t)w * recstride + R_ROWIDX);
                if (v > bv || (v == bv && ix < jstar)) {
                    bv = v;
                    jstar = ix;
                    piv = ldd(brec + (int64_t)w * recstride + R_ROWVAL);
                }
            }
            // no finite maximum (non-finite entries): the row counts as zero
            if (!(bv >= 0.0) || jstar < 0 || jstar >= n) piv = 0.0;
            jstar = __builtin_amdgcn_readfirstlane(jstar);
            if (__builtin_amdgcn_readfirstlane(piv == 0.0 ? 1 : 0)) {
                zero = true;
                if (nused == m) {
                    done = true;
                } else {
                    int mi = INT_MAX;
                    for (int i = tid; i < m; i += T)
                        if (!ldi(used + i)) {
                            mi = i;
                            break;
                        }
                    double ds = 0.0;
                    // lowest untried row: an argmax of equal values picks the lowest index
                    double key = mi < m ? 1.0 : -1.0;
                    wg_argmax(key, mi, ds, redv, redi, reds);
                    if (key < 0.0 || mi >= m)
                        done = true;
                    else
                        istar = mi;
                }
            } else {
                double* Vk = V + (int64_t)k * n;
                double nv2 = 0.0;
                for (int j = c0 + tid; j < c1; j += T) {
                    const double v = Vk[j] / piv;
                    Vk[j] = v;
                    nv2 += v * v;
                }
                for (int p = tid; p < k; p += T) s_b[p] = ldd(V + (int64_t)p * n + jstar);
                double yj[kMaxD];
                for (int a = 0; a < d; ++a) yj[a] = Y[a * N + jstar];
                __syncthreads();
                double* Uk = U + (int64_t)k * m;
                double nu2 = 0.0, bu = -1.0, bs = 0.0;
                int bui = INT_MAX;
                for (int i = r0 + tid; i < r1; i += T) {
                    double r2 = 0.0;
                    for (int a = 0; a < d; ++a) {
                        const double t = X[a * N + i] - yj[a];
                        r2 += t * t;
                    }
                    double u = kfun(kp, r2);
                    for (int p = 0; p < k; ++p) u -= U[(int64_t)p * m + i] * s_b[p];
                    Uk[i] = u;
                    nu2 += u * u;
                    if (!ldi(used + i) && fabs(u) > bu) {
                        bu = fabs(u);
                        bui = i;
                    }
                }
                nu2 = wg_sum(nu2, redv);
                nv2 = wg_sum(nv2, redv);
                wg_argmax(bu, bui, bs, redv, redi, reds);
                if (tid == 0) {
                    std_(mine + R_NU2, nu2);
                    std_(mine + R_NV2, nv2);
                    std_(mine + R_UABS, bu);
                    std_(mine + R_UIDX, (double)bui);
                }
                // cross products (U_p . u)(V_p . v) over the owned slices, p < k
                const int lane = tid & 63, wv = tid >> 6;
                for (int p = wv; p < k; p += NW) {
                    double su = 0.0, sv = 0.0;
                    const double* Up = U + (int64_t)p * m;
                    const double* Vp = V + (int64_t)p * n;
                    for (int i = r0 + lane; i < r1; i += 64) su += Up[i] * Uk[i];
                    for (int j = c0 + lane; j < c1; j += 64) sv += Vp[j] * Vk[j];
                    su = wave_sum(su);
                    sv = wave_sum(sv);
                    if (lane == 0) {
                        std_(mine + R_CROSS + p, su);
                        std_(mine + R_CROSS + cap + p, sv);
                    }
                }
            }
        }
        gsync();
        // ---- the candidate term's size; sampled residuals when it is small
        bool small = false;
        double S2new = 0.0, tsz = 0.0;
        int ix = -1;
        const int sr = min(m, kAcaSamples), str = m / sr;
        const int sc = min(n, kAcaSamples), stc = n / sc;
        done = __builtin_amdgcn_readfirstlane(done ? 1 : 0) != 0;
        zero = __builtin_amdgcn_readfirstlane(zero ? 1 : 0) != 0;
        istar = __builtin_amdgcn_readfirstlane(istar);
        if (!done && !zero) {
            double nu2 = 0.0, nv2 = 0.0, bu = -1.0;
            int bui = INT_MAX;
            for (int w = 0; w < wpb; ++w) {
                const double* rw = brec + (int64_t)w * recstride;
                nu2 += ldd(rw + R_NU2);
                nv2 += ldd(rw + R_NV2);
                const double v = ldd(rw + R_UABS);
                const int i = (int)ldd(rw + R_UIDX);
                if (v > bu || (v == bu && i < bui)) {
                    bu = v;
                    bui = i;
                }
            }
            double cr = 0.0;
            for (int p = tid; p < k; p += T) {
                double su = 0.0, sv = 0.0;
                for (int w = 0; w < wpb; ++w) {
                    su += ldd(brec + (int64_t)w * recstride + R_CROSS + p);
                    sv += ldd(brec + (int64_t)w * recstride + R_CROSS + cap + p);
                }
                cr += su * sv;
            }
            const double cross = wg_sum(cr, redv);
            S2new = S2 + 2.0 * cross + nu2 * nv2;
            tsz = sqrt(nu2 * nv2);
            ix = (bu >= 0.0 && bui >= 0 && bui < m) ? bui : -1;
            small = __builtin_amdgcn_readfirstlane(
                        (k > 0 && sqrt(nu2 * nv2) <= tol * sqrt(S2new)) ? 1 : 0) != 0;
            if (small) {
                const int offr = (int)(((int64_t)checks * 997) % str);
                const int offc = (int)(((int64_t)checks * 991) % stc);
                double er = 0.0, ec = 0.0, bb = 0.0, bsv = 0.0;
                int bbi = INT_MAX;
                for (int q = 0; q < sr; ++q) {
                    const int i = q * str + offr;
                    __syncthreads();
                    for (int p = tid; p < k; p += T) s_a[p] = ldd(U + (int64_t)p * m + i);
                    __syncthreads();
                    const bool untried = !ldi(used + i);
                    for (int j = c0 + tid; j < c1; j += T) {
                        double r2 = 0.0;
                        for (int a = 0; a < d; ++a) {
                            const double t = X[a * N + i] - Y[a * N + j];
                            r2 += t * t;
                        }
                        double v = kfun(kp, r2);
                        for (int p = 0; p < k; ++p) v -= s_a[p] * V[(int64_t)p * n + j];
                        er += v * v;
                        const double av = fabs(v);
                        if (untried && av > 0.0 && (av > bb || (av == bb && i < bbi))) {
                            bb = av;
                            bbi = i;
                        }
                    }
                }
                for (int q = 0; q < sc; ++q) {
                    const int j = q * stc + offc;
                    __syncthreads();
                    for (int p = tid; p < k; p += T) s_b[p] = ldd(V + (int64_t)p * n + j);
                    __syncthreads();
                    for (int i = r0 + tid; i < r1; i += T) {
                        double r2 = 0.0;
                        for (int a = 0; a < d; ++a) {
                            const double t = X[a * N + i] - Y[a * N + j];
                            r2 += t * t;
                        }
                        double v = kfun(kp, r2);
                        for (int p = 0; p < k; ++p) v -= U[(int64_t)p * m + i] * s_b[p];
                        ec += v * v;
                        const double av = fabs(v);
                        if (!ldi(used + i) && av > 0.0 && (av > bb || (av == bb && i < bbi))) {
                            bb = av;
                            bbi = i;
                        }
                    }
                }
                er = wg_sum(er, redv);
                ec = wg_sum(ec, redv);
                wg_argmax(bb, bbi, bsv, redv, redi, reds);
                if (tid == 0) {
                    std_(mine + R_ER, er);
                    std_(mine + R_EC, ec);
                    std_(mine + R_BABS, bb);
                    std_(mine + R_BIDX, (double)bbi);
                }
            }
        }
        gsync();
        // ---- decision (the same in every workgroup of the block)
        if (!done && !zero) {
            int next = -1;
            if (small) {
                double er = 0.0, ec = 0.0, bb = 0.0;
                int bbi = INT_MAX;
                for (int w = 0; w < wpb; ++w) {
                    const double* rw = brec + (int64_t)w * recstride;
                    er += ldd(rw + R_ER);
                    ec += ldd(rw + R_EC);
                    const double v = ldd(rw + R_BABS);
                    const int i = (int)ldd(rw + R_BIDX);
                    if (v > bb || (v == bb && i < bbi)) {
                        bb = v;
                        bbi = i;
                    }
                }
                er *= (double)m / (double)sr;
                ec *= (double)n / (double)sc;
                const double lim = 0.25 * tol * tol * S2;
                ++checks;
                if (er <= lim && ec <= lim)
                    done = true;
                else if (bb > 0.0 && bbi >= 0 && bbi < m)
                    next = bbi;
            }
            if (!done) {
                S2 = S2new;
                if (wl == 0 && tid == 0) {
                    pivots[J.pv + 2 * k] = istar;
                    pivots[J.pv + 2 * k + 1] = jstar;
                    tsize[J.pv / 2 + k] = tsz;
                }
                k += 1;
                const int nx = next >= 0 ? next : ix;
                if (nused == m || nx < 0 || nx >= m)
                    done = true;
                else
                    istar = nx;
            }
        }
        if (wl == 0 && tid == 0) sti(doneflags + b, done ? 1 : 0);
        gsync();
        bool all = true;
        for (int bb = 0; bb < njobs; ++bb) all = all && ldi(doneflags + bb) != 0;
        // the state every lane computed alike, as scalars: the branches around
        // the barriers are then uniform to the compiler too
        all = __builtin_amdgcn_readfirstlane(all ? 1 : 0) != 0;
        done = __builtin_amdgcn_readfirstlane(done ? 1 : 0) != 0;
        k = __builtin_amdgcn_readfirstlane(k);
        istar = __builtin_amdgcn_readfirstlane(istar);
        nused = __builtin_amdgcn_readfirstlane(nused);
        checks = __builtin_amdgcn_readfirstlane(checks);
        if (all) break;
    }
    if (wl == 0 && tid == 0) {
        ranks[b] = k;
        overflow[b] = ovf ? 1 : 0;
        s2out[b] = S2;
    }
}

// Precision-aware truncation of factors stored in a lower precision: the
// trailing terms whose sizes |u_k| |v_k| add up to at most tau |S|_F (a few
// units of the storage's rounding of the block) are dropped; their sum is a
// bound on the Frobenius norm of what is dropped.  At least one term stays.
__global__ void k_trunc(const AcaJob* __restrict__ jobs, int64_t njobs,
                        const double* __restrict__ tsize, const double* __restrict__ s2,
                        const int32_t* __restrict__ overflow, double tau,
                        int32_t* __restrict__ ranks) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= njobs || overflow[t]) return;
    const double* ts = tsize + jobs[t].pv / 2;
    const double lim = tau * sqrt(fmax(s2[t], 0.0));
    int r = ranks[t];
    double tail = 0.0;
    while (r > 1 && tail + ts[r - 1] <= lim) {
        tail += ts[r - 1];
        --r;
    }
    ranks[t] = r;
}

template <typename S>
__device__ __forceinline__ S to_storage(double v);
template <>
__device__ __forceinline__ double to_storage<double>(double v) {
    return v;
}
template <>
__device__ __forceinline__ float to_storage<float>(double v) {
    return (float)v;
}
template <>
__device__ __forceinline__ bf16 to_storage<bf16>(double v) {
    return (bf16)bf16_bits(v);
}

// copy each job's first r columns of U and rows of V into the arena (terms
// fstride<S> elements apart, zero padded) and record the addresses in the
// block table
template <typename S>
__global__ void k_pack(const AcaJob* __restrict__ jobs, const double* __restrict__ wsbase,
                       const int32_t* __restrict__ ranks, const int64_t* __restrict__ uoff,
                       const int64_t* __restrict__ voff, S* __restrict__ arena_u,
                       S* __restrict__ arena_v, BlockDesc* __restrict__ blocks) {
    const AcaJob J = jobs[blockIdx.x];
    const int r = ranks[blockIdx.x];
    const double* gU = wsbase + J.ws;
    const double* gV = gU + (int64_t)J.cap * J.m;
    S* dU = arena_u + uoff[blockIdx.x];
    S* dV = arena_v + voff[blockIdx.x];
    const int64_t lu = fstride<S>(J.m), lv = fstride<S>(J.n);
    for (int64_t e = threadIdx.x; e < (int64_t)r * lu; e += blockDim.x) {
        const int64_t k = e / lu, i = e - k * lu;
        dU[e] = to_storage<S>(i < J.m ? gU[k * J.m + i] : 0.0);
    }
    for (int64_t e = threadIdx.x; e < (int64_t)r * lv; e += blockDim.x) {
        const int64_t k = e / lv, j = e - k * lv;
        dV[e] = to_storage<S>(j < J.n ? gV[k * J.n + j] : 0.0);
    }
    if (threadIdx.x == 0) {
        BlockDesc& b = blocks[J.block];
        b.rank = r;
        b.U = reinterpret_cast<uint64_t>(dU);
        b.V = reinterpret_cast<uint64_t>(dV);
    }
}

// every factor starts on a 16-byte boundary: sizes rounded up to `align` elements
__global__ void k_sizes(const AcaJob* __restrict__ jobs, const int32_t* __restrict__ ranks,
                        int64_t njobs, int align, int pad8, int64_t* __restrict__ su,
                        int64_t* __restrict__ sv) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= njobs) return;
    const int64_t lu = pad8 ? fstride<bf16>(jobs[t].m) : jobs[t].m;
    const int64_t lv = pad8 ? fstride<bf16>(jobs[t].n) : jobs[t].n;
    su[t] = ((int64_t)ranks[t] * lu + align - 1) / align * align;
    sv[t] = ((int64_t)ranks[t] * lv + align - 1) / align * align;
}

// skeleton form (eq. keq1 with the LU of eq. keq2): the r x r matrix
// K(sigma, tau) = U(sigma, :) V(:, tau) stored as one LU array: on and below
// the diagonal L[i][k] = U(sigma_i, k) (lower, the pivots on the diagonal),
// above it V(i, tau_k) (unit upper); then the pivots sigma (rows of A) and
// tau (columns of B) as int32
template <typename S>
__global__ void k_pack_skel(const AcaJob* __restrict__ jobs, const double* __restrict__ wsbase,
                            const int32_t* __restrict__ ranks, const int32_t* __restrict__ pivots,
                            const int64_t* __restrict__ moff, const int64_t* __restrict__ poff,
                            S* __restrict__ arena_m, int32_t* __restrict__ arena_p,
                            BlockDesc* __restrict__ blocks) {
    const AcaJob J = jobs[blockIdx.x];
    const int r = ranks[blockIdx.x];
    const double* gU = wsbase + J.ws;
    const double* gV = gU + (int64_t)J.cap * J.m;
    const int32_t* pv = pivots + J.pv;
    S* M = arena_m + moff[blockIdx.x];
    int32_t* P = arena_p + poff[blockIdx.x];
    for (int64_t e = threadIdx.x; e < (int64_t)r * r; e += blockDim.x) {
        const int i = (int)(e / r), k = (int)(e - (int64_t)i * r);
        const double v = k <= i ? gU[(int64_t)k * J.m + pv[2 * i]]
                                : gV[(int64_t)i * J.n + pv[2 * k + 1]];
        M[e] = to_storage<S>(v);
    }
    for (int k = threadIdx.x; k < r; k += blockDim.x) {
        P[k] = pv[2 * k];
        P[r + k] = pv[2 * k + 1];
    }
    if (threadIdx.x == 0) {
        BlockDesc& b = blocks[J.block];
        b.rank = r;
        b.U = reinterpret_cast<uint64_t>(M);
        b.V = reinterpret_cast<uint64_t>(P);
    }
}

size_t job_lds_bytes(const AcaJob& j) {
    return sizeof(double) * (2 * (size_t)j.cap + (size_t)j.cap * (j.m + j.n)) + (size_t)j.m + 8;
}

size_t job_ws_doubles(const AcaJob& j) {
    return (size_t)j.cap * (j.m + j.n) + ((size_t)j.m + 7) / 8;
}

size_t storage_size(int storage) {
    return storage == HODLR_FP32 ? 4 : (storage == HODLR_BF16 ? 2 : 8);
}

// elements between rank terms of a factor of length len in this storage
int64_t term_stride(int64_t len, size_t es) { return es == 2 ? fstride<bf16>(len) : len; }

// factor sizes rounded to 16 bytes, so every U and V starts 16-byte aligned
int64_t padded(int64_t elems, size_t es) {
    const int64_t a = 16 / (int64_t)es;
    return (elems + a - 1) / a * a;
}

// host-side element access in a storage buffer of element size es
void put_elem(char* buf, int64_t idx, size_t es, double v) {
    if (es == 8) {
        ((double*)buf)[idx] = v;
    } else if (es == 4) {
        ((float*)buf)[idx] = (float)v;
    } else {
        ((uint16_t*)buf)[idx] = bf16_bits(v);
    }
}

double get_elem(const char* buf, int64_t idx, size_t es) {
    if (es == 8) return ((const double*)buf)[idx];
    if (es == 4) return (double)((const float*)buf)[idx];
    return (double)bf16_to_float(((const uint16_t*)buf)[idx]);
}

struct ChunkResult {
    std::vector<int32_t> ranks, overflow;
};

enum class AcaMode { Global, Lds, Coop };

// Truncation level of FP32-stored factors: eight units of FP32 rounding
// (2^-21), or the ACA tolerance when that is larger.
double trunc_tau(hodlr_t h) { return std::max(h->tol, std::ldexp(1.0, -21)); }

}  // namespace
bool verbose();
namespace {

// workgroups that can be resident at once for the cooperative kernel
int coop_capacity(hodlr_t h, size_t lds_bytes) {
    int per_cu = 0, cus = 0;
    HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_aca_coop, T, lds_bytes));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    return std::max(per_cu, 0) * std::max(cus, 0);
}

// compress one chunk of jobs, pack into a new arena
void run_chunk(hodlr_t h, std::vector<AcaJob>& jobs, AcaMode mode, size_t lds_bytes,
               std::vector<int32_t>& ranks_out, std::vector<int32_t>& ovf_out, hipStream_t s) {
    const bool lds = mode == AcaMode::Lds;
    const int64_t nj = (int64_t)jobs.size();
    size_t ws_total = 0, pv_total = 0;
    for (auto& j : jobs) {
        j.ws = (int64_t)ws_total;
        ws_total += job_ws_doubles(j);
        j.pv = (int64_t)pv_total;
        pv_total += 2 * (size_t)j.cap;
    }
    int32_t* dpiv = (int32_t*)dalloc(h, sizeof(int32_t) * std::max<size_t>(pv_total, 1));
    double* dts = (double*)dalloc(h, sizeof(double) * std::max<size_t>(pv_total / 2, 1));
    double* ds2 = (double*)dalloc(h, sizeof(double) * std::max<int64_t>(nj, 1));
    AcaJob* djobs = (AcaJob*)dalloc(h, sizeof(AcaJob) * nj);
    double* ws = (double*)dalloc(h, sizeof(double) * std::max<size_t>(ws_total, 1));
    int32_t* dr = (int32_t*)dalloc(h, sizeof(int32_t) * nj);
    int32_t* dov = (int32_t*)dalloc(h, sizeof(int32_t) * nj);
    HIP_CHECK(hipMemcpyAsync(djobs, jobs.data(), sizeof(AcaJob) * nj, hipMemcpyHostToDevice, s));
    const double tol = h->tol;
    if (mode == AcaMode::Coop) {
        // one cooperative launch: every job gets wpb workgroups, all resident
        int capmax = 1;
        std::vector<int64_t> uoff(nj);
        int64_t ut = 0;
        for (int64_t t = 0; t < nj; ++t) {
            capmax = std::max(capmax, jobs[t].cap);
            uoff[t] = ut;
            ut += jobs[t].m;
        }
        const size_t clds = sizeof(double) * 2 * (size_t)capmax;
        const int G = coop_capacity(h, clds);
        if (G < nj)
            fail(HODLR_EDEVICE, "cooperative ACA: fewer resident workgroups than blocks");
        int wpb = (int)std::min<int64_t>(G / nj, 128);
        for (auto& j : jobs) wpb = std::min(wpb, std::max(1, std::max(j.m, j.n) / 256));
        wpb = std::max(wpb, 1);
        const int recstride = coop::R_CROSS + 2 * capmax;
        int* dused = (int*)dalloc(h, sizeof(int) * std::max<int64_t>(ut, 1));
        int64_t* duoff = (int64_t*)dalloc(h, sizeof(int64_t) * nj);
        double* drec = (double*)dalloc(h, sizeof(double) * (size_t)nj * wpb * recstride);
        int* ddone = (int*)dalloc(h, sizeof(int) * nj);
        HIP_CHECK(hipMemcpyAsync(duoff, uoff.data(), sizeof(int64_t) * nj, hipMemcpyHostToDevice, s));
        const double* a_pts = h->pts;
        int64_t a_N = h->N;
        int a_d = h->d;
        KParams a_kp = h->kp;
        double a_tol = tol;
        int a_nj = (int)nj;
        void* args[] = {(void*)&a_pts, (void*)&a_N,   (void*)&a_d,    (void*)&a_kp,
                        (void*)&a_tol, (void*)&djobs, (void*)&a_nj,   (void*)&wpb,
                        (void*)&ws,    (void*)&dused, (void*)&duoff,  (void*)&drec,
                        (void*)&recstride, (void*)&ddone, (void*)&dr, (void*)&dov,
                        (void*)&dpiv, (void*)&dts, (void*)&ds2};
        if (verbose())
            std::fprintf(stderr, "[hodlr] ACA (cooperative) %lld blocks x %d workgroups\n",
                         (long long)nj, wpb);
        {
            // one cooperative launch in flight per process: two partly resident
            // ones could wait on each other's workgroups
            static std::mutex coop_mu;
            std::lock_guard<std::mutex> lk(coop_mu);
            HIP_CHECK(hipLaunchCooperativeKernel((const void*)k_aca_coop,
                                                 dim3((unsigned)(nj * wpb)), dim3(T), args, clds,
                                                 s));
            HIP_CHECK(hipStreamSynchronize(s));
        }
        dfree(h, dused);
        dfree(h, duoff);
        dfree(h, drec);
        dfree(h, ddone);
    } else if (lds) {
        HIP_CHECK(hipFuncSetAttribute((const void*)k_aca<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
        k_aca<true><<<(unsigned)nj, T, lds_bytes, s>>>(h->pts, h->N, h->d, h->kp, tol, djobs, ws,
                                                       dr, dov, dpiv, dts, ds2);
    } else {
        size_t small = 0;
        for (auto& j : jobs) small = std::max(small, sizeof(double) * 2 * (size_t)j.cap);
        HIP_CHECK(hipFuncSetAttribute((const void*)k_aca<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)small));
        k_aca<false><<<(unsigned)nj, T, small, s>>>(h->pts, h->N, h->d, h->kp, tol, djobs, ws,
                                                    dr, dov, dpiv, dts, ds2);
    }
    HIP_CHECK(hipGetLastError());
    // FP32 factors: drop the trailing terms below the storage's resolution
    if (h->opts.storage == HODLR_FP32 && !h->opts.skeleton) {
        k_trunc<<<nblk(nj, 256), 256, 0, s>>>(djobs, nj, dts, ds2, dov, trunc_tau(h), dr);
        HIP_CHECK(hipGetLastError());
    }
    ranks_out.resize(nj);
    ovf_out.resize(nj);
    HIP_CHECK(hipMemcpyAsync(ranks_out.data(), dr, sizeof(int32_t) * nj, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(ovf_out.data(), dov, sizeof(int32_t) * nj, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    // pack the jobs that converged; overflowing ones are retried by the caller
    std::vector<AcaJob> ok;
    std::vector<int32_t> okr;
    for (int64_t t = 0; t < nj; ++t)
        if (!ovf_out[t]) {
            ok.push_back(jobs[t]);
            okr.push_back(ranks_out[t]);
        }
    const int64_t nk = (int64_t)ok.size();
    if (nk > 0 && h->opts.skeleton) {
        HIP_CHECK(hipMemcpyAsync(djobs, ok.data(), sizeof(AcaJob) * nk, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(dr, okr.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
        const size_t es = storage_size(h->opts.storage);
        std::vector<int64_t> mo(nk), po(nk);
        int64_t tm = 0, tp = 0;
        for (int64_t t = 0; t < nk; ++t) {
            mo[t] = tm;
            po[t] = tp;
            tm += padded((int64_t)okr[t] * okr[t], es);
            tp += padded(2 * (int64_t)okr[t], 4);
        }
        int64_t* dmo = (int64_t*)dalloc(h, sizeof(int64_t) * nk);
        int64_t* dpo = (int64_t*)dalloc(h, sizeof(int64_t) * nk);
        HIP_CHECK(hipMemcpyAsync(dmo, mo.data(), sizeof(int64_t) * nk, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(dpo, po.data(), sizeof(int64_t) * nk, hipMemcpyHostToDevice, s));
        char* arena = (char*)dalloc(h, es * (size_t)tm + 4 * (size_t)tp + 16);
        h->arenas.push_back(arena);
        int32_t* ap = reinterpret_cast<int32_t*>(arena + es * (size_t)tm);
        if (h->opts.storage == HODLR_FP32)
            k_pack_skel<float><<<(unsigned)nk, 256, 0, s>>>(djobs, ws, dr, dpiv, dmo, dpo,
                                                            (float*)arena, ap, h->blocks);
        else
            k_pack_skel<double><<<(unsigned)nk, 256, 0, s>>>(djobs, ws, dr, dpiv, dmo, dpo,
                                                             (double*)arena, ap, h->blocks);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(s));
        dfree(h, dmo);
        dfree(h, dpo);
    } else if (nk > 0) {
        HIP_CHECK(hipMemcpyAsync(djobs, ok.data(), sizeof(AcaJob) * nk, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(dr, okr.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
        int64_t* su = (int64_t*)dalloc(h, sizeof(int64_t) * nk);
        int64_t* sv = (int64_t*)dalloc(h, sizeof(int64_t) * nk);
        int64_t* ou = (int64_t*)dalloc(h, sizeof(int64_t) * nk);
        int64_t* ov = (int64_t*)dalloc(h, sizeof(int64_t) * nk);
        const size_t es = storage_size(h->opts.storage);
        k_sizes<<<nblk(nk, 256), 256, 0, s>>>(djobs, dr, nk, (int)(16 / es), es == 2 ? 1 : 0,
                                               su, sv);
        HIP_CHECK(hipGetLastError());
        exclusive_scan_i64(su, ou, nk, s);
        exclusive_scan_i64(sv, ov, nk, s);
        int64_t tu = 0, tv = 0;
        for (int64_t t = 0; t < nk; ++t) {
            tu += padded((int64_t)okr[t] * term_stride(ok[t].m, es), es);
            tv += padded((int64_t)okr[t] * term_stride(ok[t].n, es), es);
        }
        // 16 bytes of slack: kernels may read whole 16-byte words at the end
        char* arena = (char*)dalloc(h, es * (size_t)(tu + tv) + 16);
        h->arenas.push_back(arena);
        if (h->opts.storage == HODLR_FP32)
            k_pack<float><<<(unsigned)nk, 256, 0, s>>>(djobs, ws, dr, ou, ov, (float*)arena,
                                                       (float*)arena + tu, h->blocks);
        else if (h->opts.storage == HODLR_BF16)
            k_pack<bf16><<<(unsigned)nk, 256, 0, s>>>(djobs, ws, dr, ou, ov, (bf16*)arena,
                                                      (bf16*)arena + tu, h->blocks);
        else
            k_pack<double><<<(unsigned)nk, 256, 0, s>>>(djobs, ws, dr, ou, ov, (double*)arena,
                                                        (double*)arena + tu, h->blocks);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(s));
        dfree(h, su);
        dfree(h, sv);
        dfree(h, ou);
        dfree(h, ov);
    }
    dfree(h, djobs);
    dfree(h, ws);
    dfree(h, dr);
    dfree(h, dov);
    dfree(h, dpiv);
    dfree(h, dts);
    dfree(h, ds2);
}

}  // namespace

// progress lines on stderr when HODLR_VERBOSE is set (long builds)
bool verbose() {
    static const bool v = std::getenv("HODLR_VERBOSE") != nullptr;
    return v;
}

void compress_all(hodlr_t h, hipStream_t s) {
    int dev_lds = 0;
    HIP_CHECK(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    const size_t static_lds = 1024;
    const size_t lds_limit = (size_t)std::min(dev_lds, 64 * 1024) - static_lds;
    size_t freeb = 0, totalb = 0;
    HIP_CHECK(hipMemGetInfo(&freeb, &totalb));
    const size_t ws_budget = std::max<size_t>(std::min<size_t>(freeb / 4, (size_t)16 << 30), 64 << 20);
    const int maxr = h->opts.max_rank > 0 ? h->opts.max_rank : INT_MAX;

    // blocks with at least this many rows plus columns are spread over many
    // workgroups (HODLR_ACA_COOP_MIN overrides it, for tests)
    int64_t coop_min = 16384;
    if (const char* e = std::getenv("HODLR_ACA_COOP_MIN"))
        if (std::atoll(e) > 0) coop_min = std::atoll(e);
    std::vector<AcaJob> lds_jobs, glob_jobs, coop_jobs;
    for (int64_t b = 0; b < h->nblocks; ++b) {
        const BlockDesc& bd = h->hblocks[b];
        AcaJob j{};
        j.a0 = bd.a0;
        j.m = bd.m;
        j.b0 = bd.b0;
        j.n = bd.n;
        j.kmax = std::min(std::min(bd.m, bd.n), maxr);
        j.block = b;
        j.cap = j.kmax;
        if ((int64_t)bd.m + bd.n >= coop_min && j.kmax > 0) {
            j.cap = std::min(j.kmax, kAcaMaxRank);
            coop_jobs.push_back(j);
        } else if (j.kmax <= kAcaMaxRank && job_lds_bytes(j) <= lds_limit) {
            lds_jobs.push_back(j);
        } else {
            j.cap = std::min(j.kmax, 256);
            glob_jobs.push_back(j);
        }
    }
    std::vector<int32_t> rk, ov;
    // the largest blocks first, cooperatively, in chunks that leave each block
    // at least 16 workgroups and fit the workspace budget
    if (!coop_jobs.empty()) {
        const int G = coop_capacity(h, sizeof(double) * 2 * kAcaMaxRank);
        const size_t per_launch = (size_t)std::max(1, G / 16);
        for (size_t i = 0; i < coop_jobs.size();) {
            std::vector<AcaJob> chunk;
            size_t bytes = 0;
            while (i < coop_jobs.size() && chunk.size() < per_launch &&
                   (chunk.empty() || bytes + 8 * job_ws_doubles(coop_jobs[i]) <= ws_budget)) {
                bytes += 8 * job_ws_doubles(coop_jobs[i]);
                chunk.push_back(coop_jobs[i++]);
            }
            run_chunk(h, chunk, AcaMode::Coop, 0, rk, ov, s);
            for (size_t t = 0; t < chunk.size(); ++t)
                if (ov[t])
                    fail(HODLR_EUNSUPPORTED,
                         "an ACA rank exceeds the device compressor's limit of 1024; "
                         "set max_rank");
        }
    }
    // LDS-resident blocks, in chunks bounded by the workspace budget
    for (size_t i = 0; i < lds_jobs.size();) {
        std::vector<AcaJob> chunk;
        size_t bytes = 0, lmax = 0;
        while (i < lds_jobs.size() &&
               (chunk.empty() || bytes + 8 * job_ws_doubles(lds_jobs[i]) <= ws_budget)) {
            bytes += 8 * job_ws_doubles(lds_jobs[i]);
            lmax = std::max(lmax, job_lds_bytes(lds_jobs[i]));
            chunk.push_back(lds_jobs[i++]);
        }
        run_chunk(h, chunk, AcaMode::Lds, lmax, rk, ov, s);
        if (verbose())
            std::fprintf(stderr, "[hodlr] ACA (LDS) %zu / %zu blocks\n", i, lds_jobs.size());
    }
    // workspace blocks: a first pass with a modest rank cap, retries with more room
    while (!glob_jobs.empty()) {
        std::vector<AcaJob> retry;
        for (size_t i = 0; i < glob_jobs.size();) {
            std::vector<AcaJob> chunk;
            size_t bytes = 0;
            while (i < glob_jobs.size() &&
                   (chunk.empty() || bytes + 8 * job_ws_doubles(glob_jobs[i]) <= ws_budget)) {
                bytes += 8 * job_ws_doubles(glob_jobs[i]);
                chunk.push_back(glob_jobs[i++]);
            }
            run_chunk(h, chunk, AcaMode::Global, 0, rk, ov, s);
            if (verbose())
                std::fprintf(stderr, "[hodlr] ACA (workspace, rank cap %d) %zu / %zu blocks\n",
                             chunk.empty() ? 0 : chunk[0].cap, i, glob_jobs.size());
            for (size_t t = 0; t < chunk.size(); ++t)
                if (ov[t]) {
                    AcaJob j = chunk[t];
                    if (j.cap >= std::min(j.kmax, kAcaMaxRank))
                        fail(HODLR_EUNSUPPORTED,
                             "an ACA rank exceeds the device compressor's limit of 1024; "
                             "set max_rank");
                    j.cap = std::min(std::min(j.kmax, kAcaMaxRank), j.cap * 4);
                    retry.push_back(j);
                }
        }
        glob_jobs.swap(retry);
    }
    for (int l = 1; l <= h->kappa; ++l) h->lev[l].has_factors = true;
    finalize_factors(h, s);
}

// ranks -> projection offsets; host copy of the block table
__global__ void k_rank_of(const BlockDesc* __restrict__ b, int64_t n, int64_t* __restrict__ r) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) r[t] = b[t].rank;
}
__global__ void k_set_toff(BlockDesc* __restrict__ b, int64_t n, const int64_t* __restrict__ off) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) b[t].toff = off[t];
}

void finalize_factors(hodlr_t h, hipStream_t s) {
    const int64_t nb = h->nblocks;
    if (nb > 0) {
        int64_t* r = (int64_t*)dalloc(h, sizeof(int64_t) * nb);
        int64_t* o = (int64_t*)dalloc(h, sizeof(int64_t) * nb);
        k_rank_of<<<nblk(nb, 256), 256, 0, s>>>(h->blocks, nb, r);
        HIP_CHECK(hipGetLastError());
        exclusive_scan_i64(r, o, nb, s);
        k_set_toff<<<nblk(nb, 256), 256, 0, s>>>(h->blocks, nb, o);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(h->hblocks.data(), h->blocks, sizeof(BlockDesc) * nb,
                                 hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        dfree(h, r);
        dfree(h, o);
    }
    int64_t tt = 0;
    for (int64_t b = 0; b < nb; ++b) tt += std::max(h->hblocks[b].rank, 0);
    h->t_total = tt;
    plan_apply(h);
}

// ---------------------------------------------------------------------------
// factor import / export in the interaction list's CSR order
// ---------------------------------------------------------------------------
namespace {
struct HostCsr {
    std::vector<int64_t> ptr, eref;
    std::vector<int32_t> col;
};
HostCsr host_csr(hodlr_t h, int level, hipStream_t s) {
    const LevelData& Lv = h->lev[level];
    HostCsr c;
    c.ptr.resize(Lv.nb + 1);
    c.col.resize(std::max<int64_t>(Lv.nnz, 1));
    c.eref.resize(std::max<int64_t>(Lv.nnz, 1));
    HIP_CHECK(hipMemcpyAsync(c.ptr.data(), Lv.il_ptr, sizeof(int64_t) * (Lv.nb + 1),
                             hipMemcpyDeviceToHost, s));
    if (Lv.nnz) {
        HIP_CHECK(hipMemcpyAsync(c.col.data(), Lv.il_col, sizeof(int32_t) * Lv.nnz,
                                 hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(c.eref.data(), Lv.eref, sizeof(int64_t) * Lv.nnz,
                                 hipMemcpyDeviceToHost, s));
    }
    HIP_CHECK(hipStreamSynchronize(s));
    return c;
}
}  // namespace

void import_level(hodlr_t h, int level, const int32_t* ranks, const double* U, const double* V,
                  hipStream_t s) {
    LevelData& Lv = h->lev[level];
    HostCsr c = host_csr(h, level, s);
    const std::vector<int32_t>& st = Lv.hstart;
    const size_t es = storage_size(h->opts.storage);
    // validate and size the arena (forward entries only)
    int64_t tu = 0, tv = 0;
    for (int64_t A = 0; A < Lv.nb; ++A)
        for (int64_t e = c.ptr[A]; e < c.ptr[A + 1]; ++e) {
            const int64_t B = c.col[e];
            const int64_t m = st[A + 1] - st[A], n = st[B + 1] - st[B];
            if (ranks[e] < 0 || ranks[e] > std::min(m, n))
                fail(HODLR_EINVAL, "imported rank out of range");
            if ((c.eref[e] & 1) == 0) {
                tu += padded(ranks[e] * term_stride(m, es), es);
                tv += padded(ranks[e] * term_stride(n, es), es);
            }
        }
    if ((tu + tv) > 0 && (!U || !V)) fail(HODLR_EINVAL, "factor arrays missing");
    std::vector<char> hbuf(es * (size_t)(tu + tv) + 16, 0);
    char* arena = (char*)dalloc(h, hbuf.size());
    h->arenas.push_back(arena);
    int64_t ou = 0, ov = 0, pu = 0, pv = 0;
    for (int64_t A = 0; A < Lv.nb; ++A)
        for (int64_t e = c.ptr[A]; e < c.ptr[A + 1]; ++e) {
            const int64_t B = c.col[e];
            const int64_t m = st[A + 1] - st[A], n = st[B + 1] - st[B];
            const int64_t r = ranks[e];
            if ((c.eref[e] & 1) == 0) {
                BlockDesc& bd = h->hblocks[c.eref[e] >> 1];
                bd.rank = (int32_t)r;
                bd.U = reinterpret_cast<uint64_t>(arena + es * pu);
                bd.V = reinterpret_cast<uint64_t>(arena + es * (tu + pv));
                const int64_t lu = term_stride(m, es), lv = term_stride(n, es);
                for (int64_t k = 0; k < r; ++k)
                    for (int64_t i = 0; i < m; ++i)
                        put_elem(hbuf.data(), pu + k * lu + i, es, U[ou + k * m + i]);
                for (int64_t k = 0; k < r; ++k)
                    for (int64_t j = 0; j < n; ++j)
                        put_elem(hbuf.data(), tu + pv + k * lv + j, es, V[ov + k * n + j]);
                pu += padded(r * lu, es);
                pv += padded(r * lv, es);
            }
            ou += r * m;
            ov += r * n;
        }
    HIP_CHECK(hipMemcpyAsync(arena, hbuf.data(), hbuf.size(), hipMemcpyHostToDevice, s));
    if (Lv.nblk)
        HIP_CHECK(hipMemcpyAsync(h->blocks + Lv.blk0, h->hblocks.data() + Lv.blk0,
                                 sizeof(BlockDesc) * Lv.nblk, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
    Lv.has_factors = true;
    bool all = true;
    for (int l = 1; l <= h->kappa; ++l) all = all && h->lev[l].has_factors;
    if (all) finalize_factors(h, s);
}

void export_level(hodlr_t h, int level, int32_t* ranks, int64_t* u_elems, int64_t* v_elems,
                  double* U, double* V, hipStream_t s) {
    LevelData& Lv = h->lev[level];
    if (!Lv.has_factors) fail(HODLR_EINVAL, "level has no factors");
    HostCsr c = host_csr(h, level, s);
    const std::vector<int32_t>& st = Lv.hstart;
    const size_t es = storage_size(h->opts.storage);
    int64_t ou = 0, ov = 0;
    std::vector<char> tmp;
    for (int64_t A = 0; A < Lv.nb; ++A)
        for (int64_t e = c.ptr[A]; e < c.ptr[A + 1]; ++e) {
            const int64_t B = c.col[e];
            const int64_t m = st[A + 1] - st[A], n = st[B + 1] - st[B];
            const BlockDesc& bd = h->hblocks[c.eref[e] >> 1];
            const bool tr = (c.eref[e] & 1) != 0;
            const int64_t r = bd.rank;
            if (ranks) ranks[e] = (int32_t)r;
            // a transposed entry's U is the stored V and its V the stored U
            const uint64_t srcU = tr ? bd.V : bd.U;
            const uint64_t srcV = tr ? bd.U : bd.V;
            // the factor with |A| rows has term stride term_stride(|A|) in either
            // orientation (a transposed entry's U is the stored V of (B,A))
            const int64_t su = term_stride(m, es), sv = term_stride(n, es);
            if (U && r * m) {
                tmp.resize(es * r * su);
                HIP_CHECK(hipMemcpy(tmp.data(), reinterpret_cast<void*>(srcU), es * r * su,
                                    hipMemcpyDeviceToHost));
                for (int64_t k = 0; k < r; ++k)
                    for (int64_t i = 0; i < m; ++i) U[ou + k * m + i] = get_elem(tmp.data(), k * su + i, es);
            }
            if (V && r * n) {
                tmp.resize(es * r * sv);
                HIP_CHECK(hipMemcpy(tmp.data(), reinterpret_cast<void*>(srcV), es * r * sv,
                                    hipMemcpyDeviceToHost));
                for (int64_t k = 0; k < r; ++k)
                    for (int64_t j = 0; j < n; ++j) V[ov + k * n + j] = get_elem(tmp.data(), k * sv + j, es);
            }
            ou += r * m;
            ov += r * n;
        }
    if (u_elems) *u_elems = ou;
    if (v_elems) *v_elems = ov;
}

}  // namespace hodlr
