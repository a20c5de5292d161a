// Solves (alpha I + beta K~) U = F with GMRES and iterative refinement.
//
// The outer loop refines in FP64: r = F - (alpha u + beta K~_hi u) with the
// FP64 representation, u += d.  Each correction d comes from one restarted
// cycle of GMRES on the low-precision representation (K~_lo, e.g. BF16 or
// FP32 factors) for the residual equation, stopped when its own residual
// estimate falls below inner_tol relative to |r|.  The Krylov basis, the
// Gram-Schmidt orthogonalisation (classical, applied twice) and the norms are
// FP64; the small Hessenberg systems and Givens rotations are solved on the
// host in FP64.  The columns of F are solved together: every Arnoldi step
// applies the operator to all of them in one product, and a column whose
// estimate has converged stops updating its own rotations.
//
// Reductions are deterministic: partial sums per block of rows are added on
// the host in block order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {

constexpr int TB = 256;        // threads per block of the vector kernels
constexpr int CHUNK = 4096;    // rows per partial-sum block

// partial dot products of w (column c) with the first nv basis vectors of
// column c: out[(blk * nrhs + c) * nvmax + i]; basis layout V[(i * nrhs + c) * N + n]
__global__ void k_multidot(const double* __restrict__ V, int nv, int nvmax,
                           const double* __restrict__ W, int64_t N, int nrhs,
                           double* __restrict__ out) {
    __shared__ double red[TB / 64];
    const int c = blockIdx.y;
    const int64_t n0 = (int64_t)blockIdx.x * CHUNK;
    const int64_t n1 = min(N, n0 + CHUNK);
    double w[CHUNK / TB];
#pragma unroll
    for (int t = 0; t < CHUNK / TB; ++t) {
        const int64_t n = n0 + threadIdx.x + (int64_t)t * TB;
        w[t] = n < n1 ? W[(int64_t)c * N + n] : 0.0;
    }
    for (int i = 0; i < nv; ++i) {
        const double* __restrict__ v = V + ((int64_t)i * nrhs + c) * N;
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < CHUNK / TB; ++t) {
            const int64_t n = n0 + threadIdx.x + (int64_t)t * TB;
            if (n < n1) a += v[n] * w[t];
        }
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < TB / 64; ++k) s += red[k];
            out[((int64_t)blockIdx.x * nrhs + c) * nvmax + i] = s;
        }
        __syncthreads();
    }
}

// W[c] += sgn * sum_i coef[c * nvmax + i] V[i][c]
__global__ void k_multiaxpy(const double* __restrict__ V, int nv, int nvmax,
                            const double* __restrict__ coef, double sgn, double* __restrict__ W,
                            int64_t N, int nrhs) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    const int64_t n = t - (int64_t)c * N;
    double a = 0.0;
    for (int i = 0; i < nv; ++i) a += coef[c * nvmax + i] * V[((int64_t)i * nrhs + c) * N + n];
    W[t] += sgn * a;
}

// Y[c] = s[c] X[c]
__global__ void k_scale(const double* __restrict__ X, const double* __restrict__ sc,
                        double* __restrict__ Y, int64_t N, int nrhs) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    Y[t] = sc[t / N] * X[t];
}

// R = F - alpha U - beta KU  (F, U with leading dimensions; R, KU packed N x nrhs)
__global__ void k_residual(const double* __restrict__ F, int64_t ldf, const double* __restrict__ U,
                           int64_t ldu, const double* __restrict__ KU, double alpha, double beta,
                           double* __restrict__ R, int64_t N, int nrhs) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    const int64_t n = t - (int64_t)c * N;
    R[t] = F[c * ldf + n] - alpha * U[c * ldu + n] - beta * KU[t];
}

// R = F (R packed N x nrhs); reads nothing but F
__global__ void k_copy_cols(const double* __restrict__ F, int64_t ldf, double* __restrict__ R,
                            int64_t N, int nrhs) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    const int64_t n = t - (int64_t)c * N;
    R[t] = F[c * ldf + n];
}

// U[c] += D[c]; or U[c] = 0 when D is null
__global__ void k_update(double* __restrict__ U, int64_t ldu, const double* __restrict__ D,
                         int64_t N, int nrhs) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    const int64_t n = t - (int64_t)c * N;
    U[c * ldu + n] = D ? U[c * ldu + n] + D[t] : 0.0;
}

__global__ void k_zero(double* __restrict__ Y, int64_t n) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) Y[t] = 0.0;
}

// Y = alpha X + beta Y (packed)
__global__ void k_axpby(const double* __restrict__ X, double alpha, double* __restrict__ Y,
                        double beta, int64_t n) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) Y[t] = alpha * X[t] + beta * Y[t];
}

struct Dev {
    std::vector<void*> p;
    ~Dev() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    T* get(size_t n) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            fail(HODLR_ENOMEM, "solver workspace allocation failed");
        }
        p.push_back(q);
        return (T*)q;
    }
};

}  // namespace

void solve(hodlr_t hi, hodlr_t lo, double alpha, double beta, const double* F, int64_t ldf,
           int nrhs, double* U, int64_t ldu, const hodlr_solve_opts& o, hodlr_solve_info* info,
           hipStream_t s) {
    const int64_t N = hi->N;
    const int m = o.restart;
    const int nvmax = m + 1;
    const int64_t NR = N * nrhs;
    const int nchunk = (int)((N + CHUNK - 1) / CHUNK);
    const unsigned g = nblk(NR, TB);
    Dev dev;
    double* V = dev.get<double>((size_t)nvmax * NR);   // Krylov basis
    double* W = dev.get<double>(NR);
    double* R = dev.get<double>(NR);
    double* KU = dev.get<double>(NR);
    double* part = dev.get<double>((size_t)nchunk * nrhs * nvmax);
    double* coef = dev.get<double>((size_t)nrhs * nvmax);
    double* sc = dev.get<double>(nrhs);
    std::vector<double> hpart((size_t)nchunk * nrhs * nvmax), hcoef((size_t)nrhs * nvmax);

    // column-wise dot products of W with the first nv basis vectors (or
    // with W itself: V = W, nv = 1), summed over blocks in order
    auto dots = [&](const double* Vb, int nv, const double* Wb, std::vector<double>& res) {
        k_multidot<<<dim3(nchunk, nrhs), TB, 0, s>>>(Vb, nv, nvmax, Wb, N, nrhs, part);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(hpart.data(), part, sizeof(double) * hpart.size(),
                                 hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        res.assign((size_t)nrhs * nvmax, 0.0);
        for (int b = 0; b < nchunk; ++b)
            for (int c = 0; c < nrhs; ++c)
                for (int i = 0; i < nv; ++i)
                    res[(size_t)c * nvmax + i] += hpart[((size_t)b * nrhs + c) * nvmax + i];
    };
    auto norms = [&](const double* X, std::vector<double>& nr) {
        std::vector<double> d;
        // V layout with nv = 1 and nrhs columns is a packed N x nrhs matrix
        dots(X, 1, X, d);
        nr.resize(nrhs);
        for (int c = 0; c < nrhs; ++c) nr[c] = std::sqrt(d[(size_t)c * nvmax]);
    };
    auto apply = [&](hodlr_t h, const double* X, double* Y, int prec) {
        // Y = alpha X + beta K~ X
        matvec(h, X, N, nrhs, HODLR_FP64, Y, N, prec, nullptr, 0, s);
        k_axpby<<<g, TB, 0, s>>>(X, alpha, Y, beta, NR);
        HIP_CHECK(hipGetLastError());
    };
    const int hi_prec = HODLR_FP64;
    const int lo_prec = lo->opts.storage == HODLR_BF16 ? HODLR_FP32 : o.lo_compute;

    std::vector<double> fn;
    {
        // ||F|| per column: copy F into R (packed) first; U and R may hold
        // anything (the caller's output buffer, fresh memory)
        k_copy_cols<<<g, TB, 0, s>>>(F, ldf, R, N, nrhs);
        HIP_CHECK(hipGetLastError());
        norms(R, fn);
        for (int c = 0; c < nrhs; ++c)
            if (!std::isfinite(fn[c])) fail(HODLR_ENONFINITE, "F holds NaN or Inf");
    }
    if (!o.use_initial_guess) k_update<<<g, TB, 0, s>>>(U, ldu, nullptr, N, nrhs);
    HIP_CHECK(hipGetLastError());

    info->outer_iters = 0;
    info->inner_iters = 0;
    info->converged = 0;
    std::vector<double> rn, H((size_t)nrhs * nvmax * m), cs((size_t)nrhs * m), sn((size_t)nrhs * m),
        gv((size_t)nrhs * nvmax), h1, h2, hn;
    for (int outer = 0;; ++outer) {
        // r = F - A_hi u
        if (outer == 0 && !o.use_initial_guess) {
            k_copy_cols<<<g, TB, 0, s>>>(F, ldf, R, N, nrhs);
        } else {
            matvec(hi, U, ldu, nrhs, HODLR_FP64, KU, N, hi_prec, nullptr, 0, s);
            k_residual<<<g, TB, 0, s>>>(F, ldf, U, ldu, KU, alpha, beta, R, N, nrhs);
        }
        HIP_CHECK(hipGetLastError());
        norms(R, rn);
        double rel = 0.0;
        for (int c = 0; c < nrhs; ++c) {
            if (!std::isfinite(rn[c]))
                fail(HODLR_ENONFINITE, o.use_initial_guess && outer == 0
                                           ? "the initial guess U holds NaN or Inf"
                                           : "the residual became NaN or Inf");
            // a zero right-hand side: the absolute residual
            rel = std::max(rel, fn[c] > 0 ? rn[c] / fn[c] : rn[c]);
        }
        if (outer < 64) info->history[outer] = rel;
        info->rel_residual = rel;
        info->outer_iters = outer;
        if (rel <= o.tol) {
            info->converged = 1;
            break;
        }
        if (outer >= o.max_outer) break;
        // one GMRES(m) cycle on A_lo d = r
        std::vector<double> s0(nrhs);
        for (int c = 0; c < nrhs; ++c) s0[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
        HIP_CHECK(hipMemcpyAsync(sc, s0.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
        k_scale<<<g, TB, 0, s>>>(R, sc, V, N, nrhs);
        HIP_CHECK(hipGetLastError());
        std::fill(gv.begin(), gv.end(), 0.0);
        std::vector<int> steps(nrhs, 0);
        std::vector<char> active(nrhs, 1);
        for (int c = 0; c < nrhs; ++c) {
            gv[(size_t)c * nvmax] = rn[c];
            if (!(rn[c] > 0)) active[c] = 0;
        }
        int j = 0;
        for (; j < m; ++j) {
            bool any = false;
            for (int c = 0; c < nrhs; ++c) any = any || active[c];
            if (!any) break;
            apply(lo, V + (size_t)j * NR, W, lo_prec);
            // classical Gram-Schmidt, twice
            std::vector<double> hsum((size_t)nrhs * nvmax, 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                dots(V, j + 1, W, h1);
                HIP_CHECK(hipMemcpyAsync(coef, h1.data(), sizeof(double) * h1.size(),
                                         hipMemcpyHostToDevice, s));
                k_multiaxpy<<<g, TB, 0, s>>>(V, j + 1, nvmax, coef, -1.0, W, N, nrhs);
                HIP_CHECK(hipGetLastError());
                for (size_t t = 0; t < h1.size(); ++t) hsum[t] += h1[t];
            }
            norms(W, hn);
            for (int c = 0; c < nrhs; ++c) s0[c] = hn[c] > 1e-300 ? 1.0 / hn[c] : 0.0;
            HIP_CHECK(hipMemcpyAsync(sc, s0.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
            k_scale<<<g, TB, 0, s>>>(W, sc, V + (size_t)(j + 1) * NR, N, nrhs);
            HIP_CHECK(hipGetLastError());
            ++info->inner_iters;
            // Givens rotations per active column
            for (int c = 0; c < nrhs; ++c) {
                if (!active[c]) continue;
                double* hc = &H[((size_t)c * m + j) * nvmax];
                for (int i = 0; i <= j; ++i) hc[i] = hsum[(size_t)c * nvmax + i];
                hc[j + 1] = hn[c];
                for (int i = 0; i < j; ++i) {
                    const double a = cs[(size_t)c * m + i] * hc[i] + sn[(size_t)c * m + i] * hc[i + 1];
                    const double b = -sn[(size_t)c * m + i] * hc[i] + cs[(size_t)c * m + i] * hc[i + 1];
                    hc[i] = a;
                    hc[i + 1] = b;
                }
                const double den = std::hypot(hc[j], hc[j + 1]);
                const double cj = den > 0 ? hc[j] / den : 1.0, sj = den > 0 ? hc[j + 1] / den : 0.0;
                cs[(size_t)c * m + j] = cj;
                sn[(size_t)c * m + j] = sj;
                hc[j] = den;
                hc[j + 1] = 0.0;
                double* gc = &gv[(size_t)c * nvmax];
                gc[j + 1] = -sj * gc[j];
                gc[j] = cj * gc[j];
                steps[c] = j + 1;
                if (std::fabs(gc[j + 1]) <= o.inner_tol * rn[c] || hn[c] <= 1e-300) active[c] = 0;
            }
        }
        // y = R^-1 g per column; d = V y
        std::fill(hcoef.begin(), hcoef.end(), 0.0);
        for (int c = 0; c < nrhs; ++c) {
            const int k = steps[c];
            for (int i = k - 1; i >= 0; --i) {
                double v = gv[(size_t)c * nvmax + i];
                for (int l = i + 1; l < k; ++l)
                    v -= H[((size_t)c * m + l) * nvmax + i] * hcoef[(size_t)c * nvmax + l];
                const double dgl = H[((size_t)c * m + i) * nvmax + i];
                hcoef[(size_t)c * nvmax + i] = dgl != 0.0 ? v / dgl : 0.0;
            }
        }
        HIP_CHECK(hipMemcpyAsync(coef, hcoef.data(), sizeof(double) * hcoef.size(),
                                 hipMemcpyHostToDevice, s));
        k_zero<<<g, TB, 0, s>>>(W, NR);
        k_multiaxpy<<<g, TB, 0, s>>>(V, std::max(j, 1), nvmax, coef, 1.0, W, N, nrhs);
        k_update<<<g, TB, 0, s>>>(U, ldu, W, N, nrhs);
        HIP_CHECK(hipGetLastError());
    }
    HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace hodlr
