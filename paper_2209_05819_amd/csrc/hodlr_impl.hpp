// Internal declarations of the MI355X HODLRdD library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hodlr.h"

namespace hodlr {

struct Error {
    hodlr_status code;
    std::string msg;
};

[[noreturn]] inline void fail(hodlr_status c, const std::string& m) { throw Error{c, m}; }

#define HIP_CHECK(expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::hodlr::fail(HODLR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxD = 8;
constexpr int kMaxLevels = 32;
constexpr int kAcaMaxRank = 1024;   // per-block ACA rank limit of the device compressor

// Kernel function parameters as the device sees them.
struct KParams {
    int kind;
    double h;
    double inv_h;
    double inv_h2;
    double scale;
    double diag;
};

// 1/sqrt(x), x > 0, in FP64: the hardware estimate refined by two Newton
// steps y <- y (3/2 - (x/2) y^2), each of which roughly doubles the number
// of correct bits (three operations a step: y^2, one FMA, one product).
__device__ __forceinline__ double rsqrt_fp64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
#pragma unroll
    for (int i = 0; i < 2; ++i) y *= fma(-hx, y * y, 1.5);
    return y;
}

// r2 = |x - y|^2; returns scale * f(r).  FP64 and FP32 variants.
__device__ __forceinline__ double kfun(const KParams& k, double r2) {
    double f;
    switch (k.kind) {
    case HODLR_K_LOG: f = 0.5 * log(r2); break;
    case HODLR_K_INV_R: f = rsqrt_fp64(r2); break;
    case HODLR_K_INV_R2: f = 1.0 / r2; break;
    case HODLR_K_GAUSS: f = exp(-r2 * k.inv_h2); break;
    case HODLR_K_EXP: f = exp(-sqrt(r2) * k.inv_h); break;
    case HODLR_K_R: f = sqrt(r2); break;
    case HODLR_K_SIN: f = sin(sqrt(r2)); break;
    default: f = 1.0 / sqrt(1.0 + sqrt(r2)); break;
    }
    return k.scale * f;
}

// FP32: 1/r and 1/r^2 by the hardware reciprocal (square root), 1 ulp, without
// a rescaled path for r^2 below the smallest normal FP32 number (where 1/r
// exceeds 1.8e19 and the product has no accuracy left in FP32 anyway).
__device__ __forceinline__ float kfun(const KParams& k, float r2) {
    float f;
    switch (k.kind) {
    case HODLR_K_LOG: f = 0.5f * __logf(r2); break;
    case HODLR_K_INV_R: f = __builtin_amdgcn_rsqf(r2); break;
    case HODLR_K_INV_R2: f = __builtin_amdgcn_rcpf(r2); break;
    case HODLR_K_GAUSS: f = __expf(-r2 * (float)k.inv_h2); break;
    case HODLR_K_EXP: f = __expf(-sqrtf(r2) * (float)k.inv_h); break;
    case HODLR_K_R: f = sqrtf(r2); break;
    case HODLR_K_SIN: f = sinf(sqrtf(r2)); break;
    default: f = rsqrtf(1.0f + sqrtf(r2)); break;
    }
    return (float)k.scale * f;
}

// the same with the kernel function fixed at compile time (KIND < 0: chosen
// at run time)
template <int KIND, typename T>
__device__ __forceinline__ T kfun_k(const KParams& k, T r2) {
    if constexpr (KIND < 0) {
        return kfun(k, r2);
    } else {
        KParams kk = k;
        kk.kind = KIND;   // a constant: the switch folds away
        return kfun(kk, r2);
    }
}

// A device address held as an integer, as a pointer into the global address
// space (global loads rather than generic ones, which also count against the
// LDS wait counter).
template <typename T>
using gptr_t = const T __attribute__((address_space(1)))*;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte word
template <typename T>
__device__ __forceinline__ gptr_t<T> as_global(uint64_t a) {
    return (gptr_t<T>)a;
}

// BF16 factor storage: the upper 16 bits of an IEEE binary32, rounded to
// nearest even.  A distinct type so that loads convert by bit pattern.
enum class bf16 : uint16_t {};

__host__ __device__ inline uint16_t bf16_from_float(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP64 -> BF16 through FP32 (both round to nearest even; the double rounding
// differs from a direct rounding only on exact BF16 ties after the first)
__host__ __device__ inline uint16_t bf16_bits(double v) { return bf16_from_float((float)v); }

__host__ __device__ inline float bf16_to_float(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Elements between consecutive rank terms of a stored factor of length
// `len` (U: |A| per column, V: |B| per row).  BF16 terms are padded with
// zeros to a multiple of 8 elements, so every term starts 16-byte aligned
// and matrix-core operands load as whole 16-byte words.
template <typename S>
__host__ __device__ constexpr int64_t fstride(int64_t len) {
    return len;
}
template <>
__host__ __device__ constexpr int64_t fstride<bf16>(int64_t len) {
    return (len + 7) & ~(int64_t)7;
}

// factor element i of a stored factor, converted to the compute type
template <typename C, typename S>
__device__ __forceinline__ C ldf(gptr_t<S> p, int64_t i) {
    return (C)p[i];
}
template <typename C>
__device__ __forceinline__ C ldf(gptr_t<bf16> p, int64_t i) {
    return (C)bf16_to_float((uint16_t)p[i]);
}

// The same, for factor elements a kernel reads exactly once per product.
// FP64 factors take a nontemporal load (measured a few percent faster for
// this stream); 4- and 2-byte elements measured slower with it and take the
// ordinary load.
template <typename C, typename S>
__device__ __forceinline__ C ldf_once(gptr_t<S> p, int64_t i) {
    if constexpr (sizeof(S) == 8) {
        return (C)__builtin_nontemporal_load(p + i);
    } else {
        return ldf<C>(p, i);
    }
}

// One stored low-rank block: rows = box A (|A| = m, tree offset a0),
// columns = box B (|B| = n, tree offset b0).  U is m x r column by column,
// V is r x n row by row, both in the storage type at byte addresses U, V,
// consecutive terms fstride<S>(m) resp. fstride<S>(n) elements apart.
struct BlockDesc {
    int32_t a0, m, b0, n;
    int32_t rank, level;
    int64_t toff;       // offset of this block's projections in the t/s buffers
    uint64_t U, V;      // device addresses
    int64_t cfwd;       // contribution segment of U (V x_B) to the rows of A
    int64_t cbwd;       // contribution segment of V^T (U^T x_A) to the rows of B (symmetric)
};

// rows [lo, lo+cnt) of leaf box `leaf` (first row leaf0) and its near-field
// source ranges nrng[nb0 .. nb0+nn)
struct NearItem {
    int32_t leaf, lo, cnt, leaf0;
    int64_t nb0;
    int32_t nn, pad;
};

// contribution segments a leaf's rows receive at one level: ne segments of
// len values each, the leaf's first row at contrib[base] of the first one
struct SegRef {
    int64_t base;
    int32_t len, ne;
};

struct LevelData {
    int64_t nb = 0;
    int32_t* start = nullptr;    // device, nb+1
    uint64_t* key = nullptr;     // device, nb
    int32_t* coord = nullptr;    // device, nb*d
    int64_t* il_ptr = nullptr;   // device, nb+1
    int32_t* il_col = nullptr;   // device, nnz
    int64_t nnz = 0;
    int64_t* eref = nullptr;     // device, per IL entry: (stored block << 1) | transposed
    int64_t blk0 = 0, nblk = 0;  // range in the global block table
    std::vector<int32_t> hstart; // host copy of start
    // bit 0: active (its parent was subdivided); bit 1: leaf.  A uniform tree
    // has every box active and its leaves on the last level.
    uint8_t* flags = nullptr;    // device, nb
    std::vector<uint8_t> hflags; // host copy
    // dense near-field pairs of this level (rows: the level's boxes)
    int64_t* near_ptr = nullptr;
    int32_t* near_col = nullptr;
    int64_t near_nnz = 0;
    bool has_factors = false;
};

// Matrix-core product records (BF16 factors).  A projection job computes
// t = F x over the panel [p0, p0 + plen) of the factor's columns for all
// its terms: F = V (t = V x_B) or F = U (s = U^T x_A).
struct MJob {
    uint64_t F;
    int64_t out;        // fin: BF16 projection offset; else FP32 partial offset
    int32_t r, len;     // rank; factor length (term stride fstride<bf16>(len))
    int32_t x0;         // tree row of the factor's column 0
    int32_t p0, plen;
    int32_t fin;        // 1 when the panel is the whole factor
};
struct MRed {           // sum of the np panel partials of one projection
    int64_t out, part;
    int32_t r16, np;
};
struct MEnt {           // an interaction-list entry (A,B) in the expansion:
    uint64_t F;         // the factor with |A| rows (U, or V of the stored (B,A))
    int64_t t;          // its projections (t of (A,B), or s of the stored (B,A))
    int32_t r, pad;
};
struct MTile {          // rows of a target box A at one level applied by one workgroup
    int32_t row0, rows; // tree row of the tile, rows in it
    int32_t len, rowoff;// |A|, offset of the tile in A
    int64_t e0;         // entries [e0, e0 + ne) in interaction-list order
    int32_t ne, pad;
};

// Projections of a block too large for one workgroup: term k of block blk,
// rows segment seg of nseg of both sides; its partial sums go to slot p of
// the partial buffer, [p][side][seg][column].
constexpr int kProjSegMax = 16;
struct ProjSeg {
    int32_t blk, k, seg, nseg;
    int64_t p;
};
// the sum of a term's nseg partials, in segment order, into t (and s) at
// offset dst (the block's term offset plus k)
struct ProjSum {
    int64_t dst, p;
    int32_t nseg, pad;
};

struct WorkItem {   // launch planning record: a block (or box) and a sub-range
    int32_t id;
    int32_t lo;
    int32_t cnt;
    int32_t level;
};

// Skeleton form: the partial sum of one side's skeleton projection of block
// blk over the sources [lo, lo + cnt) of the other box (side 0: K(sigma, B)
// x_B, side 1: K(tau, A) x_A), rank values written at dst
struct SkelProj {
    int32_t blk, side, lo, cnt;
    int64_t dst;
};
// and, per block, where its partials are: nsf segments of rank values from
// pf (side 0), nsb from pb (side 1)
struct SkelSolve {
    int64_t pf, pb;
    int32_t nsf, nsb;
};

}  // namespace hodlr

struct hodlr_handle_s {
    int64_t N = 0;
    int d = 0;
    hodlr_kernel kern{};
    hodlr::KParams kp{};
    int leaf = 0;
    double tol = 0;
    hodlr_opts opts{};
    int device = 0;
    int kappa = 0, lmax = 0;
    double lo[8]{}, side = 1.0;
    double* pts = nullptr;       // device, SoA tree order: pts[a*N + p]
    int32_t* perm = nullptr;     // device, tree position -> user index
    uint64_t* keys = nullptr;    // device, sorted Morton keys
    hodlr::LevelData lev[hodlr::kMaxLevels];
    int64_t* near_ptr = nullptr;
    int32_t* near_col = nullptr;
    int64_t near_nnz = 0;
    int64_t near_pairs = 0;
    // stored blocks (all levels)
    hodlr::BlockDesc* blocks = nullptr;   // device
    std::vector<hodlr::BlockDesc> hblocks;
    int64_t nblocks = 0;
    int64_t t_total = 0;                  // sum of ranks
    std::vector<void*> arenas;            // factor storage allocations
    // launch plans
    hodlr::BlockDesc* class_blocks = nullptr;  // copies of the descriptors, by size class
    std::vector<int64_t> class_off;        // class c: [class_off[c], class_off[c+1])
    int64_t cls_felems[8]{}, cls_velems[8]{};  // factor / vector elements per class
    int64_t split_blocks = 0, split_felems = 0;
    hodlr::ProjSeg* proj_items = nullptr;  // segmented projections of the blocks too large
                                           // for one workgroup
    hodlr::ProjSum* proj_sums = nullptr;   // their per-term sums
    int64_t n_proj_sums = 0;
    int64_t n_proj_items = 0;
    hodlr::WorkItem* exp_items = nullptr;  // 64-row chunks of those blocks (level = side)
    int64_t n_exp_items = 0;
    // skeleton form: segmented skeleton projections, per-block solves,
    // 256-row expansions (level = side)
    hodlr::SkelProj* skel_proj = nullptr;
    int64_t n_skel_proj = 0;
    hodlr::SkelSolve* skel_solve = nullptr;
    hodlr::WorkItem* skel_exp = nullptr;
    int64_t n_skel_exp = 0;
    int64_t skel_part_total = 0;           // partial values of the projections
    int64_t skel_max_rank = 0;
    hodlr::NearItem* near_items = nullptr; // 64-row chunks of the leaves
    int64_t n_near_items = 0;
    int64_t near_max_ranges = 0;           // most near-list boxes of a leaf
    int2* near_rng = nullptr;              // tree-order ranges of the near-list boxes
    hodlr::SegRef* leaf_seg = nullptr;     // [leaf][level-1] contribution segments
    // matrix-core plan (BF16 factors, several right-hand sides), two passes:
    // projection jobs by workgroup width W = 1, 2, 4, 8 waves, the reductions
    // of the blocks projected in several panels, and per level the 128-row
    // tiles of the target boxes with their interaction-list entries
    hodlr::MJob* mjobs = nullptr;
    std::vector<int64_t> mjob_off;          // W class c: [mjob_off[c], mjob_off[c+1])
    hodlr::MRed* mreds = nullptr;
    int64_t n_mreds = 0;
    hodlr::MEnt* ments = nullptr;
    hodlr::MTile* mtiles = nullptr;
    std::vector<int64_t> mtile_off;         // level l: [mtile_off[l-1], mtile_off[l])
    int64_t mt_total = 0;                   // BF16 projection elements per right-hand side
    int64_t mpart_total = 0;                // FP32 panel partials per right-hand side
    int64_t mjob_felems[4]{}, mjob_velems[4]{}, mjob_count[4]{};
    int64_t mexp_felems = 0;
    int64_t contrib_total = 0;             // contribution elements per right-hand side
    int64_t nleaf = 0;
    // plan of the persistent product (one launch walks every stage): the
    // size classes with class 5 limited to blocks of at most 2304 rows and
    // columns, the larger blocks on the segmented route (projections per
    // term and row segment, their sums, 64-row expansions)
    hodlr::BlockDesc* p_class_blocks = nullptr;
    std::vector<int64_t> p_class_off;
    hodlr::ProjSeg* p_proj = nullptr;
    hodlr::ProjSum* p_psum = nullptr;
    hodlr::WorkItem* p_exp = nullptr;
    int64_t p_n_proj = 0, p_n_psum = 0, p_n_exp = 0;
    int* p_ctr = nullptr;       // its launch counters: claim, done, exit, error, diagnostics
    int use_persistent = -1;    // product route: 1 persistent; 0 or -1 (not chosen) per-class
    int tune_cls[8]{};          // tile-shape candidate of each single-RHS block class
    void* p_dslot = nullptr;    // device slot table and claim queue of the last product
    void* p_dsegs = nullptr;
    size_t p_segcap = 0;
    std::vector<int64_t> p_key; // what they were built for (pointers, sizes, types)
    int64_t p_nclaims = 0;
    size_t p_nseg = 0;
    int p_nstages = 0;
    int p_seg_side = 1024;      // persistent plan: blocks wider than this take the segmented route
    std::vector<int32_t> cls_ids;   // stored blocks in class order (host)
    std::vector<int64_t> split_ids; // the blocks wider than 4608 (host)
    // matvec workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // second stream of the product (default priority): the near field, which
    // is bound by arithmetic, runs on it while the low-rank stages stream the
    // factors from HBM on the caller's stream; fork and join by events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t device_bytes = 0;
    double build_ms[4]{};
    std::unordered_map<void*, size_t> allocs;
};

namespace hodlr {

// device memory held by a handle (tracked for the budget)
void* dalloc(hodlr_t h, size_t bytes);
void dfree(hodlr_t h, void* p);

// tree.hip
void build_tree(hodlr_t h, const double* points_host, hipStream_t s);
// lists.hip
void build_lists(hodlr_t h, hipStream_t s);
void build_block_table(hodlr_t h, hipStream_t s);
// aca.hip
void compress_all(hodlr_t h, hipStream_t s);
// apply.hip
void plan_apply(hodlr_t h);

// Largest byte offset, relative to a buffer resource's base, that the
// matrix-core passes form for a BF16 factor of rank r and length len (up to
// nrp <= 32 right-hand sides).  Their buffer loads move a lane with nothing
// to read past the resource's range by adding 2^31 to its offset, so every
// offset must stay below kMcoreRange for that sum to land past the range
// instead of wrapping to a real address.
constexpr int64_t kMcoreRange = (int64_t)1 << 31;
int64_t mcore_extent(int64_t r, int64_t len, int nrp);
// ev: nullptr or nev = 5 or 5 + kApplyClasses events: [0] before the
// product, [1] after permute-in, [2] after all block projections (one-pass
// blocks and split projections), [3] after the split expansions, [4] after
// gather + near field + permute-out; [5 + c] after the launch of size class c
constexpr int kApplyClasses = 6;
void matvec(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y, int64_t ldy,
            int compute_prec, hipEvent_t const* ev, int nev, hipStream_t s);
// grows the handle's product workspace to what nrhs columns need
void reserve_workspace(hodlr_t h, int nrhs, int compute_prec, hipStream_t s);
// whether a product takes the persistent route (one launch) with these types
bool persistent_route(hodlr_t h, int x_prec, int compute_prec);
// products of several handles in one persistent launch (same x_prec for all;
// compute precision = storage precision, FP64 or FP32); ctr: four zeroed ints
// owned by the caller, dslot/dsegs: device tables the caller owns, with room
// for nslots slots and *segcap segments (grown with dalloc on h0 if needed)
// asynchronous batched products (no synchronisation; completion by the
// caller's events) with preallocated tables of up to max_slots handles and
// segcap queue segments
void* batch_tables_create(int max_slots, size_t segcap);
void batch_tables_destroy(void* tables);
void matvec_batch_async(int nslots, hodlr_t const* hs, const void* const* X, const int64_t* ldx,
                        const int* nrhs, int x_prec, void* const* Y, const int64_t* ldy,
                        void* tables, hipStream_t s);
// times the tile-shape candidates of the block classes and the two routes
// on this handle, keeps the fastest of each (see hodlr_autotune)
void autotune(hodlr_t h, int nrhs, int x_prec, int compute_prec, hodlr_tuning* out,
              hipStream_t s);
void matvec_batch(int nslots, hodlr_t const* hs, const void* const* X, const int64_t* ldx,
                  const int* nrhs, int x_prec, void* const* Y, const int64_t* ldy, int* ctr,
                  hipStream_t s);
// the product with its workspace in the library's static scratch array and
// the near field on s (no allocation, no second stream)
constexpr int64_t kScratchBytes = (int64_t)64 << 20;
void matvec_noalloc(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y,
                    int64_t ldy, int compute_prec, hipStream_t s);
// serve.hip
hodlr_status server_create(const hodlr_server_opts& o, hodlr_server_t* out);
void server_destroy(hodlr_server_t S);
int server_add(hodlr_server_t S, hodlr_t h);
size_t server_room(hodlr_server_t S);
int server_batch_cols(hodlr_server_t S);
hodlr_status server_submit(hodlr_server_t S, const hodlr_request& r, int64_t* id, std::string& err);
hodlr_status server_wait(hodlr_server_t S, int64_t id, int block, int* done, double* queue_us,
                         double* run_us, std::string& err);
void server_stats(hodlr_server_t S, hodlr_server_stats* st);
// solve.hip: (alpha I + beta K~) U = F, FP64 refinement over GMRES on lo
void solve(hodlr_t hi, hodlr_t lo, double alpha, double beta, const double* F, int64_t ldf,
           int nrhs, double* U, int64_t ldu, const hodlr_solve_opts& o, hodlr_solve_info* info,
           hipStream_t s);
// factor import / export in aca.hip
void import_level(hodlr_t h, int level, const int32_t* ranks, const double* U, const double* V,
                  hipStream_t s);
void export_level(hodlr_t h, int level, int32_t* ranks, int64_t* u_elems, int64_t* v_elems,
                  double* U, double* V, hipStream_t s);
void finalize_factors(hodlr_t h, hipStream_t s);

// prim.hip: device-wide primitives
void sort_pairs_u64(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout,
                    int64_t n, int end_bit, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
void segmented_sort_i32(const int32_t* in, int32_t* out, int64_t nnz, int64_t nseg,
                        const int64_t* offsets, hipStream_t s);

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace hodlr
