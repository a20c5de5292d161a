/*
 * hodlr_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the HODLRdD method of Khan,
 * Kandappan and Ambikasaran (arXiv 2209.05819), written from the paper to
 * check the GPU library against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the GPU library never links,
 * includes or calls it, and it shares no code with the GPU library.
 *
 * What it computes:
 *   - the direct sum b = K q (the plain definition of the product);
 *   - the method step by step: computational hyper-cube, 2^d tree (paper
 *     sec. 5.2), interaction lists (table "Notations", def. "HODLRdD
 *     admissibility", sec. 5.3), ACA compression of every interaction-list
 *     block (Alg. "HODLRdD Initialization", eq. keq1) and the matrix-vector
 *     product (Alg. "HODLRdD matrix-vector Product").
 *
 * All index sets are in "tree order": the points sorted by (Morton key,
 * original index).  Factor layout of a block (A,B) with |A| = m, |B| = n and
 * rank r: U is m x r stored column by column (U[k*m + i]), V is r x n stored
 * row by row (V[k*n + j]); the block is approximated by U V.
 */
#ifndef HODLR_ORACLE_H
#define HODLR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* kernel kinds; K(i,j) = scale * f(r), r = |x_i - x_j|_2, for i != j and
 * K(i,i) = diag (decided by global point index). */
enum { OK_LOG = 0, OK_INV_R = 1, OK_INV_R2 = 2, OK_GAUSS = 3, OK_EXP = 4,
       OK_R = 5, OK_SIN = 6, OK_INV_SQRT1P = 7 };

typedef struct {
    int kind;
    double h;      /* length scale of OK_GAUSS (exp(-r^2/h^2)) and OK_EXP (exp(-r/h)) */
    double scale;  /* multiplies f(r) */
    double diag;   /* value of K(i,i) */
} ork_kernel;

typedef struct ohodlr_s ohodlr;

/* status codes (same meaning as the GPU library's, defined independently) */
enum { ORK_OK = 0, ORK_EINVAL = 1, ORK_ENOMEM = 2 };

/* f(r) for two points (no diagonal rule). */
double ohodlr_kernel_eval(const ork_kernel* k, const double* x, const double* y, int d);
/* dense block out[i*n + j] = scale * f(|X_i - Y_j|), X m x d, Y n x d row-major. */
void ohodlr_kernel_block(const ork_kernel* k, const double* X, int64_t m,
                         const double* Y, int64_t n, int d, double* out);

/* Tree + lists.  points: N x d row-major (user order, copied).
 * has_domain != 0: the hyper-cube is [lo, lo+side]^d (points outside -> EINVAL);
 * otherwise the bounding cube.  level_rule 0: kappa = smallest level whose
 * fullest box holds at most leaf points; 1: smallest kappa with
 * leaf * 2^(d kappa) >= N; 2: adaptive tree, depth as rule 0, and a box is
 * subdivided only while it holds more than leaf points (leaves on several
 * levels; see ohodlr_box_flags). */
ohodlr* ohodlr_create(const double* points, int64_t N, int d, int has_domain,
                      const double* lo, double side, int leaf, int level_rule,
                      int* status);
/* The same with another admissibility: adjacent boxes sharing a hyper-surface
 * of dimension <= adm_dim are admissible (-1: far field only; 0: HODLRdD,
 * as ohodlr_create; d-1: every pair, HODLR). */
ohodlr* ohodlr_create_adm(const double* points, int64_t N, int d, int has_domain,
                          const double* lo, double side, int leaf, int level_rule, int adm_dim,
                          int* status);
void ohodlr_destroy(ohodlr* h);

int     ohodlr_kappa(const ohodlr* h);
int     ohodlr_lmax(const ohodlr* h);
void    ohodlr_domain(const ohodlr* h, double* lo, double* side);
void    ohodlr_perm(const ohodlr* h, int64_t* perm);        /* perm[pos] = original index */
void    ohodlr_keys(const ohodlr* h, uint64_t* keys);       /* sorted Morton keys */
void    ohodlr_quantized(const ohodlr* h, int64_t* q);      /* N x d, user order */
int64_t ohodlr_nboxes(const ohodlr* h, int level);
/* start: nb+1 offsets into tree order; key: level key; coord: nb x d */
void    ohodlr_boxes(const ohodlr* h, int level, int64_t* start, uint64_t* key, int32_t* coord);
int64_t ohodlr_il_nnz(const ohodlr* h, int level);
void    ohodlr_il(const ohodlr* h, int level, int64_t* ptr, int32_t* col);
/* dense near-field pairs of level kappa (all of them in a uniform tree) */
int64_t ohodlr_near_nnz(const ohodlr* h);
void    ohodlr_near(const ohodlr* h, int64_t* ptr, int32_t* col);
/* dense near-field pairs of one level: rows are the level's boxes, columns
 * the boxes B with (A, B) dense (both active, not admissible, one a leaf) */
int64_t ohodlr_near_level_nnz(const ohodlr* h, int level);
void    ohodlr_near_level(const ohodlr* h, int level, int64_t* ptr, int32_t* col);
/* per box of a level: bit 0 active (its parent was subdivided), bit 1 leaf */
void    ohodlr_box_flags(const ohodlr* h, int level, uint8_t* flags);

/* ACA (partial pivoting) on an explicit m x n matrix M (row-major).
 * U must hold m*min(m,n) and V min(m,n)*n doubles; pivots min(m,n) each.
 * Returns the rank. */
int ohodlr_aca_dense(const double* M, int64_t m, int64_t n, double tol, int max_rank,
                     double* U, double* V, int64_t* piv_row, int64_t* piv_col);

/* Compress every interaction-list block (paper order, both (A,B) and (B,A)).
 * Only target boxes A lying inside tree-order rows [row0, row1) are treated
 * (row0 = 0, row1 = N for all).  Returns status. */
int ohodlr_compress(ohodlr* h, const ork_kernel* k, double tol, int max_rank,
                    int64_t row0, int64_t row1);
/* ranks of the IL entries of a level (CSR order); -1 for untreated entries */
void    ohodlr_ranks(const ohodlr* h, int level, int32_t* ranks);
int64_t ohodlr_factor_elems(const ohodlr* h, int level, int which /*0 U, 1 V*/);
void    ohodlr_factors(const ohodlr* h, int level, double* U, double* V);
/* install factors for every IL entry of a level (same packed layout) */
int     ohodlr_set_factors(ohodlr* h, int level, const int32_t* ranks,
                           const double* U, const double* V);

/* b = K~ q with the stored factors plus the dense near field (Alg. matvec).
 * q, b: N x nrhs column-major, user order.  Only rows of target boxes inside
 * [row0,row1) (tree order) are computed; other rows of b are set to 0. */
int ohodlr_matvec(const ohodlr* h, const ork_kernel* k, const double* q, int nrhs,
                  double* b, int64_t row0, int64_t row1);

/* Direct sum b_i = sum_j K(i,j) q_j (ascending j).  rows == NULL: all rows,
 * else only rows[0..nrows) and b is nrows x nrhs. */
void ohodlr_direct(const double* points, int64_t N, int d, const ork_kernel* k,
                   const double* q, int nrhs, const int64_t* rows, int64_t nrows,
                   double* b);

int ohodlr_num_threads(void);
void ohodlr_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
