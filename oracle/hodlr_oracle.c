/*
 * hodlr_oracle.c -- TEST INFRASTRUCTURE ONLY (see hodlr_oracle.h).
 *
 * Plain FP64 C, one obvious loop per step of the paper's method.  Parallelism
 * is OpenMP over independent target boxes / rows only, so every result is
 * computed by one thread in a fixed order.  Compiled with
 * -O2 -fno-fast-math -ffp-contract=off.
 */
#include "hodlr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Kernel functions F1..F8 of sec. 3 (list of eight kernels), the 4D Laplace   */
/* kernel 1/r^2 of sec. 6.2 and the Gaussian of sec. 6.3.                      */
/* ------------------------------------------------------------------------- */
double ohodlr_kernel_eval(const ork_kernel* k, const double* x, const double* y, int d)
{
    double r2 = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = x[a] - y[a];
        r2 += t * t;
    }
    double r = sqrt(r2);
    double f;
    switch (k->kind) {
    case OK_LOG:        f = log(r); break;
    case OK_INV_R:      f = 1.0 / r; break;
    case OK_INV_R2:     f = 1.0 / (r * r); break;
    case OK_GAUSS:      f = exp(-(r * r) / (k->h * k->h)); break;
    case OK_EXP:        f = exp(-r / k->h); break;
    case OK_R:          f = r; break;
    case OK_SIN:        f = sin(r); break;
    case OK_INV_SQRT1P: f = 1.0 / sqrt(1.0 + r); break;
    default:            f = NAN; break;
    }
    return k->scale * f;
}

void ohodlr_kernel_block(const ork_kernel* k, const double* X, int64_t m,
                         const double* Y, int64_t n, int d, double* out)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            out[i * n + j] = ohodlr_kernel_eval(k, X + i * d, Y + j * d, d);
}

/* entry of the full kernel matrix, diagonal decided by global index */
static double entry(const ork_kernel* k, const double* P, int d, int64_t gi, int64_t gj)
{
    if (gi == gj) return k->diag;
    return ohodlr_kernel_eval(k, P + gi * d, P + gj * d, d);
}

int ohodlr_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of later parallel loops (timing on a given number of cores) */
void ohodlr_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Tree (sec. 5.2) and interaction lists (sec. 5.3, table of notations)        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nb;
    int64_t* start;   /* nb+1 */
    uint64_t* key;    /* nb */
    int32_t* coord;   /* nb*d */
    uint8_t* flag;    /* nb: bit 0 active (its parent was subdivided), bit 1 leaf */
    /* dense near-field pairs of this level (rows: active boxes) */
    int64_t* near_ptr;
    int32_t* near_col;
    /* interaction list (levels >= 1) */
    int64_t* il_ptr;
    int32_t* il_col;
    /* factors per IL entry */
    int32_t* rank;
    double** U;
    double** V;
} olevel;

struct ohodlr_s {
    int64_t N;
    int d, Lmax, kappa, leaf, rule;
    int adm;            /* largest shared hyper-surface dimension that is admissible */
    double lo[8], side;
    double* pts_user;   /* N*d user order */
    double* pts;        /* N*d tree order */
    int64_t* q;         /* N*d quantized coordinates, user order */
    uint64_t* key;      /* N, tree order */
    int64_t* perm;      /* tree position -> user index */
    olevel lev[64];
};

typedef struct { uint64_t key; int64_t idx; } kv;

static int kv_cmp(const void* a, const void* b)
{
    const kv* x = (const kv*)a;
    const kv* y = (const kv*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/* coordinates of the level-l box containing quantized point q: q >> (Lmax-l) */
static void build_level(ohodlr* h, int l)
{
    olevel* L = &h->lev[l];
    const int d = h->d;
    const int shift = d * (h->Lmax - l);
    int64_t nb = 0;
    for (int64_t p = 0; p < h->N; ++p)
        if (p == 0 || (h->key[p] >> shift) != (h->key[p - 1] >> shift)) ++nb;
    L->nb = nb;
    L->start = (int64_t*)malloc(sizeof(int64_t) * (nb + 1));
    L->key = (uint64_t*)malloc(sizeof(uint64_t) * (nb ? nb : 1));
    L->coord = (int32_t*)malloc(sizeof(int32_t) * (nb ? nb : 1) * d);
    int64_t b = 0;
    for (int64_t p = 0; p < h->N; ++p) {
        if (p == 0 || (h->key[p] >> shift) != (h->key[p - 1] >> shift)) {
            L->start[b] = p;
            L->key[b] = h->key[p] >> shift;
            const int64_t* qq = h->q + h->perm[p] * d;
            for (int a = 0; a < d; ++a) L->coord[b * d + a] = (int32_t)(qq[a] >> (h->Lmax - l));
            ++b;
        }
    }
    L->start[nb] = h->N;
}

static int64_t level_max_count(const ohodlr* h, int l)
{
    const int shift = h->d * (h->Lmax - l);
    int64_t best = 0, run = 0;
    for (int64_t p = 0; p < h->N; ++p) {
        if (p == 0 || (h->key[p] >> shift) != (h->key[p - 1] >> shift)) run = 0;
        ++run;
        if (run > best) best = run;
    }
    return best;
}

/* Interaction list membership at one level (table of notations and the
 * admissibility definitions of sec. 5).  Two distinct boxes are admissible
 * when they are far apart (at least one box between them) or adjacent and
 * sharing a hyper-surface of dimension <= t (the number of equal integer
 * coordinates): t = 0 is the HODLRdD condition (vertex sharing), t = -1
 * keeps only the far field (strong admissibility of H-matrices), t = d-1
 * admits every pair (weak admissibility of HODLR).  A pair enters the list
 * of the level where it first becomes admissible: its parents must not be
 * admissible (equal, or adjacent sharing a hyper-surface of dimension > t).
 * With t = 0 the parents' condition is the "clan" read with d' >= 1 (the
 * reading documented with the library). */
static int in_il(const int32_t* A, const int32_t* B, int d, int t)
{
    int same = 1, par_max = 0, par_eq = 0, chd_max = 0, chd_eq = 0;
    for (int a = 0; a < d; ++a) {
        if (A[a] != B[a]) same = 0;
        int32_t P = A[a] >> 1, Q = B[a] >> 1;
        int dp = abs(P - Q);
        if (dp > par_max) par_max = dp;
        if (P == Q) ++par_eq;
        int dc = abs(A[a] - B[a]);
        if (dc > chd_max) chd_max = dc;
        if (dc == 0) ++chd_eq;
    }
    if (same) return 0;
    int parents_open = (par_max == 0) || (par_max == 1 && par_eq > t);
    if (!parents_open) return 0;
    return chd_max >= 2 || (chd_max == 1 && chd_eq <= t);
}

/* near field at the leaves: the box itself and the adjacent boxes that are
 * not admissible (sharing a hyper-surface of dimension > t). */
static int in_near(const int32_t* A, const int32_t* B, int d, int t)
{
    int mx = 0, eq = 0;
    for (int a = 0; a < d; ++a) {
        int dc = abs(A[a] - B[a]);
        if (dc > mx) mx = dc;
        if (dc == 0) ++eq;
    }
    if (mx == 0) return 1;
    return mx == 1 && eq > t;
}

/* Active and leaf boxes.  Uniform trees (rules 0, 1): every box is active
 * and the leaves are the boxes of level kappa.  Adaptive tree (rule 2, the
 * adaptive 2^d tree the paper mentions in sec. 5.2): a box is subdivided only
 * while it holds more than `leaf` points, so a box is active when its parent
 * holds more than `leaf` points (then so do all its ancestors), and an active
 * box is a leaf when it holds at most `leaf` points or lies on level kappa.
 * The boxes below a leaf still partition its points but take no part in the
 * lists. */
static void build_flags(ohodlr* h)
{
    for (int l = 0; l <= h->kappa; ++l) {
        olevel* L = &h->lev[l];
        L->flag = (uint8_t*)calloc((size_t)(L->nb ? L->nb : 1), 1);
        const olevel* P = l > 0 ? &h->lev[l - 1] : NULL;
        int64_t par = 0;
        for (int64_t A = 0; A < L->nb; ++A) {
            const int64_t cnt = L->start[A + 1] - L->start[A];
            int act, lf;
            if (h->rule != 2) {
                act = 1;
                lf = l == h->kappa;
            } else {
                if (P) {
                    while (P->start[par + 1] <= L->start[A]) ++par;
                    act = P->start[par + 1] - P->start[par] > h->leaf;
                } else {
                    act = 1;
                }
                lf = act && (cnt <= h->leaf || l == h->kappa);
            }
            L->flag[A] = (uint8_t)((act ? 1 : 0) | (lf ? 2 : 0));
        }
    }
}

static int active(const olevel* L, int64_t A) { return L->flag[A] & 1; }
static int is_leaf(const olevel* L, int64_t A) { return (L->flag[A] & 2) != 0; }

/* pairs of level l compressed at this level: both boxes active (their
 * parents were subdivided and their parents' pair not admissible) and the
 * pair admissible */
static int il_pair(const ohodlr* h, const olevel* L, int64_t A, int64_t B)
{
    if (!active(L, A) || !active(L, B)) return 0;
    return in_il(L->coord + A * h->d, L->coord + B * h->d, h->d, h->adm);
}

/* dense pairs of level l: both active, not admissible (the box itself or an
 * adjacent box sharing a hyper-surface of dimension > t), and one of them a
 * leaf, so the pair is not subdivided further */
static int near_pair(const ohodlr* h, const olevel* L, int64_t A, int64_t B)
{
    if (!active(L, A) || !active(L, B)) return 0;
    if (!is_leaf(L, A) && !is_leaf(L, B)) return 0;
    return in_near(L->coord + A * h->d, L->coord + B * h->d, h->d, h->adm);
}

static void build_lists(ohodlr* h, int l)
{
    olevel* L = &h->lev[l];
    const int64_t nb = L->nb;
    L->il_ptr = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
    /* count (brute force over every box pair) */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = 0; A < nb; ++A) {
        int64_t c = 0;
        for (int64_t B = 0; B < nb; ++B)
            if (il_pair(h, L, A, B)) ++c;
        L->il_ptr[A + 1] = c;
    }
    for (int64_t A = 0; A < nb; ++A) L->il_ptr[A + 1] += L->il_ptr[A];
    int64_t nnz = L->il_ptr[nb];
    L->il_col = (int32_t*)malloc(sizeof(int32_t) * (nnz ? nnz : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = 0; A < nb; ++A) {
        int64_t c = L->il_ptr[A];
        for (int64_t B = 0; B < nb; ++B)
            if (il_pair(h, L, A, B)) L->il_col[c++] = (int32_t)B;
    }
    L->rank = (int32_t*)malloc(sizeof(int32_t) * (nnz ? nnz : 1));
    L->U = (double**)calloc(nnz ? nnz : 1, sizeof(double*));
    L->V = (double**)calloc(nnz ? nnz : 1, sizeof(double*));
    for (int64_t e = 0; e < nnz; ++e) L->rank[e] = -1;
}

static void build_near(ohodlr* h, int l)
{
    olevel* L = &h->lev[l];
    const int64_t nb = L->nb;
    L->near_ptr = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = 0; A < nb; ++A) {
        int64_t c = 0;
        for (int64_t B = 0; B < nb; ++B)
            if (near_pair(h, L, A, B)) ++c;
        L->near_ptr[A + 1] = c;
    }
    for (int64_t A = 0; A < nb; ++A) L->near_ptr[A + 1] += L->near_ptr[A];
    int64_t nnz = L->near_ptr[nb];
    L->near_col = (int32_t*)malloc(sizeof(int32_t) * (nnz ? nnz : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = 0; A < nb; ++A) {
        int64_t c = L->near_ptr[A];
        for (int64_t B = 0; B < nb; ++B)
            if (near_pair(h, L, A, B)) L->near_col[c++] = (int32_t)B;
    }
}

ohodlr* ohodlr_create(const double* points, int64_t N, int d, int has_domain,
                      const double* lo, double side, int leaf, int level_rule,
                      int* status)
{
    return ohodlr_create_adm(points, N, d, has_domain, lo, side, leaf, level_rule, 0, status);
}

ohodlr* ohodlr_create_adm(const double* points, int64_t N, int d, int has_domain,
                          const double* lo, double side, int leaf, int level_rule, int adm_dim,
                          int* status)
{
    *status = ORK_EINVAL;
    if (N < 1 || d < 1 || d > 8 || leaf < 1) return NULL;
    if (adm_dim < -1 || adm_dim > d - 1) return NULL;
    for (int64_t i = 0; i < N * d; ++i)
        if (!isfinite(points[i])) return NULL;
    ohodlr* h = (ohodlr*)calloc(1, sizeof(ohodlr));
    h->N = N; h->d = d; h->leaf = leaf; h->rule = level_rule; h->adm = adm_dim;
    h->Lmax = 63 / d < 30 ? 63 / d : 30;

    /* computational hyper-cube C (sec. 5.2) */
    if (has_domain) {
        if (!(side > 0.0)) { free(h); return NULL; }
        for (int a = 0; a < d; ++a) h->lo[a] = lo[a];
        h->side = side;
        for (int64_t i = 0; i < N; ++i)
            for (int a = 0; a < d; ++a) {
                double x = points[i * d + a];
                if (x < h->lo[a] || x > h->lo[a] + side) { free(h); return NULL; }
            }
    } else {
        double mn[8], mx[8];
        for (int a = 0; a < d; ++a) { mn[a] = points[a]; mx[a] = points[a]; }
        for (int64_t i = 1; i < N; ++i)
            for (int a = 0; a < d; ++a) {
                double x = points[i * d + a];
                if (x < mn[a]) mn[a] = x;
                if (x > mx[a]) mx[a] = x;
            }
        double s = 0.0;
        for (int a = 0; a < d; ++a) {
            h->lo[a] = mn[a];
            double w = mx[a] - mn[a];
            if (w > s) s = w;
        }
        h->side = s > 0.0 ? s : 1.0;
    }

    h->pts_user = (double*)malloc(sizeof(double) * N * d);
    memcpy(h->pts_user, points, sizeof(double) * N * d);

    /* quantized coordinates at the finest representable level and Morton keys
     * (dimension 0 most significant inside each level's group of d bits) */
    const int L = h->Lmax;
    const double scale = ldexp(1.0, L);
    const int64_t qmax = ((int64_t)1 << L) - 1;
    h->q = (int64_t*)malloc(sizeof(int64_t) * N * d);
    kv* tmp = (kv*)malloc(sizeof(kv) * N);
    for (int64_t i = 0; i < N; ++i) {
        for (int a = 0; a < d; ++a) {
            double t = (points[i * d + a] - h->lo[a]) / h->side;
            double f = floor(t * scale);
            int64_t qi = (int64_t)f;
            if (qi < 0) qi = 0;
            if (qi > qmax) qi = qmax;
            h->q[i * d + a] = qi;
        }
        uint64_t key = 0;
        for (int b = L - 1; b >= 0; --b)
            for (int a = 0; a < d; ++a)
                key = (key << 1) | (uint64_t)((h->q[i * d + a] >> b) & 1);
        tmp[i].key = key;
        tmp[i].idx = i;
    }
    qsort(tmp, (size_t)N, sizeof(kv), kv_cmp);
    h->key = (uint64_t*)malloc(sizeof(uint64_t) * N);
    h->perm = (int64_t*)malloc(sizeof(int64_t) * N);
    h->pts = (double*)malloc(sizeof(double) * N * d);
    for (int64_t p = 0; p < N; ++p) {
        h->key[p] = tmp[p].key;
        h->perm[p] = tmp[p].idx;
        for (int a = 0; a < d; ++a) h->pts[p * d + a] = points[tmp[p].idx * d + a];
    }
    free(tmp);

    /* depth kappa */
    int kappa = 0;
    if (level_rule == 0 || level_rule == 2) {
        while (kappa < L && level_max_count(h, kappa) > leaf) ++kappa;
    } else {
        /* smallest kappa with leaf * 2^(d kappa) >= N, in integers:
         * leaf * 2^bits >= N  <=>  leaf >= ceil(N / 2^bits) */
        while (kappa < L) {
            int bits = d * kappa;
            if (bits >= 62) break;
            int64_t need = (N + ((int64_t)1 << bits) - 1) >> bits;
            if ((int64_t)leaf >= need) break;
            ++kappa;
        }
    }
    h->kappa = kappa;
    for (int l = 0; l <= kappa; ++l) build_level(h, l);
    build_flags(h);
    for (int l = 1; l <= kappa; ++l) build_lists(h, l);
    for (int l = 0; l <= kappa; ++l) build_near(h, l);
    *status = ORK_OK;
    return h;
}

void ohodlr_destroy(ohodlr* h)
{
    if (!h) return;
    for (int l = 0; l <= h->kappa; ++l) {
        olevel* L = &h->lev[l];
        free(L->start); free(L->key); free(L->coord); free(L->flag);
        free(L->near_ptr); free(L->near_col);
        if (L->il_ptr) {
            int64_t nnz = L->il_ptr[L->nb];
            for (int64_t e = 0; e < nnz; ++e) { free(L->U[e]); free(L->V[e]); }
            free(L->il_ptr); free(L->il_col); free(L->rank); free(L->U); free(L->V);
        }
    }
    free(h->pts_user); free(h->pts); free(h->q); free(h->key); free(h->perm);
    free(h);
}

int ohodlr_kappa(const ohodlr* h) { return h->kappa; }
int ohodlr_lmax(const ohodlr* h) { return h->Lmax; }
void ohodlr_domain(const ohodlr* h, double* lo, double* side)
{
    for (int a = 0; a < h->d; ++a) lo[a] = h->lo[a];
    *side = h->side;
}
void ohodlr_perm(const ohodlr* h, int64_t* perm) { memcpy(perm, h->perm, sizeof(int64_t) * h->N); }
void ohodlr_keys(const ohodlr* h, uint64_t* keys) { memcpy(keys, h->key, sizeof(uint64_t) * h->N); }
void ohodlr_quantized(const ohodlr* h, int64_t* q) { memcpy(q, h->q, sizeof(int64_t) * h->N * h->d); }
int64_t ohodlr_nboxes(const ohodlr* h, int level)
{
    if (level < 0 || level > h->kappa) return -1;
    return h->lev[level].nb;
}
void ohodlr_boxes(const ohodlr* h, int level, int64_t* start, uint64_t* key, int32_t* coord)
{
    const olevel* L = &h->lev[level];
    memcpy(start, L->start, sizeof(int64_t) * (L->nb + 1));
    memcpy(key, L->key, sizeof(uint64_t) * L->nb);
    memcpy(coord, L->coord, sizeof(int32_t) * L->nb * h->d);
}
int64_t ohodlr_il_nnz(const ohodlr* h, int level)
{
    if (level < 1 || level > h->kappa) return -1;
    return h->lev[level].il_ptr[h->lev[level].nb];
}
void ohodlr_il(const ohodlr* h, int level, int64_t* ptr, int32_t* col)
{
    const olevel* L = &h->lev[level];
    memcpy(ptr, L->il_ptr, sizeof(int64_t) * (L->nb + 1));
    memcpy(col, L->il_col, sizeof(int32_t) * L->il_ptr[L->nb]);
}
int64_t ohodlr_near_nnz(const ohodlr* h) { return ohodlr_near_level_nnz(h, h->kappa); }
void ohodlr_near(const ohodlr* h, int64_t* ptr, int32_t* col)
{
    ohodlr_near_level(h, h->kappa, ptr, col);
}
int64_t ohodlr_near_level_nnz(const ohodlr* h, int level)
{
    if (level < 0 || level > h->kappa) return -1;
    return h->lev[level].near_ptr[h->lev[level].nb];
}
void ohodlr_near_level(const ohodlr* h, int level, int64_t* ptr, int32_t* col)
{
    const olevel* L = &h->lev[level];
    memcpy(ptr, L->near_ptr, sizeof(int64_t) * (L->nb + 1));
    memcpy(col, L->near_col, sizeof(int32_t) * L->near_ptr[L->nb]);
}
void ohodlr_box_flags(const ohodlr* h, int level, uint8_t* flags)
{
    const olevel* L = &h->lev[level];
    memcpy(flags, L->flag, (size_t)L->nb);
}

/* ------------------------------------------------------------------------- */
/* ACA with partial pivoting (Bebendorf; Tyrtyshnikov), eq. keq1.
 * The approximation is the sum of rank-one terms u_k v_k^T where v_k is the
 * residual of the pivot row scaled by its largest entry and u_k the residual
 * of the pivot column.  A candidate term is "small" when |u||v| <= tol |S|_F,
 * S the approximation including it.  At a small term the stop is confirmed
 * on samples of the residual of the approximation without it: 16 evenly
 * spaced rows and 16 evenly spaced columns (all of them in a smaller block;
 * the c-th confirmation of a block shifts them by 997c and 991c modulo the
 * spacing), each sum of squares scaled to an estimate of |K - S|_F^2.  The
 * iteration ends, dropping the small term, when both estimates are at most
 * (tol/2)^2 |S|_F^2 (half the tolerance: a residual gathered near a shared
 * hyper-surface can hide from the samples).  Otherwise the term is kept and
 * the next pivot row is the untried row holding the largest sampled residual
 * entry.  The iteration also ends when the rank reaches its cap or every row
 * was tried.
 * ------------------------------------------------------------------------- */
typedef double (*entry_fn)(const void* ctx, int64_t i, int64_t j);

typedef struct {
    double* U; double* V;     /* growable: U column k at U[k*m], V row k at V[k*n] */
    int64_t cap;
    int64_t* piv_r; int64_t* piv_c;
} aca_out;

static int grow(aca_out* o, int64_t m, int64_t n, int64_t need)
{
    if (need <= o->cap) return 1;
    int64_t nc = o->cap ? o->cap * 2 : 8;
    while (nc < need) nc *= 2;
    double* U = (double*)realloc(o->U, sizeof(double) * m * nc);
    if (!U) return 0;
    o->U = U;
    double* V = (double*)realloc(o->V, sizeof(double) * n * nc);
    if (!V) return 0;
    o->V = V;
    int64_t* pr = (int64_t*)realloc(o->piv_r, sizeof(int64_t) * nc);
    int64_t* pc = (int64_t*)realloc(o->piv_c, sizeof(int64_t) * nc);
    if (!pr || !pc) return 0;
    o->piv_r = pr; o->piv_c = pc;
    o->cap = nc;
    return 1;
}

/* residual entry K(i,j) - sum_{p<k} U[p][i] V[p][j] */
static double resid(entry_fn E, const void* ctx, const aca_out* o, int64_t m, int64_t n,
                    int64_t k, int64_t i, int64_t j)
{
    double s = E(ctx, i, j);
    for (int64_t p = 0; p < k; ++p) s -= o->U[p * m + i] * o->V[p * n + j];
    return s;
}

enum { ACA_SAMPLES = 16 };

/* Sampled confirmation of a stop (check number c of this block).  Returns 1
 * when both scaled estimates of |K - S|_F^2 are at most (tol/2)^2 S2; otherwise
 * 0 and *next = the untried row of the largest sampled residual entry (-1 if
 * every sampled entry of an untried row is zero). */
static int aca_confirm(entry_fn E, const void* ctx, const aca_out* o, int64_t m, int64_t n,
                       int64_t k, double tol, double S2, int64_t c, const char* used,
                       int64_t* next)
{
    int64_t sr = m < ACA_SAMPLES ? m : ACA_SAMPLES, str = m / sr;
    int64_t sc = n < ACA_SAMPLES ? n : ACA_SAMPLES, stc = n / sc;
    int64_t offr = (c * 997) % str, offc = (c * 991) % stc;
    double er = 0.0, ec = 0.0, best = 0.0;
    int64_t bi = -1;
    for (int64_t t = 0; t < sr; ++t) {
        int64_t i = t * str + offr;
        for (int64_t j = 0; j < n; ++j) {
            double v = resid(E, ctx, o, m, n, k, i, j);
            er += v * v;
            if (!used[i] && (fabs(v) > best || (fabs(v) == best && bi >= 0 && i < bi))) {
                best = fabs(v);
                bi = i;
            }
        }
    }
    for (int64_t t = 0; t < sc; ++t) {
        int64_t j = t * stc + offc;
        for (int64_t i = 0; i < m; ++i) {
            double v = resid(E, ctx, o, m, n, k, i, j);
            ec += v * v;
            if (!used[i] && (fabs(v) > best || (fabs(v) == best && bi >= 0 && i < bi))) {
                best = fabs(v);
                bi = i;
            }
        }
    }
    er *= (double)m / (double)sr;
    ec *= (double)n / (double)sc;
    *next = bi;
    const double lim = 0.25 * tol * tol * S2;
    return er <= lim && ec <= lim;
}

static int aca_core(entry_fn E, const void* ctx, int64_t m, int64_t n, double tol,
                    int64_t kmax, aca_out* o)
{
    int64_t k = 0;
    double S2 = 0.0;
    char* used = (char*)calloc((size_t)m, 1);
    double* r = (double*)malloc(sizeof(double) * n);
    int64_t nused = 0;
    int64_t istar = 0;
    int64_t nchecks = 0;    /* sampled confirmations done */
    while (k < kmax) {
        /* residual of the pivot row */
        for (int64_t j = 0; j < n; ++j) r[j] = resid(E, ctx, o, m, n, k, istar, j);
        int64_t jstar = 0;
        for (int64_t j = 1; j < n; ++j)
            if (fabs(r[j]) > fabs(r[jstar])) jstar = j;
        if (!used[istar]) { used[istar] = 1; ++nused; }
        if (r[jstar] == 0.0) {
            if (nused == m) break;
            int64_t i = 0;
            while (used[i]) ++i;
            istar = i;
            continue;
        }
        if (!grow(o, m, n, k + 1)) { free(used); free(r); return -1; }
        double piv = r[jstar];
        double* v = o->V + k * n;
        double* u = o->U + k * m;
        for (int64_t j = 0; j < n; ++j) v[j] = r[j] / piv;
        for (int64_t i = 0; i < m; ++i) u[i] = resid(E, ctx, o, m, n, k, i, jstar);
        double nu2 = 0.0, nv2 = 0.0;
        for (int64_t i = 0; i < m; ++i) nu2 += u[i] * u[i];
        for (int64_t j = 0; j < n; ++j) nv2 += v[j] * v[j];
        double cross = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double du = 0.0, dv = 0.0;
            for (int64_t i = 0; i < m; ++i) du += o->U[p * m + i] * u[i];
            for (int64_t j = 0; j < n; ++j) dv += o->V[p * n + j] * v[j];
            cross += du * dv;
        }
        double S2new = S2 + 2.0 * cross + nu2 * nv2;
        int64_t next = -1;
        /* a small candidate term: stop without it if the samples of the
         * residual confirm the tolerance, else keep it and go on */
        if (k > 0 && sqrt(nu2 * nv2) <= tol * sqrt(S2new) &&
            aca_confirm(E, ctx, o, m, n, k, tol, S2, nchecks++, used, &next))
            break;
        S2 = S2new;
        o->piv_r[k] = istar;
        o->piv_c[k] = jstar;
        ++k;
        if (nused == m) break;
        if (next < 0) {
            /* next pivot row: largest |u_i| among rows not tried yet */
            for (int64_t i = 0; i < m; ++i)
                if (!used[i] && (next < 0 || fabs(u[i]) > fabs(u[next]))) next = i;
        }
        istar = next;
    }
    free(used); free(r);
    return (int)k;
}

typedef struct { const double* M; int64_t n; } dense_ctx;
static double dense_entry(const void* c, int64_t i, int64_t j)
{
    const dense_ctx* x = (const dense_ctx*)c;
    return x->M[i * x->n + j];
}

int ohodlr_aca_dense(const double* M, int64_t m, int64_t n, double tol, int max_rank,
                     double* U, double* V, int64_t* piv_row, int64_t* piv_col)
{
    int64_t kmax = m < n ? m : n;
    if (max_rank > 0 && max_rank < kmax) kmax = max_rank;
    dense_ctx c = {M, n};
    aca_out o = {0};
    int r = aca_core(dense_entry, &c, m, n, tol, kmax, &o);
    if (r > 0) {
        memcpy(U, o.U, sizeof(double) * m * r);
        memcpy(V, o.V, sizeof(double) * n * r);
        memcpy(piv_row, o.piv_r, sizeof(int64_t) * r);
        memcpy(piv_col, o.piv_c, sizeof(int64_t) * r);
    }
    free(o.U); free(o.V); free(o.piv_r); free(o.piv_c);
    return r;
}

typedef struct {
    const ork_kernel* k; const double* pts; int d;
    int64_t i0, j0;   /* tree-order offsets of the row and column boxes */
    const int64_t* perm;
} blk_ctx;
static double blk_entry(const void* c, int64_t i, int64_t j)
{
    const blk_ctx* x = (const blk_ctx*)c;
    int64_t pi = x->i0 + i, pj = x->j0 + j;
    if (x->perm[pi] == x->perm[pj]) return x->k->diag;
    return ohodlr_kernel_eval(x->k, x->pts + pi * x->d, x->pts + pj * x->d, x->d);
}

int ohodlr_compress(ohodlr* h, const ork_kernel* k, double tol, int max_rank,
                    int64_t row0, int64_t row1)
{
    int status = ORK_OK;
    for (int l = 1; l <= h->kappa; ++l) {
        olevel* L = &h->lev[l];
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t A = 0; A < L->nb; ++A) {
            if (L->start[A] < row0 || L->start[A + 1] > row1) continue;
            for (int64_t e = L->il_ptr[A]; e < L->il_ptr[A + 1]; ++e) {
                int64_t B = L->il_col[e];
                int64_t m = L->start[A + 1] - L->start[A];
                int64_t n = L->start[B + 1] - L->start[B];
                int64_t kmax = m < n ? m : n;
                if (max_rank > 0 && max_rank < kmax) kmax = max_rank;
                blk_ctx c = {k, h->pts, h->d, L->start[A], L->start[B], h->perm};
                aca_out o = {0};
                int r = aca_core(blk_entry, &c, m, n, tol, kmax, &o);
                if (r < 0) {
#pragma omp atomic write
                    status = ORK_ENOMEM;
                    r = 0;
                }
                free(L->U[e]); free(L->V[e]);
                L->U[e] = r > 0 ? (double*)realloc(o.U, sizeof(double) * m * r) : NULL;
                L->V[e] = r > 0 ? (double*)realloc(o.V, sizeof(double) * n * r) : NULL;
                if (r <= 0) { free(o.U); free(o.V); }
                free(o.piv_r); free(o.piv_c);
                L->rank[e] = r;
            }
        }
    }
    return status;
}

void ohodlr_ranks(const ohodlr* h, int level, int32_t* ranks)
{
    const olevel* L = &h->lev[level];
    memcpy(ranks, L->rank, sizeof(int32_t) * L->il_ptr[L->nb]);
}

int64_t ohodlr_factor_elems(const ohodlr* h, int level, int which)
{
    const olevel* L = &h->lev[level];
    int64_t tot = 0;
    for (int64_t A = 0; A < L->nb; ++A)
        for (int64_t e = L->il_ptr[A]; e < L->il_ptr[A + 1]; ++e) {
            int64_t B = L->il_col[e];
            int64_t r = L->rank[e] > 0 ? L->rank[e] : 0;
            int64_t sz = which == 0 ? L->start[A + 1] - L->start[A] : L->start[B + 1] - L->start[B];
            tot += r * sz;
        }
    return tot;
}

void ohodlr_factors(const ohodlr* h, int level, double* U, double* V)
{
    const olevel* L = &h->lev[level];
    int64_t ou = 0, ov = 0;
    for (int64_t A = 0; A < L->nb; ++A)
        for (int64_t e = L->il_ptr[A]; e < L->il_ptr[A + 1]; ++e) {
            int64_t B = L->il_col[e];
            int64_t r = L->rank[e] > 0 ? L->rank[e] : 0;
            int64_t m = L->start[A + 1] - L->start[A];
            int64_t n = L->start[B + 1] - L->start[B];
            if (r) {
                memcpy(U + ou, L->U[e], sizeof(double) * m * r);
                memcpy(V + ov, L->V[e], sizeof(double) * n * r);
            }
            ou += m * r;
            ov += n * r;
        }
}

int ohodlr_set_factors(ohodlr* h, int level, const int32_t* ranks, const double* U, const double* V)
{
    if (level < 1 || level > h->kappa) return ORK_EINVAL;
    olevel* L = &h->lev[level];
    int64_t ou = 0, ov = 0;
    for (int64_t A = 0; A < L->nb; ++A)
        for (int64_t e = L->il_ptr[A]; e < L->il_ptr[A + 1]; ++e) {
            int64_t B = L->il_col[e];
            int64_t r = ranks[e];
            int64_t m = L->start[A + 1] - L->start[A];
            int64_t n = L->start[B + 1] - L->start[B];
            if (r < 0 || r > (m < n ? m : n)) return ORK_EINVAL;
            free(L->U[e]); free(L->V[e]);
            L->U[e] = L->V[e] = NULL;
            if (r) {
                L->U[e] = (double*)malloc(sizeof(double) * m * r);
                L->V[e] = (double*)malloc(sizeof(double) * n * r);
                memcpy(L->U[e], U + ou, sizeof(double) * m * r);
                memcpy(L->V[e], V + ov, sizeof(double) * n * r);
            }
            L->rank[e] = (int32_t)r;
            ou += m * r;
            ov += n * r;
        }
    return ORK_OK;
}

/* ------------------------------------------------------------------------- */
/* Matrix-vector product, Alg. "HODLRdD matrix-vector Product":                */
/* low-rank blocks of every level, then the dense self and d'>=1 neighbour     */
/* blocks at the leaves (formed entry by entry here).                          */
/* ------------------------------------------------------------------------- */
int ohodlr_matvec(const ohodlr* h, const ork_kernel* k, const double* q, int nrhs,
                  double* b, int64_t row0, int64_t row1)
{
    const int64_t N = h->N;
    const int d = h->d;
    for (int l = 1; l <= h->kappa; ++l) {
        const olevel* L = &h->lev[l];
        for (int64_t A = 0; A < L->nb; ++A) {
            if (L->start[A] < row0 || L->start[A + 1] > row1) continue;
            for (int64_t e = L->il_ptr[A]; e < L->il_ptr[A + 1]; ++e)
                if (L->rank[e] < 0) return ORK_EINVAL;
        }
    }
    double* x = (double*)malloc(sizeof(double) * N);
    double* y = (double*)malloc(sizeof(double) * N);
    int64_t maxr = 1;
    for (int l = 1; l <= h->kappa; ++l) {
        const olevel* L = &h->lev[l];
        for (int64_t e = 0; e < L->il_ptr[L->nb]; ++e)
            if (L->rank[e] > maxr) maxr = L->rank[e];
    }
    for (int c = 0; c < nrhs; ++c) {
        const double* qc = q + (int64_t)c * N;
        for (int64_t p = 0; p < N; ++p) { x[p] = qc[h->perm[p]]; y[p] = 0.0; }
        /* low-rank part, level by level */
        for (int l = 1; l <= h->kappa; ++l) {
            const olevel* L = &h->lev[l];
#pragma omp parallel
            {
                double* t = (double*)malloc(sizeof(double) * maxr);
#pragma omp for schedule(dynamic, 1)
                for (int64_t A = 0; A < L->nb; ++A) {
                    if (L->start[A] < row0 || L->start[A + 1] > row1) continue;
                    int64_t a0 = L->start[A], m = L->start[A + 1] - a0;
                    for (int64_t e = L->il_ptr[A]; e < L->il_ptr[A + 1]; ++e) {
                        int64_t B = L->il_col[e];
                        int64_t b0 = L->start[B], n = L->start[B + 1] - b0;
                        int64_t r = L->rank[e];
                        for (int64_t p = 0; p < r; ++p) {
                            double s = 0.0;
                            for (int64_t j = 0; j < n; ++j) s += L->V[e][p * n + j] * x[b0 + j];
                            t[p] = s;
                        }
                        for (int64_t i = 0; i < m; ++i) {
                            double s = 0.0;
                            for (int64_t p = 0; p < r; ++p) s += L->U[e][p * m + i] * t[p];
                            y[a0 + i] += s;
                        }
                    }
                }
                free(t);
            }
        }
        /* dense near-field pairs of every level (only level kappa in a
         * uniform tree) */
        for (int l = 0; l <= h->kappa; ++l) {
            const olevel* L = &h->lev[l];
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t A = 0; A < L->nb; ++A) {
                if (L->near_ptr[A] == L->near_ptr[A + 1]) continue;
                if (L->start[A] < row0 || L->start[A + 1] > row1) continue;
                for (int64_t i = L->start[A]; i < L->start[A + 1]; ++i) {
                    double s = 0.0;
                    for (int64_t e = L->near_ptr[A]; e < L->near_ptr[A + 1]; ++e) {
                        int64_t B = L->near_col[e];
                        for (int64_t j = L->start[B]; j < L->start[B + 1]; ++j) {
                            double kij = h->perm[i] == h->perm[j]
                                             ? k->diag
                                             : ohodlr_kernel_eval(k, h->pts + i * d, h->pts + j * d, d);
                            s += kij * x[j];
                        }
                    }
                    y[i] += s;
                }
            }
        }
        double* bc = b + (int64_t)c * N;
        for (int64_t p = 0; p < N; ++p) bc[h->perm[p]] = (p >= row0 && p < row1) ? y[p] : 0.0;
        /* rows outside the range keep 0 (y[p] may hold partial sums there) */
    }
    free(x); free(y);
    return ORK_OK;
}

/* The plain definition: b_i = sum_j K(i,j) q_j. */
void ohodlr_direct(const double* P, int64_t N, int d, const ork_kernel* k,
                   const double* q, int nrhs, const int64_t* rows, int64_t nrows,
                   double* b)
{
    int64_t R = rows ? nrows : N;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < R; ++t) {
        int64_t i = rows ? rows[t] : t;
        for (int c = 0; c < nrhs; ++c) {
            const double* qc = q + (int64_t)c * N;
            double s = 0.0;
            for (int64_t j = 0; j < N; ++j) s += entry(k, P, d, i, j) * qc[j];
            b[(int64_t)c * R + t] = s;
        }
    }
}
