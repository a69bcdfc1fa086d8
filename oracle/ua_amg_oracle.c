/*
 * ua_amg_oracle.c -- serial FP64 reference of unsmoothed-aggregation AMG
 * (Brannick, Chen, Hu, Zikatanov, "Parallel Unsmoothed Aggregation Algebraic
 * Multigrid Algorithms on GPUs").
 *
 * TEST INFRASTRUCTURE.  This file is the correctness oracle of the HIP library:
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or helper with the GPU library, and
 * it is written for a reader checking it against the paper, not for speed.
 *
 * What it computes, in the paper's order:
 *   Sec. 2, eq. (2.2)-(2.4): piecewise-constant P from a partition into aggregates,
 *       A_c = P^T A P evaluated as sums of fine entries over aggregate pairs.
 *   Sec. 3.2, eq. (3.2): priorities v_i = d_i + ((i mod 12) + rand())/12.
 *   Sec. 3.1-3.2, Alg. 2: parallel aggregation in synchronous passes; a pass
 *       (A) picks the unprocessed vertices whose priority beats every unprocessed
 *       vertex within graph distance 1 or 2, (B) forms an aggregate around each.
 *   Sec. 5.1: aggregate k is the one whose coarse vertex is the k-th smallest index.
 *   Alg. 1: the setup loop over levels.
 *   Sec. 4.1: l1-Jacobi smoother M_ii = a_ii + sum_{j!=i} |a_ij|, or the damped
 *       Jacobi smoother M^-1 = omega D^-1 (option).
 *   Sec. 4.2: prolongation (Pv)_i = v[agg[i]], restriction (P^T v)_I = sum_{agg[j]=I} v_j.
 *   Sec. 4.3-4.4: K-cycle (nonlinear AMLI cycle: nu flexible-CG steps on every
 *       coarse level, preconditioned recursively) as the preconditioner of an
 *       outer nonlinear (flexible) preconditioned CG.
 *
 * Readings taken where the paper is silent or ambiguous (each also listed in the
 * design notes of the repository):
 *   - d_i is the number of structural off-diagonal entries of row i of A_l.
 *   - i in (i mod 12) is the 0-based, level-local index.
 *   - rand() for vertex i on level l is fmix32(i XOR s_l)/2^32, fmix32 being the
 *     MurmurHash3 32-bit finaliser (a bijection) and s_l the low 32 bits of the
 *     (l+1)-th output of SplitMix64 seeded with the user seed.  Priorities are then
 *     unique, so the strict comparisons of Alg. 2 never tie.  They are compared
 *     exactly as the integer 2^32 * 12 * v_i = (12 d_i + (i mod 12)) 2^32 + hash.
 *   - "Distance 1 or 2 among unprocessed vertices" is measured in the graph that
 *     remains after processed vertices are removed (Sec. 3.1: the selection is
 *     re-applied to the remaining graph).
 *   - An aggregate is its coarse vertex plus its unprocessed neighbours (distance
 *     1); with a size limit t only the first t-1 such neighbours in ascending
 *     index join it and the others stay unprocessed for later passes.
 *   - Setup continues while n_l > n_0 and l+1 < L; a level whose aggregation keeps
 *     more than stall_ratio * n_l aggregates is not built (coarsening stalled).
 *   - Every structural entry of A_c is kept (no dropping).
 *   - The coarsest level is solved with a dense Cholesky factorisation.
 *   - One pre- and one post-smoothing l1-Jacobi sweep; the pre-sweep starts from 0.
 *     The damping factor of the damped Jacobi variant is not given; it is a
 *     parameter (default 2/3).
 *   - The outer iteration stops when ||b - A x||_2 <= tol ||b||_2 for the true
 *     residual (checked when the recursive residual first says so).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MATRIX 2
#define ORC_ERR_NOMEM 3
#define ORC_ERR_NOT_CONVERGED 5
#define ORC_ERR_BREAKDOWN 6
#define ORC_ERR_INTERNAL 7

#define ORC_MAX_LEVELS 64

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers, from their published definitions.           */
/* ------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea, Flood 2014): k-th output (k = 0, 1, ...) of the
 * generator whose state starts at `seed` and advances by the golden gamma. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL * (k + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* MurmurHash3 32-bit finaliser (Appleby); a bijection on 32-bit words. */
uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6BU;
    h ^= h >> 13;
    h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

static double now_ms(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

/* ------------------------------------------------------------------------- */
/* CSR checks and products.                                                   */
/* ------------------------------------------------------------------------- */

/* Square CSR, columns strictly ascending and in range, diagonal present and > 0. */
int orc_check_csr(int n, int nnz, const int *rp, const int *ci, const double *va)
{
    if (n < 1 || nnz < n || !rp || !ci || !va) return ORC_ERR_ARG;
    if (rp[0] != 0 || rp[n] != nnz) return ORC_ERR_MATRIX;
    for (int i = 0; i < n; i++) {
        if (rp[i + 1] < rp[i]) return ORC_ERR_MATRIX;
        int diag = 0;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] < 0 || ci[p] >= n) return ORC_ERR_MATRIX;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return ORC_ERR_MATRIX;
            if (!isfinite(va[p])) return ORC_ERR_MATRIX;
            if (ci[p] == i) {
                if (!(va[p] > 0.0)) return ORC_ERR_MATRIX;
                diag = 1;
            }
        }
        if (!diag) return ORC_ERR_MATRIX;
    }
    return ORC_OK;
}

/* y = A x, each row summed in column order. */
void orc_spmv(int n, const int *rp, const int *ci, const double *va, const double *x, double *y)
{
    for (int i = 0; i < n; i++) {
        double s = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; p++) s += va[p] * x[ci[p]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------- */
/* Setup: priorities, parallel aggregation, numbering, coarse operator.       */
/* ------------------------------------------------------------------------- */

/* eq. (3.2), scaled by 12 * 2^32 so it is an exact integer:
 *   key_i = (12 d_i + (i mod 12)) * 2^32 + fmix32(i XOR s_l),
 * where d_i counts the structural off-diagonal entries of row i. */
void orc_priorities(int n, const int *rp, const int *ci, uint64_t seed, int level, uint64_t *key)
{
    uint32_t s_l = (uint32_t)orc_splitmix64(seed, (uint64_t)level);
    for (int i = 0; i < n; i++) {
        uint64_t d = 0;
        for (int p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] != i) d++;
        uint64_t whole = 12 * d + (uint64_t)(i % 12);
        key[i] = (whole << 32) | (uint64_t)orc_fmix32((uint32_t)i ^ s_l);
    }
}

/* Alg. 2 in synchronous passes.  On return owner[i] is the coarse vertex whose
 * aggregate holds i and pass_of[i] (if not NULL) the 0-based pass that processed
 * i.  cap = t (maximum aggregate size, counting the coarse vertex), 0 = no limit.
 * Returns the number of passes, or a negative error code. */
int orc_paa(int n, const int *rp, const int *ci, const uint64_t *key, int cap,
            int *owner, int *pass_of)
{
    unsigned char *unproc = (unsigned char *)malloc((size_t)n);
    unsigned char *centre = (unsigned char *)malloc((size_t)n);
    if (!unproc || !centre) {
        free(unproc);
        free(centre);
        return -ORC_ERR_NOMEM;
    }
    for (int i = 0; i < n; i++) {
        unproc[i] = 1;
        owner[i] = -1;
        if (pass_of) pass_of[i] = -1;
    }
    int remaining = n, passes = 0, err = 0;
    while (remaining > 0) {
        /* (A) / step (2b): i is a coarse vertex of this pass when its priority is
         * larger than that of every unprocessed j with 0 < d(i,j) < 3, distance
         * taken in the graph of the unprocessed vertices. */
        int found = 0;
        for (int i = 0; i < n; i++) {
            centre[i] = 0;
            if (!unproc[i]) continue;
            int is_max = 1;
            for (int p = rp[i]; p < rp[i + 1] && is_max; p++) {
                int j = ci[p];
                if (j == i || !unproc[j]) continue;
                if (key[j] > key[i]) { is_max = 0; break; }
                for (int q = rp[j]; q < rp[j + 1]; q++) {
                    int k = ci[q];
                    if (k == i || k == j || !unproc[k]) continue;
                    if (key[k] > key[i]) { is_max = 0; break; }
                }
            }
            centre[i] = (unsigned char)is_max;
            found += is_max;
        }
        if (found == 0) { err = ORC_ERR_INTERNAL; break; }
        /* (B) / step (2c): the aggregate of coarse vertex i is i and its
         * unprocessed neighbours, ascending, at most cap-1 of them. */
        for (int i = 0; i < n && !err; i++) {
            if (!centre[i]) continue;
            if (owner[i] != -1) { err = ORC_ERR_INTERNAL; break; }
            owner[i] = i;
            int size = 1;
            for (int p = rp[i]; p < rp[i + 1]; p++) {
                int j = ci[p];
                if (j == i || !unproc[j]) continue;
                if (cap > 0 && size >= cap) break;
                if (owner[j] != -1) { err = ORC_ERR_INTERNAL; break; } /* two centres share j */
                owner[j] = i;
                size++;
            }
        }
        if (err) break;
        /* step (2e): everything claimed in this pass is now processed */
        for (int i = 0; i < n; i++) {
            if (unproc[i] && owner[i] != -1) {
                unproc[i] = 0;
                remaining--;
                if (pass_of) pass_of[i] = passes;
            }
        }
        passes++;
    }
    free(unproc);
    free(centre);
    return err ? -err : passes;
}

/* Sec. 5.1: column k of P belongs to the aggregate whose coarse vertex has the
 * k-th smallest index.  Writes agg[i] = column of the aggregate of i; returns n_c. */
int orc_number(int n, const int *owner, int *agg)
{
    int *col_of = (int *)malloc(sizeof(int) * (size_t)n);
    if (!col_of) return -ORC_ERR_NOMEM;
    int nc = 0;
    for (int i = 0; i < n; i++) col_of[i] = (owner[i] == i) ? nc++ : -1;
    for (int i = 0; i < n; i++) agg[i] = col_of[owner[i]];
    free(col_of);
    return nc;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* eq. (2.4): (A_c)_{IJ} = sum_{s in G_I} sum_{t in G_J} a_{st}.  Rows are built
 * one at a time: for the members s of G_I in ascending order and the entries of
 * row s in column order, a_{st} is added to the accumulator of column agg[t].
 * Every structural entry is kept; columns come out ascending.  The caller frees
 * *out_rp, *out_ci, *out_va. */
int orc_coarse_operator(int n, const int *rp, const int *ci, const double *va, const int *agg,
                        int nc, int **out_rp, int **out_ci, double **out_va)
{
    int nnz = rp[n];
    int *mptr = (int *)calloc((size_t)nc + 1, sizeof(int));
    int *mem = (int *)malloc(sizeof(int) * (size_t)n);
    int *mark = (int *)malloc(sizeof(int) * (size_t)nc);
    double *acc = (double *)malloc(sizeof(double) * (size_t)nc);
    int *cols = (int *)malloc(sizeof(int) * (size_t)nc);
    int *crp = (int *)malloc(sizeof(int) * ((size_t)nc + 1));
    int *cci = (int *)malloc(sizeof(int) * (size_t)nnz);
    double *cva = (double *)malloc(sizeof(double) * (size_t)nnz);
    if (!mptr || !mem || !mark || !acc || !cols || !crp || !cci || !cva) {
        free(mptr); free(mem); free(mark); free(acc); free(cols); free(crp); free(cci); free(cva);
        return ORC_ERR_NOMEM;
    }
    /* members of every aggregate, ascending (counting sort by agg, stable in i) */
    for (int i = 0; i < n; i++) mptr[agg[i] + 1]++;
    for (int I = 0; I < nc; I++) mptr[I + 1] += mptr[I];
    {
        int *fill = (int *)malloc(sizeof(int) * (size_t)nc);
        if (!fill) {
            free(mptr); free(mem); free(mark); free(acc); free(cols); free(crp); free(cci); free(cva);
            return ORC_ERR_NOMEM;
        }
        memcpy(fill, mptr, sizeof(int) * (size_t)nc);
        for (int i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
        free(fill);
    }
    for (int J = 0; J < nc; J++) mark[J] = -1;
    int out = 0;
    crp[0] = 0;
    for (int I = 0; I < nc; I++) {
        int ncols = 0;
        for (int m = mptr[I]; m < mptr[I + 1]; m++) {
            int s = mem[m];
            for (int p = rp[s]; p < rp[s + 1]; p++) {
                int J = agg[ci[p]];
                if (mark[J] != I) {
                    mark[J] = I;
                    acc[J] = 0.0;
                    cols[ncols++] = J;
                }
                acc[J] += va[p];
            }
        }
        qsort(cols, (size_t)ncols, sizeof(int), cmp_int);
        for (int q = 0; q < ncols; q++) {
            cci[out] = cols[q];
            cva[out] = acc[cols[q]];
            out++;
        }
        crp[I + 1] = out;
    }
    free(mptr); free(mem); free(mark); free(acc); free(cols);
    *out_rp = crp;
    *out_ci = (int *)realloc(cci, sizeof(int) * (size_t)(out > 0 ? out : 1));
    *out_va = (double *)realloc(cva, sizeof(double) * (size_t)(out > 0 ? out : 1));
    return ORC_OK;
}

/* Sec. 4.1: l1-Jacobi, minv_i = 1 / (a_ii + sum_{j != i} |a_ij|). */
void orc_l1_inverse_diagonal(int n, const int *rp, const int *ci, const double *va, double *minv)
{
    for (int i = 0; i < n; i++) {
        double diag = 0.0, off = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] == i) diag += va[p];
            else off += fabs(va[p]);
        }
        minv[i] = 1.0 / (diag + off);
    }
}

/* Sec. 4.1: damped Jacobi, x <- x + omega D^-1 (b - A x), i.e. minv_i = omega / a_ii. */
void orc_jacobi_inverse_diagonal(int n, const int *rp, const int *ci, const double *va, double omega, double *minv)
{
    for (int i = 0; i < n; i++) {
        double diag = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] == i) diag += va[p];
        minv[i] = omega / diag;
    }
}

/* ------------------------------------------------------------------------- */
/* Hierarchy.                                                                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n, nnz;
    int *rp, *ci;
    double *va;
    double *minv;
    int *agg;    /* n entries: coarse column of each vertex (all but the coarsest level) */
    int passes;  /* PAA passes that built the aggregation of this level */
    /* work vectors of the solve */
    double *tmp, *rc, *e, *rr, *w, *aw, *d, *ad, *dp, *adp, *x, *r, *p, *q, *z;
} orc_level;

/* Lower Cholesky factor L of the coarsest matrix, kept as the lists of its nonzero
 * entries: row i's entries left of the diagonal (ascending column) and column i's
 * entries below it (ascending row), plus the diagonal.  The substitutions visit
 * them in the order a dense loop would and skip only exact zeros, whose products
 * change no nonzero sum (the coarsest level of a random graph is mostly isolated
 * vertices, whose rows and columns of L are empty). */
typedef struct {
    int n;
    double *diag;
    int *rptr, *rcol;  /* row i: rcol[rptr[i] .. rptr[i+1]) < i */
    double *rval;
    int *cptr, *crow;  /* column i: crow[cptr[i] .. cptr[i+1]) > i */
    double *cval;
} orc_factor;

static void free_factor(orc_factor *f)
{
    free(f->diag); free(f->rptr); free(f->rcol); free(f->rval);
    free(f->cptr); free(f->crow); free(f->cval);
    memset(f, 0, sizeof(*f));
}

typedef struct {
    int nlev;
    orc_level lev[ORC_MAX_LEVELS];
    orc_factor chol; /* Cholesky factor of the coarsest matrix */
    int nu;       /* inner flexible-CG steps per coarse level visit */
    double theta; /* K-cycle threshold: later inner steps are skipped once ||rr|| < theta ||g|| */
    double setup_ms;
    int breakdown;
} orc_hierarchy;

typedef struct {
    int coarsest_size;    /* n_0 */
    int max_levels;       /* L */
    double stall_ratio;
    int max_aggregate;    /* t, 0 = unlimited */
    uint64_t seed;
    int kcycle_inner;     /* nu */
    int smoother;         /* 0: l1-Jacobi, 1: damped Jacobi */
    double jacobi_weight; /* omega of the damped Jacobi smoother */
    double kcycle_threshold; /* theta >= 0; 0 = always nu inner steps */
    double skip_ratio;       /* aggregate twice when n_l / n_c < skip_ratio (Sec. 3.3); 0 = never */
} orc_options;

static void free_level(orc_level *L, int own_matrix)
{
    if (own_matrix) {
        free(L->rp); free(L->ci); free(L->va);
    }
    free(L->minv); free(L->agg);
    free(L->tmp); free(L->rc); free(L->e); free(L->rr); free(L->w); free(L->aw);
    free(L->d); free(L->ad); free(L->dp); free(L->adp); free(L->x); free(L->r);
    free(L->p); free(L->q); free(L->z);
    memset(L, 0, sizeof(*L));
}

void orc_free(orc_hierarchy *h)
{
    if (!h) return;
    for (int l = 0; l < h->nlev; l++) free_level(&h->lev[l], 1);
    free_factor(&h->chol);
    free(h);
}

static int alloc_work(orc_level *L)
{
    size_t b = sizeof(double) * (size_t)L->n;
    double **v[] = {&L->tmp, &L->rc, &L->e, &L->rr, &L->w, &L->aw, &L->d, &L->ad,
                    &L->dp, &L->adp, &L->x, &L->r, &L->p, &L->q, &L->z};
    for (size_t k = 0; k < sizeof(v) / sizeof(v[0]); k++) {
        *v[k] = (double *)calloc(1, b);
        if (!*v[k]) return ORC_ERR_NOMEM;
    }
    return ORC_OK;
}

/* Dense Cholesky A = L L^T of the CSR matrix, then the nonzero entries of L. */
static int dense_cholesky(int n, const int *rp, const int *ci, const double *va, orc_factor *out)
{
    double *a = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    if (!a) return ORC_ERR_NOMEM;
    for (int i = 0; i < n; i++)
        for (int p = rp[i]; p < rp[i + 1]; p++) a[(size_t)i * n + ci[p]] = va[p];
    for (int j = 0; j < n; j++) {
        double s = a[(size_t)j * n + j];
        for (int k = 0; k < j; k++) s -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(s > 0.0)) {
            free(a);
            return ORC_ERR_BREAKDOWN;
        }
        double ljj = sqrt(s);
        a[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; i++) {
            double t = a[(size_t)i * n + j];
            for (int k = 0; k < j; k++) t -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = t / ljj;
        }
    }
    orc_factor f;
    memset(&f, 0, sizeof(f));
    f.n = n;
    size_t nz = 0;
    for (int i = 0; i < n; i++)
        for (int k = 0; k < i; k++) nz += a[(size_t)i * n + k] != 0.0;
    f.diag = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    f.rptr = (int *)calloc((size_t)n + 1, sizeof(int));
    f.cptr = (int *)calloc((size_t)n + 1, sizeof(int));
    f.rcol = (int *)malloc(sizeof(int) * (nz + 1));
    f.crow = (int *)malloc(sizeof(int) * (nz + 1));
    f.rval = (double *)malloc(sizeof(double) * (nz + 1));
    f.cval = (double *)malloc(sizeof(double) * (nz + 1));
    if (!f.diag || !f.rptr || !f.cptr || !f.rcol || !f.crow || !f.rval || !f.cval) {
        free(a);
        free_factor(&f);
        return ORC_ERR_NOMEM;
    }
    size_t e = 0;
    for (int i = 0; i < n; i++) {
        f.diag[i] = a[(size_t)i * n + i];
        for (int k = 0; k < i; k++)
            if (a[(size_t)i * n + k] != 0.0) {
                f.rcol[e] = k;
                f.rval[e] = a[(size_t)i * n + k];
                e++;
            }
        f.rptr[i + 1] = (int)e;
    }
    e = 0;
    for (int i = 0; i < n; i++) {
        for (int k = i + 1; k < n; k++)
            if (a[(size_t)k * n + i] != 0.0) {
                f.crow[e] = k;
                f.cval[e] = a[(size_t)k * n + i];
                e++;
            }
        f.cptr[i + 1] = (int)e;
    }
    free(a);
    *out = f;
    return ORC_OK;
}

/* L L^T x = b: forward substitution by rows of L, back substitution by columns. */
static void cholesky_solve(const orc_factor *f, const double *b, double *x)
{
    const int n = f->n;
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int p = f->rptr[i]; p < f->rptr[i + 1]; p++) s -= f->rval[p] * x[f->rcol[p]];
        x[i] = s / f->diag[i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = x[i];
        for (int p = f->cptr[i]; p < f->cptr[i + 1]; p++) s -= f->cval[p] * x[f->crow[p]];
        x[i] = s / f->diag[i];
    }
}

void orc_default_options(orc_options *o)
{
    o->coarsest_size = 64;
    o->max_levels = 40;
    o->stall_ratio = 0.9;
    o->max_aggregate = 0;
    o->seed = 0x5EED5EEDULL;
    o->kcycle_inner = 2;
    o->smoother = 0;
    o->jacobi_weight = 2.0 / 3.0;
    o->kcycle_threshold = 0.0;
    o->skip_ratio = 0.0;
}

/* One aggregation (Alg. 2 with the priorities of eq. (3.2) and the numbering of
 * Sec. 5.1) of the graph of a level; `index` selects rand()'s stream.  Returns the
 * number of aggregates (or -status) and the coarse column of every vertex. */
static int aggregate(int n, const int *rp, const int *ci, const orc_options *opt, int index, int **agg_out,
                     int *passes_out)
{
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int *owner = (int *)malloc(sizeof(int) * (size_t)n);
    int *agg = (int *)malloc(sizeof(int) * (size_t)n);
    if (!key || !owner || !agg) { free(key); free(owner); free(agg); return -ORC_ERR_NOMEM; }
    orc_priorities(n, rp, ci, opt->seed, index, key);
    int passes = orc_paa(n, rp, ci, key, opt->max_aggregate, owner, NULL);
    free(key);
    if (passes < 0) { free(owner); free(agg); return passes; }
    int nc = orc_number(n, owner, agg);
    free(owner);
    if (nc < 0) { free(agg); return nc; }
    *agg_out = agg;
    *passes_out = passes;
    return nc;
}

/* Alg. 1, setup phase.  Copies the input matrix. */
int orc_setup(int n, int nnz, const int *rp, const int *ci, const double *va,
              const orc_options *opt, orc_hierarchy **out)
{
    double t0 = now_ms();
    *out = NULL;
    if (!opt || opt->max_levels < 1 || opt->max_levels > ORC_MAX_LEVELS || opt->kcycle_inner < 1 ||
        opt->coarsest_size < 1 || opt->max_aggregate < 0 || opt->max_aggregate == 1 || opt->smoother < 0 ||
        opt->smoother > 1 || !(opt->jacobi_weight > 0.0) || !isfinite(opt->jacobi_weight) ||
        !(opt->kcycle_threshold >= 0.0) || !isfinite(opt->kcycle_threshold) || !(opt->skip_ratio >= 0.0) ||
        !isfinite(opt->skip_ratio))
        return ORC_ERR_ARG;
    int st = orc_check_csr(n, nnz, rp, ci, va);
    if (st) return st;
    orc_hierarchy *h = (orc_hierarchy *)calloc(1, sizeof(orc_hierarchy));
    if (!h) return ORC_ERR_NOMEM;
    h->nu = opt->kcycle_inner;
    h->theta = opt->kcycle_threshold;
    orc_level *L0 = &h->lev[0];
    L0->n = n;
    L0->nnz = nnz;
    L0->rp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    L0->ci = (int *)malloc(sizeof(int) * (size_t)nnz);
    L0->va = (double *)malloc(sizeof(double) * (size_t)nnz);
    h->nlev = 1;
    if (!L0->rp || !L0->ci || !L0->va) { orc_free(h); return ORC_ERR_NOMEM; }
    memcpy(L0->rp, rp, sizeof(int) * ((size_t)n + 1));
    memcpy(L0->ci, ci, sizeof(int) * (size_t)nnz);
    memcpy(L0->va, va, sizeof(double) * (size_t)nnz);

    int l = 0;
    int aggregations = 0; /* rand() of eq. (3.2) is drawn per aggregation, counted from 0 */
    while (h->lev[l].n > opt->coarsest_size && l + 1 < opt->max_levels) {
        orc_level *F = &h->lev[l];
        int passes = 0;
        int nc = aggregate(F->n, F->rp, F->ci, opt, aggregations, &F->agg, &passes);
        if (nc < 0) { orc_free(h); return -nc; }
        if ((double)nc > opt->stall_ratio * (double)F->n) { /* coarsening stalled */
            free(F->agg);
            F->agg = NULL;
            break;
        }
        aggregations++;
        F->passes = passes;
        orc_level *C = &h->lev[l + 1];
        st = orc_coarse_operator(F->n, F->rp, F->ci, F->va, F->agg, nc, &C->rp, &C->ci, &C->va);
        if (st) { orc_free(h); return st; }
        C->n = nc;
        C->nnz = C->rp[nc];
        h->nlev = l + 2;
        /* Sec. 3.3: a small coarsening ratio is compensated by applying the
         * aggregation a second time, to the coarse graph just built, and keeping only
         * the result: level l's aggregates become the unions of the second
         * aggregation's groups, and the intermediate level is not kept.  Not done
         * when the intermediate level is already coarse enough to end the hierarchy,
         * or when the second aggregation stalls. */
        if (opt->skip_ratio > 0.0 && (double)F->n < opt->skip_ratio * (double)nc && nc > opt->coarsest_size &&
            l + 2 < opt->max_levels) {
            int *agg2 = NULL, passes2 = 0;
            int nc2 = aggregate(C->n, C->rp, C->ci, opt, aggregations, &agg2, &passes2);
            if (nc2 < 0) { orc_free(h); return -nc2; }
            if ((double)nc2 <= opt->stall_ratio * (double)C->n) {
                aggregations++;
                int *rp2 = NULL, *ci2 = NULL;
                double *va2 = NULL;
                st = orc_coarse_operator(C->n, C->rp, C->ci, C->va, agg2, nc2, &rp2, &ci2, &va2);
                if (st) { free(agg2); orc_free(h); return st; }
                for (int i = 0; i < F->n; i++) F->agg[i] = agg2[F->agg[i]]; /* P = P1 P2 */
                F->passes += passes2;
                free(C->rp); free(C->ci); free(C->va);
                C->rp = rp2;
                C->ci = ci2;
                C->va = va2;
                C->n = nc2;
                C->nnz = rp2[nc2];
            }
            free(agg2);
        }
        l++;
    }
    for (int k = 0; k < h->nlev; k++) {
        orc_level *Lk = &h->lev[k];
        Lk->minv = (double *)malloc(sizeof(double) * (size_t)Lk->n);
        if (!Lk->minv || alloc_work(Lk)) { orc_free(h); return ORC_ERR_NOMEM; }
        if (opt->smoother == 1)
            orc_jacobi_inverse_diagonal(Lk->n, Lk->rp, Lk->ci, Lk->va, opt->jacobi_weight, Lk->minv);
        else
            orc_l1_inverse_diagonal(Lk->n, Lk->rp, Lk->ci, Lk->va, Lk->minv);
    }
    orc_level *Lc = &h->lev[h->nlev - 1];
    st = dense_cholesky(Lc->n, Lc->rp, Lc->ci, Lc->va, &h->chol);
    if (st) { orc_free(h); return st; }
    h->setup_ms = now_ms() - t0;
    *out = h;
    return ORC_OK;
}

int orc_num_levels(const orc_hierarchy *h) { return h ? h->nlev : 0; }
double orc_setup_ms(const orc_hierarchy *h) { return h ? h->setup_ms : 0.0; }

int orc_level_info(const orc_hierarchy *h, int l, int *n, int *nnz, int *passes)
{
    if (!h || l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    if (n) *n = h->lev[l].n;
    if (nnz) *nnz = h->lev[l].nnz;
    if (passes) *passes = h->lev[l].passes;
    return ORC_OK;
}

/* Copies level l: agg (n entries; all -1 on the coarsest), CSR, l1 inverse diagonal. */
int orc_level_export(const orc_hierarchy *h, int l, int *agg, int *rp, int *ci, double *va, double *minv)
{
    if (!h || l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    const orc_level *L = &h->lev[l];
    if (agg) {
        if (L->agg) memcpy(agg, L->agg, sizeof(int) * (size_t)L->n);
        else for (int i = 0; i < L->n; i++) agg[i] = -1;
    }
    if (rp) memcpy(rp, L->rp, sizeof(int) * ((size_t)L->n + 1));
    if (ci) memcpy(ci, L->ci, sizeof(int) * (size_t)L->nnz);
    if (va) memcpy(va, L->va, sizeof(double) * (size_t)L->nnz);
    if (minv) memcpy(minv, L->minv, sizeof(double) * (size_t)L->n);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Solve: K-cycle and outer flexible CG.                                      */
/* ------------------------------------------------------------------------- */

static void kcycle(orc_hierarchy *h, int k, const double *r, double *x);

/* nu steps of flexible CG on level c for A_c e = g from e = 0, each step
 * preconditioned by the K-cycle of level c; the result is left in lev[c].e.
 * With a threshold theta > 0 the steps after the first stop as soon as the inner
 * residual is small enough, ||rr||_2 < theta ||g||_2 (compared as squares): the
 * K-cycle's test of whether a second Krylov step is worth its recursive cost. */
static void inner_fcg(orc_hierarchy *h, int c, const double *g)
{
    orc_level *C = &h->lev[c];
    int n = C->n;
    double dad_prev = 0.0;
    for (int i = 0; i < n; i++) {
        C->e[i] = 0.0;
        C->rr[i] = g[i];
    }
    const double gg = h->theta > 0.0 ? dot(n, g, g) : 0.0;
    for (int j = 0; j < h->nu; j++) {
        if (j > 0 && h->theta > 0.0 && dot(n, C->rr, C->rr) < h->theta * h->theta * gg) return;
        kcycle(h, c, C->rr, C->w);                    /* w = B_c rr */
        orc_spmv(n, C->rp, C->ci, C->va, C->w, C->aw); /* A_c w */
        if (j == 0) {
            memcpy(C->d, C->w, sizeof(double) * (size_t)n);
            memcpy(C->ad, C->aw, sizeof(double) * (size_t)n);
        } else {
            /* new direction A_c-orthogonal to the previous one (truncation 1) */
            double gam = dot(n, C->w, C->adp) / dad_prev;
            for (int i = 0; i < n; i++) {
                C->d[i] = C->w[i] - gam * C->dp[i];
                C->ad[i] = C->aw[i] - gam * C->adp[i];
            }
        }
        double dad = dot(n, C->d, C->ad);
        if (!(dad > 0.0)) { h->breakdown = 1; return; }
        double alpha = dot(n, C->d, C->rr) / dad;
        for (int i = 0; i < n; i++) {
            C->e[i] += alpha * C->d[i];
            C->rr[i] -= alpha * C->ad[i];
        }
        memcpy(C->dp, C->d, sizeof(double) * (size_t)n);
        memcpy(C->adp, C->ad, sizeof(double) * (size_t)n);
        dad_prev = dad;
    }
}

/* x = K_k(r): one K-cycle on level k < coarsest (Alg. 1 solve phase, with the
 * coarse-grid equation solved by nu inner flexible-CG steps, Sec. 4.3). */
static void kcycle(orc_hierarchy *h, int k, const double *r, double *x)
{
    orc_level *F = &h->lev[k];
    int n = F->n;
    int L = h->nlev - 1;
    if (k == L) { /* only reached when the hierarchy has a single level */
        cholesky_solve(&h->chol, r, x);
        return;
    }
    orc_level *C = &h->lev[k + 1];
    /* pre-smoothing from x = 0 */
    for (int i = 0; i < n; i++) x[i] = F->minv[i] * r[i];
    /* restriction of the residual: rc = P^T (r - A x) */
    orc_spmv(n, F->rp, F->ci, F->va, x, F->tmp);
    for (int I = 0; I < C->n; I++) C->rc[I] = 0.0;
    for (int i = 0; i < n; i++) C->rc[F->agg[i]] += r[i] - F->tmp[i];
    /* coarse-grid correction */
    const double *e;
    if (k + 1 == L) {
        cholesky_solve(&h->chol, C->rc, C->e);
        e = C->e;
    } else {
        inner_fcg(h, k + 1, C->rc);
        e = C->e;
    }
    /* prolongation */
    for (int i = 0; i < n; i++) x[i] += e[F->agg[i]];
    /* post-smoothing */
    orc_spmv(n, F->rp, F->ci, F->va, x, F->tmp);
    for (int i = 0; i < n; i++) x[i] += F->minv[i] * (r[i] - F->tmp[i]);
}

/* z = K_0(r), exposed for tests. */
int orc_kcycle_apply(orc_hierarchy *h, const double *r, double *z)
{
    if (!h) return ORC_ERR_ARG;
    h->breakdown = 0;
    kcycle(h, 0, r, z);
    return h->breakdown ? ORC_ERR_BREAKDOWN : ORC_OK;
}

/* Outer nonlinear (flexible) preconditioned CG.  precond: 1 = K-cycle,
 * 0 = identity (then the iteration is textbook CG).  x holds the initial guess
 * on entry.  history (optional, max_iters+1 entries) receives ||r_k||/||b||. */
int orc_solve(orc_hierarchy *h, const double *b, double *x, double tol, int max_iters, int precond,
              int *iters, double *rel_res, double *solve_ms, double *history)
{
    if (!h || !b || !x || !(tol > 0.0) || max_iters < 0) return ORC_ERR_ARG;
    double t0 = now_ms();
    orc_level *F = &h->lev[0];
    int n = F->n;
    double *r = F->r, *p = F->p, *q = F->q, *z = F->z, *t = F->tmp;
    double bnorm = sqrt(dot(n, b, b));
    for (int i = 0; i < n; i++)
        if (!isfinite(b[i]) || !isfinite(x[i])) return ORC_ERR_ARG;
    h->breakdown = 0;
    *iters = 0;
    if (bnorm == 0.0) {
        for (int i = 0; i < n; i++) x[i] = 0.0;
        *rel_res = 0.0;
        if (solve_ms) *solve_ms = now_ms() - t0;
        return ORC_OK;
    }
    orc_spmv(n, F->rp, F->ci, F->va, x, t);
    for (int i = 0; i < n; i++) r[i] = b[i] - t[i];
    double rel = sqrt(dot(n, r, r)) / bnorm;
    if (history) history[0] = rel;
    int it = 0, status = ORC_ERR_NOT_CONVERGED;
    if (rel <= tol) status = ORC_OK;
    if (status != ORC_OK) {
        if (precond) kcycle(h, 0, r, z); else memcpy(z, r, sizeof(double) * (size_t)n);
        memcpy(p, z, sizeof(double) * (size_t)n);
        while (it < max_iters && !h->breakdown) {
            orc_spmv(n, F->rp, F->ci, F->va, p, q);
            double pq = dot(n, p, q);
            if (!(pq > 0.0)) { h->breakdown = 1; break; }
            double alpha = dot(n, p, r) / pq;
            for (int i = 0; i < n; i++) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            it++;
            rel = sqrt(dot(n, r, r)) / bnorm;
            if (rel <= tol) {
                /* confirm with the true residual; continue from it if it disagrees */
                orc_spmv(n, F->rp, F->ci, F->va, x, t);
                for (int i = 0; i < n; i++) r[i] = b[i] - t[i];
                rel = sqrt(dot(n, r, r)) / bnorm;
                if (history) history[it] = rel;
                if (rel <= tol) { status = ORC_OK; break; }
            } else if (history) {
                history[it] = rel;
            }
            if (precond) kcycle(h, 0, r, z); else memcpy(z, r, sizeof(double) * (size_t)n);
            if (h->breakdown) break;
            double beta = -dot(n, z, q) / pq;
            for (int i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
    }
    if (h->breakdown) status = ORC_ERR_BREAKDOWN;
    /* reported residual is always the true one */
    orc_spmv(n, F->rp, F->ci, F->va, x, t);
    double s = 0.0;
    for (int i = 0; i < n; i++) s += (b[i] - t[i]) * (b[i] - t[i]);
    *rel_res = sqrt(s) / bnorm;
    *iters = it;
    if (solve_ms) *solve_ms = now_ms() - t0;
    return status;
}

int orc_options_size(void) { return (int)sizeof(orc_options); }
