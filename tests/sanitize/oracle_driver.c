/*
 * Sanitizer run of the CPU oracle (built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py): masked products
 * of small seeded random CSR operands, every semiring, both mask modes,
 * whole-matrix and row-subset calls, empty shapes, plus the betweenness
 * oracle on a small graph. Each result is also checked against a dense
 * brute force written here (pattern exactly, values exactly for the integer
 * semirings and within 1e-12 relative for FP64). Exit status 0 = all good;
 * a sanitizer finding aborts the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t nrows, nnz;
    int64_t* rowptr;
    int32_t* colidx;
    void* values;
    int64_t* useful;
} result_t;

result_t* oracle_masked_spgemm(int64_t m, int64_t k, int64_t n, const int64_t* Arp, const int32_t* Aci,
                               const void* Av, const int64_t* Brp, const int32_t* Bci, const void* Bv,
                               const int64_t* Mrp, const int32_t* Mci, int complement, int semiring,
                               const int64_t* rows, int64_t nsel, int nthreads);
void oracle_free(result_t* r);
int oracle_bc(int64_t n, const int64_t* rp, const int32_t* ci, int64_t nsrc, const int32_t* src, double* bc,
              int nthreads);

static uint64_t rng_state = 0x12345678u;
static uint64_t next_u64(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

typedef struct {
    int64_t nrows, ncols;
    int64_t* rp;
    int32_t* ci;
    double* vf;
    int32_t* vi;
    int64_t* vl;
    uint8_t* vb;
    unsigned char* dense; /* nrows x ncols presence */
} mat_t;

/* every cell present with probability pct/100; values: small integers, U(0,1) doubles, 0/1 bytes */
static mat_t make(int64_t r, int64_t c, int pct) {
    mat_t M;
    M.nrows = r;
    M.ncols = c;
    M.dense = calloc((size_t)(r * c + 1), 1);
    M.rp = calloc((size_t)r + 1, sizeof(int64_t));
    int64_t nnz = 0;
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < c; ++j)
            if ((int)(next_u64() % 100) < pct) { M.dense[i * c + j] = 1; ++nnz; }
    M.ci = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    M.vf = malloc(sizeof(double) * (size_t)(nnz + 1));
    M.vi = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    M.vl = malloc(sizeof(int64_t) * (size_t)(nnz + 1));
    M.vb = malloc((size_t)(nnz + 1));
    int64_t p = 0;
    for (int64_t i = 0; i < r; ++i) {
        for (int64_t j = 0; j < c; ++j)
            if (M.dense[i * c + j]) {
                M.ci[p] = (int32_t)j;
                M.vf[p] = (double)(next_u64() % 1000) / 1000.0;
                M.vi[p] = (int32_t)(next_u64() % 7) - 2;
                M.vl[p] = (int64_t)(next_u64() % 7) - 2;
                M.vb[p] = (uint8_t)(next_u64() % 4 != 0);
                ++p;
            }
        M.rp[i + 1] = p;
    }
    return M;
}

static void drop(mat_t* M) {
    free(M->dense); free(M->rp); free(M->ci); free(M->vf); free(M->vi); free(M->vl); free(M->vb);
}

static const void* vals(const mat_t* M, int sr) {
    switch (sr) {
    case 0: return M->vf;
    case 2: return M->vb;
    case 3: return M->vi;
    case 4: return M->vl;
    default: return NULL;
    }
}

/* value of stored entry (i, j) of M in semiring sr as a double or an integer */
static int find(const mat_t* M, int64_t i, int64_t j) {
    for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p)
        if (M->ci[p] == j) return (int)p;
    return -1;
}

static int check(const mat_t* A, const mat_t* B, const mat_t* M, int comp, int sr, const int64_t* rows,
                 int64_t nsel) {
    result_t* R = oracle_masked_spgemm(A->nrows, A->ncols, B->ncols, A->rp, A->ci, vals(A, sr), B->rp, B->ci,
                                       vals(B, sr), M->rp, M->ci, comp, sr, rows, nsel, 2);
    if (!R) return 1;
    const int64_t n = B->ncols, cnt = rows ? nsel : A->nrows;
    int bad = 0;
    for (int64_t x = 0; x < cnt && !bad; ++x) {
        const int64_t i = rows ? rows[x] : x;
        int64_t q = R->rowptr[x];
        for (int64_t j = 0; j < n; ++j) {
            int exists = 0;
            double sf = 0;
            uint64_t su = 0;
            for (int64_t kk = 0; kk < A->ncols; ++kk) {
                const int pa = find(A, i, kk), pb = pa >= 0 ? find(B, kk, j) : -1;
                if (pa < 0 || pb < 0) continue;
                exists = 1;
                switch (sr) {
                case 0: sf += A->vf[pa] * B->vf[pb]; break;
                case 1: su += 1; break;
                case 2: su = su || (A->vb[pa] && B->vb[pb]); break;
                case 3: su = (uint32_t)((uint32_t)su + (uint32_t)A->vi[pa] * (uint32_t)B->vi[pb]); break;
                case 4: su += (uint64_t)A->vl[pa] * (uint64_t)B->vl[pb]; break;
                }
            }
            const int admitted = (M->dense[i * n + j] != 0) != (comp != 0);
            if (!(exists && admitted)) continue;
            if (q >= R->rowptr[x + 1] || R->colidx[q] != j) { bad = 1; break; }
            switch (sr) {
            case 0: {
                const double g = ((double*)R->values)[q];
                if (fabs(g - sf) > 1e-12 * fabs(sf)) bad = 1;
                break;
            }
            case 1: case 4: if ((uint64_t)((int64_t*)R->values)[q] != su) bad = 1; break;
            case 2: if (((uint8_t*)R->values)[q] != (uint8_t)su) bad = 1; break;
            case 3: if ((uint32_t)((int32_t*)R->values)[q] != (uint32_t)su) bad = 1; break;
            }
            ++q;
        }
        if (q != R->rowptr[x + 1]) bad = 1;
    }
    oracle_free(R);
    return bad;
}

int main(void) {
    int failures = 0;
    const int shapes[][6] = {{9, 7, 11, 30, 30, 40}, {1, 5, 5, 60, 60, 60}, {12, 1, 9, 50, 80, 50},
                             {6, 6, 6, 0, 50, 50}, {10, 8, 13, 45, 45, 0}, {15, 15, 15, 20, 20, 100}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s) {
        const int* d = shapes[s];
        mat_t A = make(d[0], d[1], d[3]), B = make(d[1], d[2], d[4]), M = make(d[0], d[2], d[5]);
        int64_t rows[4] = {d[0] - 1, 0, d[0] / 2, 0};
        for (int sr = 0; sr < 5; ++sr)
            for (int comp = 0; comp < 2; ++comp) {
                failures += check(&A, &B, &M, comp, sr, NULL, 0);
                failures += check(&A, &B, &M, comp, sr, rows, 4);
            }
        drop(&A); drop(&B); drop(&M);
    }
    {   /* empty shapes */
        mat_t A = make(0, 4, 50), B = make(4, 3, 50), M = make(0, 3, 50);
        failures += check(&A, &B, &M, 0, 0, NULL, 0);
        drop(&A); drop(&B); drop(&M);
        mat_t A2 = make(3, 0, 50), B2 = make(0, 3, 50), M2 = make(3, 3, 50);
        failures += check(&A2, &B2, &M2, 1, 1, NULL, 0);
        drop(&A2); drop(&B2); drop(&M2);
    }
    {   /* betweenness: a path 0-1-2-3 and a star, both sources' dependencies are finite */
        const int64_t rp[] = {0, 1, 3, 5, 6};
        const int32_t ci[] = {1, 0, 2, 1, 3, 2};
        const int32_t src[] = {0, 3, 1};
        double bc[4];
        if (oracle_bc(4, rp, ci, 3, src, bc, 2) != 0) ++failures;
        /* path 0-1-2-3: from 0, delta(1) = 2, delta(2) = 1; from 3 the mirror; from 1, delta(2) = 1 */
        if (fabs(bc[1] - 3.0) > 1e-12 || fabs(bc[2] - 4.0) > 1e-12 || bc[0] != 0.0 || bc[3] != 0.0) ++failures;
    }
    if (failures) fprintf(stderr, "%d oracle checks failed\n", failures);
    else printf("oracle sanitizer run: ok\n");
    return failures != 0;
}
