/*
 * CPU oracle for masked sparse matrix-matrix products C = M .* (A B).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU library never
 * links, includes or calls it, and it shares no code with the GPU library.
 *
 * What it computes (Section "Background and Notation"): M is m x n, A is
 * m x k, B is k x n, C is m x n. Only the pattern of M is used; M's values
 * are never read. The result is the plain definition written out:
 *
 *   1. Row-wise Gustavson product (Algorithm 1, row-parallel Gustavson
 *      SpGEMM): for every stored A(i,k), for every stored B(k,j), the product
 *      a (x) b is inserted into a sparse accumulator for row i; the first
 *      insert of column j sets the value, later inserts combine with (+).
 *      Columns are visited in stored order (ascending k, then ascending j).
 *   2. Masking: column j survives iff (j is stored in row i of M) XOR
 *      complement (Section "Classification of Algorithm Families" for the
 *      mask filter, Introduction for the complemented mask).
 *   3. Row i of C lists the surviving columns in ascending order.
 *
 * An entry of C exists iff the mask admits (i,j) and at least one k has both
 * A(i,k) and B(k,j) stored, whatever the values (the accumulator interface
 * of Section "Accumulator" returns "none" only when nothing was inserted).
 *
 * Semirings (value types in -> out):
 *   0 PLUS_TIMES_F64  double  -> double   IEEE binary64, round to nearest,
 *                                         built with -ffp-contract=off
 *   1 PLUS_PAIR_I64   ignored -> int64    (x) = 1, (+) = + mod 2^64
 *   2 LOR_LAND_BOOL   uint8   -> uint8    (x) = (a!=0)&&(b!=0), (+) = ||
 *   3 PLUS_TIMES_I32  int32   -> int32    mod 2^32 wrap-around
 *   4 PLUS_TIMES_I64  int64   -> int64    mod 2^64 wrap-around
 * A NULL value array means every stored entry holds the semiring's one.
 *
 * Parallelism: OpenMP over rows only, each thread with its own dense
 * accumulator (the coarse row parallelism of Algorithm 1). No blocking, no
 * fusion: the per-row loop is exactly the steps above.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { SR_PLUS_TIMES_F64 = 0, SR_PLUS_PAIR_I64 = 1, SR_LOR_LAND_BOOL = 2,
       SR_PLUS_TIMES_I32 = 3, SR_PLUS_TIMES_I64 = 4 };

static int out_width(int sr) {
    switch (sr) {
    case SR_PLUS_TIMES_F64: return 8;
    case SR_PLUS_PAIR_I64: return 8;
    case SR_LOR_LAND_BOOL: return 1;
    case SR_PLUS_TIMES_I32: return 4;
    case SR_PLUS_TIMES_I64: return 8;
    default: return -1;
    }
}

/* One accumulator slot holds the value as raw 8 bytes, interpreted per semiring. */
typedef union { double f; uint64_t u; } slot_t;

static slot_t load_one(int sr, const void* vals, int64_t p) {
    slot_t s; s.u = 0;
    switch (sr) {
    case SR_PLUS_TIMES_F64: s.f = vals ? ((const double*)vals)[p] : 1.0; break;
    case SR_PLUS_PAIR_I64: s.u = 1; break;
    case SR_LOR_LAND_BOOL: s.u = vals ? (((const uint8_t*)vals)[p] != 0) : 1; break;
    case SR_PLUS_TIMES_I32: s.u = vals ? (uint32_t)((const int32_t*)vals)[p] : 1u; break;
    case SR_PLUS_TIMES_I64: s.u = vals ? (uint64_t)((const int64_t*)vals)[p] : 1u; break;
    }
    return s;
}

static slot_t mul(int sr, slot_t a, slot_t b) {
    slot_t r; r.u = 0;
    switch (sr) {
    case SR_PLUS_TIMES_F64: r.f = a.f * b.f; break;
    case SR_PLUS_PAIR_I64: r.u = 1; break;
    case SR_LOR_LAND_BOOL: r.u = (a.u != 0) && (b.u != 0); break;
    case SR_PLUS_TIMES_I32: r.u = (uint32_t)((uint32_t)a.u * (uint32_t)b.u); break;
    case SR_PLUS_TIMES_I64: r.u = a.u * b.u; break;
    }
    return r;
}

static slot_t add(int sr, slot_t x, slot_t y) {
    slot_t r; r.u = 0;
    switch (sr) {
    case SR_PLUS_TIMES_F64: r.f = x.f + y.f; break;
    case SR_PLUS_PAIR_I64: r.u = x.u + y.u; break;
    case SR_LOR_LAND_BOOL: r.u = (x.u != 0) || (y.u != 0); break;
    case SR_PLUS_TIMES_I32: r.u = (uint32_t)((uint32_t)x.u + (uint32_t)y.u); break;
    case SR_PLUS_TIMES_I64: r.u = x.u + y.u; break;
    }
    return r;
}

static void store_out(int sr, void* out, int64_t p, slot_t v) {
    switch (sr) {
    case SR_PLUS_TIMES_F64: ((double*)out)[p] = v.f; break;
    case SR_PLUS_PAIR_I64: ((int64_t*)out)[p] = (int64_t)v.u; break;
    case SR_LOR_LAND_BOOL: ((uint8_t*)out)[p] = (uint8_t)(v.u != 0); break;
    case SR_PLUS_TIMES_I32: ((int32_t*)out)[p] = (int32_t)(uint32_t)v.u; break;
    case SR_PLUS_TIMES_I64: ((int64_t*)out)[p] = (int64_t)v.u; break;
    }
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

typedef struct {
    int64_t nrows;      /* number of rows computed */
    int64_t nnz;
    int64_t* rowptr;    /* [nrows+1] */
    int32_t* colidx;    /* [nnz] */
    void* values;       /* [nnz] of the output type */
    int64_t* useful;    /* [nrows] number of admitted products per row */
} oracle_result;

/*
 * Compute rows `rows[0..nsel)` of C (all rows 0..m-1 when rows == NULL).
 * Returns NULL on bad arguments or allocation failure. The caller frees the
 * result with oracle_free. Indices must be 0-based and in range; rows of M
 * may be unsorted (membership only), rows of A and B may be unsorted too:
 * the output is sorted explicitly.
 */
oracle_result* oracle_masked_spgemm(
    int64_t m, int64_t k, int64_t n,
    const int64_t* Arp, const int32_t* Aci, const void* Av,
    const int64_t* Brp, const int32_t* Bci, const void* Bv,
    const int64_t* Mrp, const int32_t* Mci,
    int complement, int semiring,
    const int64_t* rows, int64_t nsel, int nthreads)
{
    (void)k;
    int w = out_width(semiring);
    if (w < 0 || m < 0 || n < 0) return NULL;
    if (!rows) nsel = m;
    oracle_result* res = (oracle_result*)calloc(1, sizeof(oracle_result));
    if (!res) return NULL;
    res->nrows = nsel;
    int64_t* cnt = (int64_t*)calloc((size_t)nsel + 1, sizeof(int64_t));
    int32_t** rcol = (int32_t**)calloc((size_t)nsel + 1, sizeof(int32_t*));
    slot_t** rval = (slot_t**)calloc((size_t)nsel + 1, sizeof(slot_t*));
    res->useful = (int64_t*)calloc((size_t)nsel + 1, sizeof(int64_t));
    if (!cnt || !rcol || !rval || !res->useful) return NULL;
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel
    {
        /* per-thread dense accumulator over the n columns of C */
        slot_t* val = (slot_t*)malloc(sizeof(slot_t) * (size_t)(n > 0 ? n : 1));
        int64_t* stamp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t* mstamp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t* nprod = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t* kept = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int ok = val && stamp && mstamp && nprod && touched && kept;
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int64_t j = 0; j < n; ++j) { stamp[j] = -1; mstamp[j] = -1; }
        }
        {
            /* every thread reaches the work-sharing loop; a thread whose
               buffers failed to allocate skips its iterations */
#pragma omp for schedule(dynamic, 64)
            for (int64_t s = 0; s < nsel; ++s) {
                if (!ok) continue;
                int64_t i = rows ? rows[s] : s;
                int64_t nt = 0;
                /* step 1: Gustavson row i (Algorithm 1) */
                for (int64_t p = Arp[i]; p < Arp[i + 1]; ++p) {
                    int32_t kk = Aci[p];
                    slot_t a = load_one(semiring, Av, p);
                    for (int64_t q = Brp[kk]; q < Brp[kk + 1]; ++q) {
                        int32_t j = Bci[q];
                        slot_t t = mul(semiring, a, load_one(semiring, Bv, q));
                        if (stamp[j] != i) {          /* C(i,j) not yet in row: insert */
                            stamp[j] = i;
                            val[j] = t;
                            nprod[j] = 1;
                            touched[nt++] = j;
                        } else {                      /* otherwise accumulate */
                            val[j] = add(semiring, val[j], t);
                            nprod[j] += 1;
                        }
                    }
                }
                /* step 2: mask membership of row i (pattern only) */
                for (int64_t p = Mrp[i]; p < Mrp[i + 1]; ++p) mstamp[Mci[p]] = i;
                int64_t keep = 0;
                for (int64_t t = 0; t < nt; ++t) {
                    int32_t j = touched[t];
                    int in_mask = (mstamp[j] == i);
                    if (in_mask != (complement != 0)) kept[keep++] = j;
                }
                /* step 3: ascending column order */
                qsort(kept, (size_t)keep, sizeof(int32_t), cmp_i32);
                int32_t* oc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(keep > 0 ? keep : 1));
                slot_t* ov = (slot_t*)malloc(sizeof(slot_t) * (size_t)(keep > 0 ? keep : 1));
                if (!oc || !ov) {
#pragma omp atomic write
                    failed = 1;
                } else {
                    int64_t useful = 0;
                    for (int64_t t = 0; t < keep; ++t) {
                        oc[t] = kept[t];
                        ov[t] = val[kept[t]];
                        useful += nprod[kept[t]];
                    }
                    res->useful[s] = useful;
                }
                rcol[s] = oc;
                rval[s] = ov;
                cnt[s] = keep;
                /* clear this row's stamps so that a repeated row id starts clean */
                for (int64_t p = Mrp[i]; p < Mrp[i + 1]; ++p) mstamp[Mci[p]] = -1;
                for (int64_t t = 0; t < nt; ++t) stamp[touched[t]] = -1;
            }
        }
        free(val); free(stamp); free(mstamp); free(nprod); free(touched); free(kept);
    }
    if (failed) return NULL;
    /* sequential exclusive prefix sum of the row counts, then concatenation */
    res->rowptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nsel + 1));
    res->rowptr[0] = 0;
    for (int64_t s = 0; s < nsel; ++s) res->rowptr[s + 1] = res->rowptr[s] + cnt[s];
    res->nnz = res->rowptr[nsel];
    res->colidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(res->nnz > 0 ? res->nnz : 1));
    res->values = malloc((size_t)w * (size_t)(res->nnz > 0 ? res->nnz : 1));
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t base = res->rowptr[s];
        for (int64_t t = 0; t < cnt[s]; ++t) {
            res->colidx[base + t] = rcol[s][t];
            store_out(semiring, res->values, base + t, rval[s][t]);
        }
        free(rcol[s]); free(rval[s]);
    }
    free(cnt); free(rcol); free(rval);
    return res;
}

void oracle_free(oracle_result* r) {
    if (!r) return;
    free(r->rowptr); free(r->colidx); free(r->values); free(r->useful);
    free(r);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
