/*
 * Fast seeded generators for synthetic operands (input generation only; no
 * masked-product arithmetic lives here).
 *
 *  - Erdos-Renyi rows: every cell (i, j) is present independently with
 *    probability p. Row i is drawn by geometric skipping (the gap to the next
 *    present column is Geometric(p)), with a counter-based random stream per
 *    row (splitmix64 of seed and row), so the result does not depend on the
 *    thread count. Columns come out sorted and distinct.
 *  - Multi-source BFS lists: for each source s, the vertices at distance
 *    exactly L_s (with their shortest-path counts) and all vertices at
 *    distance <= L_s, by a level-synchronous queue BFS per source.
 *  - Transposition of per-source vertex lists into CSR with rows = vertices
 *    and columns = sources (ascending).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t splitmix64(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline double uniform01(uint64_t* st) {  /* in (0, 1] */
    return ((double)(splitmix64(st) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

/* Walks row i; calls emit for every present column. Returns the count. */
static int64_t er_row(int64_t i, int64_t n, double p, uint64_t seed, int32_t* out) {
    uint64_t st = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(i + 1));
    (void)splitmix64(&st);
    int64_t cnt = 0;
    if (n <= 0 || p <= 0.0) return 0;
    if (p >= 1.0) {
        for (int64_t j = 0; j < n; ++j) {
            if (out) out[cnt] = (int32_t)j;
            ++cnt;
        }
        return cnt;
    }
    const double lq = log1p(-p);
    int64_t j = -1;
    for (;;) {
        const double u = uniform01(&st);
        const double g = floor(log(u) / lq);  /* failures before the next success */
        if (g >= (double)(n - j - 1)) break;
        j += (int64_t)g + 1;
        if (out) out[cnt] = (int32_t)j;
        ++cnt;
    }
    return cnt;
}

/* Pass 1: row counts (rowcnt[m]). */
void gen_er_counts(int64_t m, int64_t n, double p, uint64_t seed, int64_t* rowcnt) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i) rowcnt[i] = er_row(i, n, p, seed, NULL);
}

/* Pass 2: columns into colidx at rowptr offsets (same random streams). */
void gen_er_fill(int64_t m, int64_t n, double p, uint64_t seed, const int64_t* rowptr, int32_t* colidx) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i) (void)er_row(i, n, p, seed, colidx + rowptr[i]);
}

/* Rows rows[0..nsel) only (the same random streams as the whole matrix):
   pass 1 counts, pass 2 fills colidx at the offsets off[0..nsel]. */
void gen_er_rows_counts(int64_t nsel, const int64_t* rows, int64_t n, double p, uint64_t seed, int64_t* cnt) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t x = 0; x < nsel; ++x) cnt[x] = er_row(rows[x], n, p, seed, NULL);
}

void gen_er_rows_fill(int64_t nsel, const int64_t* rows, int64_t n, double p, uint64_t seed, const int64_t* off,
                      int32_t* colidx) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t x = 0; x < nsel; ++x) (void)er_row(rows[x], n, p, seed, colidx + off[x]);
}

/* BFS from src up to depth L; fills dist (-1 = unseen) and sigma for the
   reached vertices, records them (in discovery order) in order[], and returns
   how many were reached. level_start[l] = first index in order[] of level l
   (l = 0..L+1). */
static int64_t bfs_one(const int64_t* rp, const int32_t* ci, int64_t src, int L, int8_t* dist, int64_t* sigma,
                       int64_t* order, int64_t* level_start) {
    int64_t cnt = 0;
    dist[src] = 0;
    sigma[src] = 1;
    order[cnt++] = src;
    level_start[0] = 0;
    for (int l = 0; l < L; ++l) {
        const int64_t a = level_start[l], b = cnt;
        level_start[l + 1] = cnt;
        for (int64_t x = a; x < b; ++x) {
            const int64_t u = order[x];
            for (int64_t q = rp[u]; q < rp[u + 1]; ++q) {
                const int32_t w = ci[q];
                if (dist[w] < 0) {
                    dist[w] = (int8_t)(l + 1);
                    sigma[w] = 0;
                    order[cnt++] = w;
                }
                if (dist[w] == l + 1) sigma[w] += sigma[u];
            }
        }
    }
    level_start[L + 1] = cnt;
    if (L == 0) level_start[1] = cnt;
    return cnt;
}

static void bfs_reset(int8_t* dist, const int64_t* order, int64_t cnt) {
    for (int64_t x = 0; x < cnt; ++x) dist[order[x]] = -1;
}

/* Counts: fcnt[s] = vertices at distance exactly lvl[s], vcnt[s] = at distance <= lvl[s]. */
int gen_bfs_counts(int64_t n, const int64_t* rp, const int32_t* ci, int64_t nsrc, const int64_t* src,
                   const int32_t* lvl, int64_t* fcnt, int64_t* vcnt) {
    int failed = 0;
#pragma omp parallel
    {
        int8_t* dist = (int8_t*)malloc((size_t)(n > 0 ? n : 1));
        int64_t* sigma = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t ls[128];
        const int ok = dist && sigma && order;
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        } else {
            memset(dist, -1, (size_t)n);
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsrc; ++s) {
            if (!ok) continue;
            const int L = lvl[s];
            const int64_t c = bfs_one(rp, ci, src[s], L, dist, sigma, order, ls);
            fcnt[s] = ls[L + 1] - ls[L];
            vcnt[s] = c;
            bfs_reset(dist, order, c);
        }
        free(dist); free(sigma); free(order);
    }
    return failed ? -1 : 0;
}

/* Lists: frontier vertices (ascending) with path counts at foff[s], visited
   vertices (ascending) at voff[s]. */
static int cmp_i64(const void* a, const void* b) {
    const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

int gen_bfs_lists(int64_t n, const int64_t* rp, const int32_t* ci, int64_t nsrc, const int64_t* src,
                  const int32_t* lvl, const int64_t* foff, int32_t* fverts, int64_t* fsigma, const int64_t* voff,
                  int32_t* vverts) {
    int failed = 0;
#pragma omp parallel
    {
        int8_t* dist = (int8_t*)malloc((size_t)(n > 0 ? n : 1));
        int64_t* sigma = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t ls[128];
        const int ok = dist && sigma && order;
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        } else {
            memset(dist, -1, (size_t)n);
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsrc; ++s) {
            if (!ok) continue;
            const int L = lvl[s];
            const int64_t c = bfs_one(rp, ci, src[s], L, dist, sigma, order, ls);
            /* visited: all reached, ascending */
            int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(c > 0 ? c : 1));
            memcpy(tmp, order, sizeof(int64_t) * (size_t)c);
            qsort(tmp, (size_t)c, sizeof(int64_t), cmp_i64);
            for (int64_t x = 0; x < c; ++x) vverts[voff[s] + x] = (int32_t)tmp[x];
            /* frontier: level L, ascending */
            const int64_t a = ls[L], b = ls[L + 1];
            memcpy(tmp, order + a, sizeof(int64_t) * (size_t)(b - a));
            qsort(tmp, (size_t)(b - a), sizeof(int64_t), cmp_i64);
            for (int64_t x = 0; x < b - a; ++x) {
                fverts[foff[s] + x] = (int32_t)tmp[x];
                fsigma[foff[s] + x] = sigma[tmp[x]];
            }
            free(tmp);
            bfs_reset(dist, order, c);
        }
        free(dist); free(sigma); free(order);
    }
    return failed ? -1 : 0;
}

/* Per-source vertex lists -> CSR with rows = vertices, columns = sources.
   Sources are visited in order, so every row lists its sources ascending. */
void gen_lists_to_csr(int64_t n, int64_t nsrc, const int64_t* off, const int32_t* verts, const int64_t* vals,
                      int64_t* rowptr, int32_t* colidx, int64_t* outvals) {
    memset(rowptr, 0, sizeof(int64_t) * (size_t)(n + 1));
    const int64_t total = off[nsrc];
    for (int64_t x = 0; x < total; ++x) rowptr[verts[x] + 1]++;
    for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(cur, rowptr, sizeof(int64_t) * (size_t)n);
    for (int64_t s = 0; s < nsrc; ++s) {
        for (int64_t x = off[s]; x < off[s + 1]; ++x) {
            const int64_t pos = cur[verts[x]]++;
            colidx[pos] = (int32_t)s;
            if (outvals) outvals[pos] = vals[x];
        }
    }
    free(cur);
}
