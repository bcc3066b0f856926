/*
 * CPU oracle for batched betweenness-centrality dependencies.
 *
 * TEST INFRASTRUCTURE ONLY (see msp_oracle.c): loaded by the tests, the smoke
 * check and the benchmark's CPU-baseline leg; it shares no code with the GPU
 * library.
 *
 * What it computes (Section "Betweenness Centrality": the multi-source
 * two-stage algorithm of Brandes): for an unweighted undirected graph given
 * by a symmetric CSR pattern and a batch of sources s_1..s_b,
 *
 *   bc[v] = sum over the batch of delta_s(v), v != s,
 *   delta_s(v) = sum over successors w of v on shortest paths from s of
 *                (sigma_s(v) / sigma_s(w)) * (1 + delta_s(w)),
 *
 * where sigma_s(v) is the number of shortest s-v paths. Each source is a
 * textbook queue BFS that counts shortest paths, followed by the dependency
 * accumulation in reverse BFS order. A source listed twice contributes twice.
 * This is Brandes's vertex-by-vertex formulation, not the matrix formulation
 * the GPU path uses, so the two check each other.
 *
 * Arithmetic: IEEE binary64, built with -ffp-contract=off. Sources run in
 * parallel (OpenMP); each thread accumulates into its own array and the
 * arrays are added in thread order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_bc(int64_t n, const int64_t* rp, const int32_t* ci, int64_t nsrc, const int32_t* src, double* bc,
              int nthreads) {
    if (n < 0 || nsrc < 0) return -1;
    for (int64_t v = 0; v < n; ++v) bc[v] = 0.0;
    if (n == 0 || nsrc == 0) return 0;
    for (int64_t j = 0; j < nsrc; ++j)
        if (src[j] < 0 || src[j] >= n) return -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    double* part = (double*)calloc((size_t)nthreads * (size_t)n, sizeof(double));
    if (!part) return -1;
    int failed = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* acc = part + (size_t)tid * (size_t)n;
        int64_t* dist = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        double* sigma = (double*)malloc(sizeof(double) * (size_t)n);
        double* delta = (double*)malloc(sizeof(double) * (size_t)n);
        int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        const int ok = dist && sigma && delta && order;
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < nsrc; ++j) {
            if (!ok) continue;
            for (int64_t v = 0; v < n; ++v) {
                dist[v] = -1;
                sigma[v] = 0.0;
                delta[v] = 0.0;
            }
            const int64_t s = src[j];
            int64_t head = 0, tail = 0;
            dist[s] = 0;
            sigma[s] = 1.0;
            order[tail++] = s;
            while (head < tail) {  // BFS, counting shortest paths
                const int64_t u = order[head++];
                for (int64_t q = rp[u]; q < rp[u + 1]; ++q) {
                    const int64_t w = ci[q];
                    if (dist[w] < 0) {
                        dist[w] = dist[u] + 1;
                        order[tail++] = w;
                    }
                    if (dist[w] == dist[u] + 1) sigma[w] += sigma[u];
                }
            }
            for (int64_t x = tail - 1; x >= 0; --x) {  // dependencies in reverse BFS order
                const int64_t w = order[x];
                for (int64_t q = rp[w]; q < rp[w + 1]; ++q) {
                    const int64_t v = ci[q];
                    if (dist[v] == dist[w] - 1) delta[v] += (sigma[v] / sigma[w]) * (1.0 + delta[w]);
                }
                if (w != s) acc[w] += delta[w];
            }
        }
        free(dist);
        free(sigma);
        free(delta);
        free(order);
    }
    if (!failed)
        for (int t = 0; t < nthreads; ++t)
            for (int64_t v = 0; v < n; ++v) bc[v] += part[(size_t)t * (size_t)n + v];
    free(part);
    return failed ? -1 : 0;
}
