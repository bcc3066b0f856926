// k-truss by iterated masked products (Section "Experimental Setup": edges
// supported by at least k-2 triangles, found by repeated masked products
// while pruning changes the graph).
//
//   C = A
//   repeat: S = C .* (C C) over plus-pair (S(i,j) = triangles through edge
//           (i,j) inside C; an edge in no triangle has no entry in S)
//           C' = the entries of S with S(i,j) >= k-2
//   until nnz(C') == nnz(C)
//
// Pruning only removes edges, so equal counts mean C' == C. The output holds
// the k-truss with each edge's support (its triangle count in the truss).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "msp.h"
#include "msp_device.hpp"
#include "msp_internal.hpp"

namespace mspk {
namespace {

constexpr int KT_T = 256;

// cnt[r] = entries of row r with value >= thresh (one wave per row)
__global__ __launch_bounds__(KT_T) void k_prune_count(int64_t n, const int64_t* __restrict__ rp,
                                                      const int64_t* __restrict__ v, int64_t thresh,
                                                      int64_t* __restrict__ cnt) {
    const int64_t first = (int64_t)blockIdx.x * (KT_T / WAVE) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (KT_T / WAVE)) {
        int64_t c = 0;
        for (int64_t x = rp[r] + lane(); x < rp[r + 1]; x += WAVE) c += v[x] >= thresh ? 1 : 0;
        c = wave_sum(c);
        if (lane() == 0) cnt[r] = c;
    }
}

// copies the kept entries of every row, in order, to out_rp[r]
__global__ __launch_bounds__(KT_T) void k_prune_copy(int64_t n, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const int64_t* __restrict__ v,
                                                     int64_t thresh, const int64_t* __restrict__ out_rp,
                                                     int32_t* __restrict__ out_ci, int64_t* __restrict__ out_v) {
    const int64_t first = (int64_t)blockIdx.x * (KT_T / WAVE) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (KT_T / WAVE)) {
        int64_t pos = out_rp[r];
        for (int64_t base = rp[r]; base < rp[r + 1]; base += WAVE) {
            const int64_t x = base + lane();
            const bool keep = x < rp[r + 1] && v[x] >= thresh;
            const uint64_t m = __ballot(keep);
            if (keep) {
                out_ci[pos + rank_below(m)] = ci[x];
                out_v[pos + rank_below(m)] = v[x];
            }
            pos += __popcll(m);
        }
    }
}

// rows are looped over, so the grid is capped (far below 2^32 work-items)
unsigned kt_blocks(int64_t n, int per) {
    return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + per - 1) / per), int64_t(1) << 20);
}

#define KT_HIP(expr)                                                                    \
    do {                                                                                \
        const hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) return set_error(MSP_ERR_DEVICE, hipGetErrorString(_e));  \
    } while (0)
#define KT_CHECK(expr)                      \
    do {                                    \
        const msp_status _st = (expr);      \
        if (_st != MSP_OK) return _st;      \
    } while (0)

}  // namespace
}  // namespace mspk

using namespace mspk;

extern "C" msp_status msp_ktruss(const msp_csr* A, int32_t k, int64_t* C_rowptr, int32_t* C_colidx,
                                 int64_t* C_support, int64_t* nnz_host, msp_ktruss_info_t* info,
                                 const msp_allocator* alloc, void* stream) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (!A || !nnz_host) return set_error(MSP_ERR_INVALID_ARGUMENT, "A and nnz_host must not be NULL");
    if (A->nrows != A->ncols) return set_error(MSP_ERR_DIMENSION_MISMATCH, "A must be square");
    if (A->nrows < 0 || A->nnz < 0) return set_error(MSP_ERR_INVALID_ARGUMENT, "negative size");
    const int64_t n = A->nrows;
    if (!C_rowptr || (A->nnz > 0 && (!C_colidx || !C_support)))
        return set_error(MSP_ERR_INVALID_ARGUMENT, "output arrays must not be NULL");
    if (!alloc || !alloc->alloc || !alloc->release) return set_error(MSP_ERR_INVALID_ARGUMENT, "no allocator");
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t thresh = (int64_t)k - 2;
    DevMem mem(alloc, s);
    // current graph (pattern): starts as A
    const int64_t* rp = A->rowptr;
    const int32_t* ci = A->colidx;
    int64_t nnz = A->nnz;
    int64_t iters = 0, products = 0;
    const int64_t* sup = nullptr;  // support of the current graph's edges (after the first iteration)
    if (k <= 2 || n == 0 || nnz == 0) {
        // every edge qualifies (support >= 0): the graph itself, support not computed (0)
        KT_HIP(hipMemcpyAsync(C_rowptr, A->rowptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
        if (nnz > 0) {
            KT_HIP(hipMemcpyAsync(C_colidx, A->colidx, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            KT_HIP(hipMemsetAsync(C_support, 0, sizeof(int64_t) * (size_t)nnz, s));
        }
        KT_HIP(hipStreamSynchronize(s));
        *nnz_host = nnz;
        return MSP_OK;
    }
    int64_t* scan_part = nullptr;
    int64_t* cnt = nullptr;
    KT_CHECK(mem.get(&scan_part, scan_partial_elems(n)));
    KT_CHECK(mem.get(&cnt, n));
    for (;;) {
        // S = C .* (C C), plus-pair
        const msp_csr Cv{n, n, nnz, rp, ci, nullptr};
        msp_plan* P = nullptr;
        msp_options opt;
        msp_options_default(&opt);
        size_t pws_bytes = 0, xws_bytes = 0;
        KT_CHECK(msp_plan_workspace_size(&Cv, &Cv, &Cv, 0, MSP_PLUS_PAIR_I64, &opt, &pws_bytes));
        void *pws = nullptr, *xws = nullptr;
        KT_CHECK(mem.bytes(&pws, pws_bytes));
        KT_CHECK(msp_plan_create(&P, &Cv, &Cv, &Cv, 0, MSP_PLUS_PAIR_I64, &opt, pws, pws_bytes, s));
        msp_plan_info_t pi;
        msp_status st = msp_plan_info(P, &pi);
        int64_t *srp = nullptr, *sv = nullptr;
        int32_t* sci = nullptr;
        int64_t snnz = 0;
        if (st == MSP_OK) st = msp_workspace_size(P, &xws_bytes);
        if (st == MSP_OK) st = mem.bytes(&xws, xws_bytes);
        if (st == MSP_OK) {
            products += pi.products;
            const int64_t cap = std::max<int64_t>(pi.upper_bound, 1);
            st = mem.get(&srp, n + 1);
            if (st == MSP_OK) st = mem.get(&sci, cap);
            if (st == MSP_OK) st = mem.get(&sv, cap);
            if (st == MSP_OK) {
                msp_csr_out So{n, n, cap, srp, sci, sv};
                st = msp_execute(P, &So, &snnz, xws, xws_bytes, s);  // synchronizes: nnz is read back
            }
        }
        msp_plan_destroy(P);
        if (xws) mem.release(xws);
        mem.release(pws);
        if (st != MSP_OK) return st;
        ++iters;
        // keep the entries with support >= k - 2
        hipLaunchKernelGGL(k_prune_count, dim3(kt_blocks(n, KT_T / WAVE)), dim3(KT_T), 0, s, n, srp, sv, thresh,
                           cnt);
        KT_HIP(hipGetLastError());
        int64_t* nrp = nullptr;
        KT_CHECK(mem.get(&nrp, n + 1));
        KT_HIP(launch_scan(cnt, nrp, n, scan_part, s));  // exclusive scan, nrp[n] = total
        int64_t nn = 0;
        KT_HIP(hipMemcpyAsync(&nn, nrp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        KT_HIP(hipStreamSynchronize(s));
        int32_t* nci = nullptr;
        int64_t* nv = nullptr;
        KT_CHECK(mem.get(&nci, nn));
        KT_CHECK(mem.get(&nv, nn));
        hipLaunchKernelGGL(k_prune_copy, dim3(kt_blocks(n, KT_T / WAVE)), dim3(KT_T), 0, s, n, srp, sci, sv, thresh,
                           nrp, nci, nv);
        KT_HIP(hipGetLastError());
        const bool done = nn == nnz;
        // the previous graph and the support product are no longer needed (stream order)
        if (rp != A->rowptr) {
            mem.release(rp);
            mem.release(ci);
            mem.release(sup);
        }
        mem.release(srp);
        mem.release(sci);
        mem.release(sv);
        rp = nrp;
        ci = nci;
        sup = nv;
        nnz = nn;
        if (done || nn == 0) break;
    }
    KT_HIP(hipMemcpyAsync(C_rowptr, rp, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz > 0) {
        KT_HIP(hipMemcpyAsync(C_colidx, ci, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
        KT_HIP(hipMemcpyAsync(C_support, sup, sizeof(int64_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    }
    KT_HIP(hipStreamSynchronize(s));
    *nnz_host = nnz;
    if (info) {
        info->iterations = iters;
        info->products = products;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return MSP_OK;
}
