// Batched betweenness-centrality dependencies on top of the masked product
// (Section "Betweenness Centrality": a multi-source two-stage algorithm whose
// forward stage uses a complemented mask and whose backward stage uses a
// normal one).
//
// Orientation (as for the BFS step): frontiers are n x b matrices, rows =
// vertices, column j = source j.
//   forward, level d = 1, 2, ...:
//     F_d = !V_{d-1} .* (A F_{d-1})    over (+, x) in FP64: F_d(v, j) is the
//                                      number of shortest paths sigma from
//                                      source j to v, v at distance d
//     V_d = V_{d-1} u pattern(F_d)     (disjoint row union)
//   backward, d = D, ..., 2 (Brandes's recursion in matrix form):
//     W_d     = (1 + delta_d) ./ sigma_d        on pattern(F_d)
//     delta_{d-1} = sigma_{d-1} .* (F_{d-1} .* (A W_d))   normal mask F_{d-1}
//   bc[v] += sum over levels d >= 1 and sources j of delta_d(v, j)
// A's values are ignored (unweighted graph); A must hold a symmetric pattern.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <utility>
#include <vector>

#include "msp.h"
#include "msp_device.hpp"
#include "msp_internal.hpp"

namespace mspk {
namespace {

constexpr int BC_T = 256;

// rp[i] = number of (sorted) entry rows below i, for i in [0, n]
__global__ void k_f0_rowptr(int64_t n, const int32_t* __restrict__ rows, int64_t cnt, int64_t* __restrict__ rp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t lo = 0, hi = cnt;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rows[mid] < i) lo = mid + 1; else hi = mid;
    }
    rp[i] = lo;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_add_rowptr(int64_t n1, const int64_t* __restrict__ a, const int64_t* __restrict__ b,
                             int64_t* __restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n1) c[i] = a[i] + b[i];
}

// Union of two row-disjoint sorted CSR patterns with rpu = rpa + rpb: one
// wave per row; an entry's place is its rank in its own row plus the number
// of smaller entries of the other row.
__global__ __launch_bounds__(BC_T) void k_union_rows(int64_t n, const int64_t* __restrict__ rpa,
                                                     const int32_t* __restrict__ cia, const int64_t* __restrict__ rpb,
                                                     const int32_t* __restrict__ cib, const int64_t* __restrict__ rpu,
                                                     int32_t* __restrict__ ciu) {
    const int64_t first = (int64_t)blockIdx.x * (BC_T / WAVE) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (BC_T / WAVE)) {
        const int64_t a0 = rpa[r], a1 = rpa[r + 1], b0 = rpb[r], b1 = rpb[r + 1], u0 = rpu[r];
        for (int64_t x = lane(); x < a1 - a0; x += WAVE) {
            const int32_t c = cia[a0 + x];
            ciu[u0 + x + (lower_bound_g(cib, b0, b1, c) - b0)] = c;
        }
        for (int64_t x = lane(); x < b1 - b0; x += WAVE) {
            const int32_t c = cib[b0 + x];
            ciu[u0 + x + (lower_bound_g(cia, a0, a1, c) - a0)] = c;
        }
    }
}

// The same union for at most BC_NARROW columns (a batch of at most that many
// sources): one wave per row marks both rows' columns in a bitmap in LDS and
// emits the set bits in column order, with no search.
constexpr int BC_NARROW = 512;

__global__ __launch_bounds__(BC_T) void k_union_rows_narrow(int64_t n, const int64_t* __restrict__ rpa,
                                                            const int32_t* __restrict__ cia,
                                                            const int64_t* __restrict__ rpb,
                                                            const int32_t* __restrict__ cib,
                                                            const int64_t* __restrict__ rpu, int32_t* __restrict__ ciu) {
    __shared__ uint32_t bits_[BC_T / WAVE][BC_NARROW / 32];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    uint32_t* bits = bits_[wv];
    const int64_t first = (int64_t)blockIdx.x * (BC_T / WAVE) + wv;
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (BC_T / WAVE)) {
        const int64_t a0 = rpa[r], a1 = rpa[r + 1], b0 = rpb[r], b1 = rpb[r + 1];
        if (a0 == a1 && b0 == b1) continue;  // wave-uniform
        int64_t pos = rpu[r];
        if (lane() < BC_NARROW / 32) bits[lane()] = 0u;
        wave_lds_sync();
        for (int64_t x = a0 + lane(); x < a1; x += WAVE) atomicOr(&bits[cia[x] >> 5], 1u << (cia[x] & 31));
        for (int64_t x = b0 + lane(); x < b1; x += WAVE) atomicOr(&bits[cib[x] >> 5], 1u << (cib[x] & 31));
        wave_lds_sync();
        for (int base = 0; base < BC_NARROW; base += WAVE) {
            const int c = base + lane();
            const bool set = (bits[c >> 5] >> (c & 31)) & 1u;
            const uint64_t m = __ballot(set);
            if (set) ciu[pos + rank_below(m)] = c;
            pos += __popcll(m);
        }
        wave_lds_sync();  // the bitmap is cleared for the next row only after every lane read it
    }
}

// w = (1 + delta) / sigma, entry by entry
__global__ void k_bc_weight(int64_t nnz, const double* __restrict__ sigma, const double* __restrict__ delta,
                            double* __restrict__ w) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        w[e] = __ddiv_rn(__dadd_rn(1.0, delta[e]), sigma[e]);
}

// delta[e] = sigma[e] * C(row(e), col(e)) for every entry e of F (C's rows are
// sorted subsets of F's rows), 0 where C has no entry.
__global__ __launch_bounds__(BC_T) void k_bc_gather(int64_t n, const int64_t* __restrict__ rpf,
                                                    const int32_t* __restrict__ cif, const double* __restrict__ sigf,
                                                    const int64_t* __restrict__ rpc, const int32_t* __restrict__ cic,
                                                    const double* __restrict__ vc, double* __restrict__ delta) {
    const int64_t first = (int64_t)blockIdx.x * (BC_T / WAVE) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (BC_T / WAVE)) {
        const int64_t f0 = rpf[r], f1 = rpf[r + 1], c0 = rpc[r], c1 = rpc[r + 1];
        for (int64_t x = f0 + lane(); x < f1; x += WAVE) {
            const int32_t c = cif[x];
            const int64_t p = lower_bound_g(cic, c0, c1, c);
            delta[x] = (p < c1 && cic[p] == c) ? __dmul_rn(sigf[x], vc[p]) : 0.0;
        }
    }
}

// The same gather for at most BC_NARROW columns: one wave per row scatters
// C's row into a dense row of values and a bitmap in LDS, then reads them at
// F's columns, with no search.
__global__ __launch_bounds__(BC_T) void k_bc_gather_narrow(int64_t n, const int64_t* __restrict__ rpf,
                                                           const int32_t* __restrict__ cif,
                                                           const double* __restrict__ sigf,
                                                           const int64_t* __restrict__ rpc,
                                                           const int32_t* __restrict__ cic,
                                                           const double* __restrict__ vc, double* __restrict__ delta) {
    __shared__ uint32_t bits_[BC_T / WAVE][BC_NARROW / 32];
    __shared__ double vals_[BC_T / WAVE][BC_NARROW];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    uint32_t* bits = bits_[wv];
    double* vals = vals_[wv];
    const int64_t first = (int64_t)blockIdx.x * (BC_T / WAVE) + wv;
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (BC_T / WAVE)) {
        const int64_t f0 = rpf[r], f1 = rpf[r + 1], c0 = rpc[r], c1 = rpc[r + 1];
        if (f0 == f1) continue;  // wave-uniform
        if (lane() < BC_NARROW / 32) bits[lane()] = 0u;
        wave_lds_sync();
        for (int64_t x = c0 + lane(); x < c1; x += WAVE) {  // columns of a row are distinct: plain stores
            const int32_t c = cic[x];
            vals[c] = vc[x];
            atomicOr(&bits[c >> 5], 1u << (c & 31));
        }
        wave_lds_sync();
        for (int64_t x = f0 + lane(); x < f1; x += WAVE) {
            const int32_t c = cif[x];
            delta[x] = ((bits[c >> 5] >> (c & 31)) & 1u) ? __dmul_rn(sigf[x], vals[c]) : 0.0;
        }
        wave_lds_sync();  // the next row rewrites the bitmap and values only after every lane read them
    }
}

// bc[row] += sum of the row's delta (one wave per row, fixed order)
__global__ __launch_bounds__(BC_T) void k_bc_rowsum(int64_t n, const int64_t* __restrict__ rp,
                                                    const double* __restrict__ delta, double* __restrict__ bc) {
    const int64_t first = (int64_t)blockIdx.x * (BC_T / WAVE) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t r = first; r < n; r += (int64_t)gridDim.x * (BC_T / WAVE)) {
        double s = 0.0;
        for (int64_t x = rp[r] + lane(); x < rp[r + 1]; x += WAVE) s = __dadd_rn(s, delta[x]);
#pragma unroll
        for (int d = WAVE / 2; d >= 1; d >>= 1) s = __dadd_rn(s, __shfl_xor(s, d, WAVE));
        if (lane() == 0 && s != 0.0) bc[r] = __dadd_rn(bc[r], s);
    }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }
// wave-per-row kernels loop over rows: the grid stays far below 2^32 work-items
unsigned row_blocks(int64_t n) { return (unsigned)std::min<int64_t>(blocks_for(n, BC_T / WAVE), int64_t(1) << 20); }
unsigned grid_cap(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + 255) / 256), 65536); }

struct Level {
    int64_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* val = nullptr;  // sigma
    int64_t nnz = 0;
};

#define BC_HIP(expr)                                                                    \
    do {                                                                                \
        const hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) return set_error(MSP_ERR_DEVICE, hipGetErrorString(_e));  \
    } while (0)
#define BC_CHECK(expr)                      \
    do {                                    \
        const msp_status _st = (expr);      \
        if (_st != MSP_OK) return _st;      \
    } while (0)

// One masked FP64 product into freshly allocated arrays (rows = n); the
// plan's workspaces come from `mem` and go back to it before returning.
msp_status masked_product(const msp_csr& A, const msp_csr& B, const msp_csr& M, int complement, hipStream_t s,
                          DevMem& mem, Level& out, int64_t& products) {
    msp_options opt;
    msp_options_default(&opt);
    size_t pws_bytes = 0, xws_bytes = 0;
    BC_CHECK(msp_plan_workspace_size(&A, &B, &M, complement, MSP_PLUS_TIMES_F64, &opt, &pws_bytes));
    void* pws = nullptr;
    BC_CHECK(mem.bytes(&pws, pws_bytes));
    msp_plan* P = nullptr;
    BC_CHECK(msp_plan_create(&P, &A, &B, &M, complement, MSP_PLUS_TIMES_F64, &opt, pws, pws_bytes, s));
    msp_plan_info_t pi;
    msp_status st = msp_plan_info(P, &pi);
    void* xws = nullptr;
    if (st == MSP_OK) st = msp_workspace_size(P, &xws_bytes);
    if (st == MSP_OK) st = mem.bytes(&xws, xws_bytes);
    if (st == MSP_OK) {
        products += pi.products;
        const int64_t cap = std::max<int64_t>(pi.upper_bound, 1);
        st = mem.get(&out.rp, A.nrows + 1);
        if (st == MSP_OK) st = mem.get(&out.ci, cap);
        if (st == MSP_OK) st = mem.get(&out.val, cap);
        if (st == MSP_OK) {
            msp_csr_out C{A.nrows, B.ncols, cap, out.rp, out.ci, out.val};
            st = msp_execute(P, &C, &out.nnz, xws, xws_bytes, s);  // synchronizes: nnz is read back
        }
    }
    msp_plan_destroy(P);
    if (xws) mem.release(xws);
    mem.release(pws);
    return st;
}

}  // namespace
}  // namespace mspk

using namespace mspk;

extern "C" msp_status msp_bc_batch(const msp_csr* A, const int32_t* sources, int64_t nsrc, double* bc,
                                   msp_bc_info_t* info, const msp_allocator* alloc, void* stream) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (!A) return set_error(MSP_ERR_INVALID_ARGUMENT, "A is NULL");
    if (A->nrows != A->ncols) return set_error(MSP_ERR_DIMENSION_MISMATCH, "A must be square");
    if (nsrc < 0 || (nsrc > 0 && !sources)) return set_error(MSP_ERR_INVALID_ARGUMENT, "bad source list");
    if (nsrc > INT32_MAX) return set_error(MSP_ERR_UNSUPPORTED, "too many sources");
    if (!alloc || !alloc->alloc || !alloc->release) return set_error(MSP_ERR_INVALID_ARGUMENT, "no allocator");
    const int64_t n = A->nrows;
    if (n > 0 && !bc) return set_error(MSP_ERR_INVALID_ARGUMENT, "bc is NULL");
    for (int64_t j = 0; j < nsrc; ++j)
        if (sources[j] < 0 || (int64_t)sources[j] >= n)
            return set_error(MSP_ERR_INVALID_ARGUMENT, "source out of range");
    if (n == 0 || nsrc == 0) return MSP_OK;
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    DevMem mem(alloc, s);
    const msp_csr Aiso{A->nrows, A->ncols, A->nnz, A->rowptr, A->colidx, nullptr};

    // level 0: row src_j holds column j with sigma = 1 (entries sorted by row, then column)
    std::vector<std::pair<int32_t, int32_t>> ent((size_t)nsrc);
    for (int64_t j = 0; j < nsrc; ++j) ent[(size_t)j] = {sources[j], (int32_t)j};
    std::sort(ent.begin(), ent.end());
    std::vector<int32_t> hrows((size_t)nsrc), hcols((size_t)nsrc);
    for (int64_t j = 0; j < nsrc; ++j) {
        hrows[(size_t)j] = ent[(size_t)j].first;
        hcols[(size_t)j] = ent[(size_t)j].second;
    }
    int32_t* drows = nullptr;
    Level f0;
    BC_CHECK(mem.get(&drows, nsrc));
    BC_CHECK(mem.get(&f0.rp, n + 1));
    BC_CHECK(mem.get(&f0.ci, nsrc));
    BC_CHECK(mem.get(&f0.val, nsrc));
    f0.nnz = nsrc;
    BC_HIP(hipMemcpyAsync(drows, hrows.data(), sizeof(int32_t) * (size_t)nsrc, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(f0.ci, hcols.data(), sizeof(int32_t) * (size_t)nsrc, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_f0_rowptr, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n, drows, nsrc, f0.rp);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_cap(nsrc)), dim3(256), 0, s, f0.val, nsrc, 1.0);
    BC_HIP(hipGetLastError());
    BC_HIP(hipStreamSynchronize(s));  // the host source lists go out of scope

    // forward: frontiers F_1..F_D and the visited pattern V
    std::vector<Level> F{f0};
    int64_t* vrp = f0.rp;
    int32_t* vci = f0.ci;
    int64_t vnnz = nsrc;
    int64_t fwd_products = 0, bwd_products = 0, frontier_nnz = 0;
    for (;;) {
        const Level& prev = F.back();
        const msp_csr Bv{n, nsrc, prev.nnz, prev.rp, prev.ci, prev.val};
        const msp_csr Vv{n, nsrc, vnnz, vrp, vci, nullptr};
        Level next;
        BC_CHECK(masked_product(Aiso, Bv, Vv, 1, s, mem, next, fwd_products));
        if (next.nnz == 0) {
            mem.release(next.rp);
            mem.release(next.ci);
            mem.release(next.val);
            break;
        }
        F.push_back(next);
        frontier_nnz += next.nnz;
        int64_t* urp = nullptr;
        int32_t* uci = nullptr;
        BC_CHECK(mem.get(&urp, n + 1));
        BC_CHECK(mem.get(&uci, vnnz + next.nnz));
        hipLaunchKernelGGL(k_add_rowptr, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n + 1, vrp, next.rp, urp);
        if (nsrc <= BC_NARROW)
            hipLaunchKernelGGL(k_union_rows_narrow, dim3(row_blocks(n)), dim3(BC_T), 0, s, n, vrp, vci, next.rp,
                               next.ci, urp, uci);
        else
            hipLaunchKernelGGL(k_union_rows, dim3(row_blocks(n)), dim3(BC_T), 0, s, n, vrp, vci, next.rp,
                               next.ci, urp, uci);
        BC_HIP(hipGetLastError());
        if (vrp != f0.rp) {
            mem.release(vrp);
            mem.release(vci);
        }
        vrp = urp;
        vci = uci;
        vnnz += next.nnz;
    }
    if (vrp != f0.rp) {
        mem.release(vrp);
        mem.release(vci);
    }
    BC_HIP(hipStreamSynchronize(s));
    const auto t1 = std::chrono::steady_clock::now();

    // backward: delta per level, aligned with the level's entries
    const int64_t D = (int64_t)F.size() - 1;
    std::vector<double*> delta((size_t)D + 1, nullptr);
    for (int64_t d = 1; d <= D; ++d) BC_CHECK(mem.get(&delta[(size_t)d], F[(size_t)d].nnz));
    if (D >= 1)
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_cap(F[(size_t)D].nnz)), dim3(256), 0, s, delta[(size_t)D],
                           F[(size_t)D].nnz, 0.0);
    for (int64_t d = D; d >= 2; --d) {
        const Level& Fd = F[(size_t)d];
        const Level& Fp = F[(size_t)d - 1];
        double* w = nullptr;
        BC_CHECK(mem.get(&w, Fd.nnz));
        hipLaunchKernelGGL(k_bc_weight, dim3(grid_cap(Fd.nnz)), dim3(256), 0, s, Fd.nnz, Fd.val,
                           delta[(size_t)d], w);
        BC_HIP(hipGetLastError());
        const msp_csr Bw{n, nsrc, Fd.nnz, Fd.rp, Fd.ci, w};
        const msp_csr Mp{n, nsrc, Fp.nnz, Fp.rp, Fp.ci, nullptr};
        Level c;
        BC_CHECK(masked_product(Aiso, Bw, Mp, 0, s, mem, c, bwd_products));
        if (nsrc <= BC_NARROW)
            hipLaunchKernelGGL(k_bc_gather_narrow, dim3(row_blocks(n)), dim3(BC_T), 0, s, n, Fp.rp, Fp.ci,
                               Fp.val, c.rp, c.ci, c.val, delta[(size_t)d - 1]);
        else
            hipLaunchKernelGGL(k_bc_gather, dim3(row_blocks(n)), dim3(BC_T), 0, s, n, Fp.rp, Fp.ci,
                               Fp.val, c.rp, c.ci, c.val, delta[(size_t)d - 1]);
        hipLaunchKernelGGL(k_bc_rowsum, dim3(row_blocks(n)), dim3(BC_T), 0, s, n, Fp.rp,
                           delta[(size_t)d - 1], bc);
        BC_HIP(hipGetLastError());
        mem.release(w);
        mem.release(c.rp);
        mem.release(c.ci);
        mem.release(c.val);
        // level d is no longer needed
        mem.release(delta[(size_t)d]);
        delta[(size_t)d] = nullptr;
    }
    BC_HIP(hipStreamSynchronize(s));
    const auto t2 = std::chrono::steady_clock::now();
    if (info) {
        info->levels = D;
        info->frontier_nnz = frontier_nnz;
        info->forward_products = fwd_products;
        info->backward_products = bwd_products;
        info->forward_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->backward_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
    }
    return MSP_OK;
}
