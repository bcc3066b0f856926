// Host runtime of the C-ABI (include/msp.h): argument checks, plan
// workspace, kernel sequencing for the one-phase and two-phase paths
// (Section "Symbolic and Numeric Phases").
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "msp.h"
#include "msp_internal.hpp"

using namespace mspk;

namespace {

thread_local std::string g_last_error;

msp_status fail(msp_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

msp_status from_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return MSP_OK;
    return fail(e == hipErrorOutOfMemory ? MSP_ERR_OUT_OF_MEMORY : MSP_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define MSP_HIP(expr)                                              \
    do {                                                           \
        const msp_status _st = from_hip((expr), #expr);            \
        if (_st != MSP_OK) return _st;                             \
    } while (0)

#define MSP_CHECK(expr)                         \
    do {                                        \
        const msp_status _st = (expr);          \
        if (_st != MSP_OK) return _st;          \
    } while (0)

// Stream-ordered allocations come from the device's default memory pool with
// an unlimited release threshold, so a plan created per call reuses memory
// released by the previous one without returning it to the driver.
std::once_flag g_pool_once[64];

void configure_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::call_once(g_pool_once[dev], [dev] {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t threshold = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
        }
    });
}

bool valid_sr(int s) { return s >= MSP_PLUS_TIMES_F64 && s <= MSP_PLUS_TIMES_I64; }

msp_status check_csr(const msp_csr* X, const char* name) {
    if (!X) return fail(MSP_ERR_INVALID_ARGUMENT, std::string(name) + " is NULL");
    if (X->nrows < 0 || X->ncols < 0 || X->nnz < 0)
        return fail(MSP_ERR_INVALID_ARGUMENT, std::string(name) + ": negative size");
    if (X->nrows >= INT32_MAX || X->ncols >= INT32_MAX)
        return fail(MSP_ERR_UNSUPPORTED, std::string(name) + ": dimension exceeds int32 column indices");
    if (!X->rowptr) return fail(MSP_ERR_INVALID_ARGUMENT, std::string(name) + ": rowptr is NULL");
    if (X->nnz > 0 && !X->colidx) return fail(MSP_ERR_INVALID_ARGUMENT, std::string(name) + ": colidx is NULL");
    return MSP_OK;
}

}  // namespace

struct msp_plan {
    hipStream_t stream = nullptr;
    Operands op{};
    int sr = 0;
    msp_options opt{};
    int64_t nnzB = 0;
    std::vector<void*> allocs;
    bool pooled = true;
    // analysis
    int64_t* flops = nullptr;
    int64_t* unit_base = nullptr;
    int8_t* bin = nullptr;
    unsigned long long* stats_d = nullptr;
    unsigned long long stats[ST_COUNT] = {};
    int64_t U = 0, S = 0, ub = 0;
    int64_t bin_count[NBINS] = {};
    int64_t bin_off[NBINS + 1] = {};
    // units
    int64_t* seg_off_d = nullptr;
    unsigned long long* seg_cursor = nullptr;
    int64_t seg_off[NBINS * NBUCKET] = {};
    int32_t* unit_row = nullptr;
    int32_t* unit_tile = nullptr;
    int64_t* stg_off = nullptr;
    int64_t* cnt = nullptr;
    int32_t* bin_units = nullptr;
    int32_t* stg_col = nullptr;
    void* stg_val = nullptr;
    int64_t* scan_partial = nullptr;
    // B^T
    int64_t* BTrp = nullptr;
    int32_t* BTci = nullptr;
    void* BTv = nullptr;
    bool symbolic_done = false;

    msp_status alloc(void** p, size_t bytes) {
        if (bytes < 256) bytes = 256;
        hipError_t e = hipErrorNotSupported;
        if (pooled) {
            e = hipMallocAsync(p, bytes, stream);
            if (e == hipErrorNotSupported) pooled = false;
        }
        if (!pooled) e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            return from_hip(e, "device allocation");
        }
        allocs.push_back(*p);
        return MSP_OK;
    }
    template <class T>
    msp_status alloc_n(T** p, int64_t n) {
        return alloc(reinterpret_cast<void**>(p), (size_t)(n > 0 ? n : 1) * sizeof(T));
    }
    // Carves several arrays out of one allocation (256-byte aligned pieces).
    struct Carve {
        std::vector<std::pair<void**, size_t>> parts;
        template <class T>
        void add(T** p, int64_t n) {
            parts.push_back({reinterpret_cast<void**>(p), (size_t)(n > 0 ? n : 1) * sizeof(T)});
        }
        void add_bytes(void** p, size_t bytes) { parts.push_back({p, bytes > 0 ? bytes : 1}); }
    };
    msp_status alloc_carve(Carve& c) {
        size_t total = 0;
        for (auto& pt : c.parts) total += (pt.second + 255) & ~(size_t)255;
        char* base = nullptr;
        MSP_CHECK(alloc(reinterpret_cast<void**>(&base), total));
        size_t off = 0;
        for (auto& pt : c.parts) {
            *pt.first = base + off;
            off += (pt.second + 255) & ~(size_t)255;
        }
        return MSP_OK;
    }
    void release() {
        for (void* p : allocs) {
            if (pooled) (void)hipFreeAsync(p, stream);
            else (void)hipFree(p);
        }
        allocs.clear();
    }
};

extern "C" {

void msp_options_default(msp_options* opt) {
    if (!opt) return;
    opt->phase = 1;
    opt->force_kind = MSP_KIND_AUTO;
    opt->validate = 0;
    opt->inner_ratio = 0;
    opt->b_transpose = nullptr;
}

const char* msp_status_string(msp_status s) {
    switch (s) {
    case MSP_OK: return "ok";
    case MSP_ERR_INVALID_ARGUMENT: return "invalid argument";
    case MSP_ERR_DIMENSION_MISMATCH: return "dimension mismatch";
    case MSP_ERR_INVALID_CSR: return "invalid CSR";
    case MSP_ERR_UNSUPPORTED: return "unsupported";
    case MSP_ERR_INSUFFICIENT_CAPACITY: return "insufficient output capacity";
    case MSP_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MSP_ERR_DEVICE: return "device error";
    default: return "unknown status";
    }
}

const char* msp_last_error(void) { return g_last_error.c_str(); }

int msp_version(void) { return 100; }

static msp_status build_transpose(msp_plan* P, bool scatter) {
    const Operands& o = P->op;
    hipStream_t s = P->stream;
    if (!P->BTrp) {
        MSP_CHECK(P->alloc_n(&P->BTrp, o.n + 1));
        MSP_HIP(launch_fill_i64(P->BTrp, o.n + 1, 0, s));
        MSP_HIP(launch_colcount(o.Bci, P->nnzB, P->BTrp, s));
        int64_t* part = nullptr;
        MSP_CHECK(P->alloc_n(&part, scan_partial_elems(o.n)));
        MSP_HIP(launch_scan(P->BTrp, P->BTrp, o.n, part, s));
        P->op.BTrp = P->BTrp;
    }
    if (scatter && !P->BTci) {
        const int vb = in_bytes(P->sr);
        MSP_CHECK(P->alloc_n(&P->BTci, P->nnzB));
        if (vb && o.Bv) MSP_CHECK(P->alloc(&P->BTv, (size_t)(P->nnzB > 0 ? P->nnzB : 1) * vb));
        unsigned long long* cursor = nullptr;
        MSP_CHECK(P->alloc_n(&cursor, o.n));
        MSP_HIP(launch_fill_i64(reinterpret_cast<int64_t*>(cursor), o.n, 0, s));
        MSP_HIP(launch_transpose_scatter(o.Brp, o.Bci, o.Bv, vb, o.k, P->BTrp, cursor, P->BTci, P->BTv, s));
        P->op.BTci = P->BTci;
        P->op.BTv = P->BTv;
    }
    return MSP_OK;
}

static msp_status plan_create_impl(msp_plan* P, const msp_csr* A, const msp_csr* B, const msp_csr* M,
                                   int complement, msp_semiring semiring, const msp_options* opt,
                                   hipStream_t stream, bool want_staging) {
    MSP_CHECK(check_csr(A, "A"));
    MSP_CHECK(check_csr(B, "B"));
    MSP_CHECK(check_csr(M, "M"));
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    if (complement != 0 && complement != 1) return fail(MSP_ERR_INVALID_ARGUMENT, "complement must be 0 or 1");
    if (A->ncols != B->nrows || M->nrows != A->nrows || M->ncols != B->ncols)
        return fail(MSP_ERR_DIMENSION_MISMATCH, "need A.ncols == B.nrows, M.nrows == A.nrows, M.ncols == B.ncols");
    msp_options o;
    msp_options_default(&o);
    if (opt) o = *opt;
    if (o.phase == 0) o.phase = 1;
    if (o.phase != 1 && o.phase != 2) return fail(MSP_ERR_INVALID_ARGUMENT, "phase must be 1 or 2");
    if (o.force_kind < MSP_KIND_AUTO || o.force_kind > MSP_KIND_INNER)
        return fail(MSP_ERR_INVALID_ARGUMENT, "unknown force_kind");
    if (o.inner_ratio < 0) return fail(MSP_ERR_INVALID_ARGUMENT, "inner_ratio must be >= 0");
    if (complement && o.force_kind != MSP_KIND_AUTO && o.force_kind != MSP_KIND_DENSE)
        return fail(MSP_ERR_UNSUPPORTED, "a complemented mask supports only the dense kind");
    if (o.b_transpose) {
        MSP_CHECK(check_csr(o.b_transpose, "B^T"));
        if (o.b_transpose->nrows != B->ncols || o.b_transpose->ncols != B->nrows ||
            o.b_transpose->nnz != B->nnz)
            return fail(MSP_ERR_DIMENSION_MISMATCH, "B^T must be B.ncols x B.nrows with nnz(B) entries");
    }
    configure_pool();
    P->stream = stream;
    P->sr = semiring;
    P->opt = o;
    P->nnzB = B->nnz;
    Operands& op = P->op;
    op.m = A->nrows; op.k = A->ncols; op.n = B->ncols;
    op.Arp = A->rowptr; op.Aci = A->colidx; op.Av = A->values;
    op.Brp = B->rowptr; op.Bci = B->colidx; op.Bv = B->values;
    op.Mrp = M->rowptr; op.Mci = M->colidx;
    op.complement = complement;
    const int64_t m = op.m;
    hipStream_t s = stream;

    // workspace sized by the operand shapes
    {
        msp_plan::Carve c;
        c.add(&P->stats_d, ST_COUNT);
        c.add(&P->flops, m);
        c.add(&P->unit_base, m + 1);
        c.add(&P->bin, m);
        c.add(&P->scan_partial, scan_partial_elems(m + 1));
        MSP_CHECK(P->alloc_carve(c));
    }
    MSP_HIP(hipMemsetAsync(P->stats_d, 0, sizeof(unsigned long long) * ST_COUNT, s));
    if (o.validate) {
        unsigned long long* err = P->stats_d + ST_ERROR;
        MSP_HIP(launch_validate(A->rowptr, A->colidx, A->nrows, A->ncols, A->nnz, err, s));
        MSP_HIP(launch_validate(B->rowptr, B->colidx, B->nrows, B->ncols, B->nnz, err, s));
        MSP_HIP(launch_validate(M->rowptr, M->colidx, M->nrows, M->ncols, M->nnz, err, s));
        if (o.b_transpose)
            MSP_HIP(launch_validate(o.b_transpose->rowptr, o.b_transpose->colidx, o.b_transpose->nrows,
                                    o.b_transpose->ncols, o.b_transpose->nnz, err, s));
        // validation must finish before the analysis trusts the row pointers
        unsigned long long e = 0;
        MSP_HIP(hipMemcpyAsync(&e, err, sizeof(e), hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
        if (e) return fail(MSP_ERR_INVALID_CSR, "an operand violates the CSR invariants");
    }
    const bool inner_possible = !complement && (o.force_kind == MSP_KIND_INNER ||
                                                (o.force_kind == MSP_KIND_AUTO && o.inner_ratio > 0));
    if (o.b_transpose) {
        op.BTrp = o.b_transpose->rowptr;
        op.BTci = o.b_transpose->colidx;
        op.BTv = o.b_transpose->values;
    } else if (inner_possible) {
        MSP_CHECK(build_transpose(P, o.force_kind == MSP_KIND_INNER));
    }

    AnalysisArgs aa{};
    aa.op = op;
    aa.force_kind = o.force_kind;
    aa.inner_ratio = inner_possible ? o.inner_ratio : 0;
    aa.colcnt_rp = op.BTrp;
    aa.flops = P->flops;
    aa.tiles = P->unit_base;
    aa.bin = P->bin;
    aa.stats = P->stats_d;
    MSP_HIP(launch_analysis(aa, s));
    MSP_HIP(launch_scan(P->unit_base, P->unit_base, m, P->scan_partial, s));
    MSP_HIP(hipMemcpyAsync(P->stats, P->stats_d, sizeof(P->stats), hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    P->U = (int64_t)P->stats[ST_UNITS];
    P->S = (int64_t)P->stats[ST_STAGING];
    P->ub = (int64_t)P->stats[ST_UB];
    // bins in order; inside a bin, flops buckets from the heaviest down
    P->bin_off[0] = 0;
    int64_t run = 0;
    for (int b = 0; b < NBINS; ++b) {
        P->bin_off[b] = run;
        for (int q = NBUCKET - 1; q >= 0; --q) {
            P->seg_off[b * NBUCKET + q] = run;
            run += (int64_t)P->stats[ST_BIN0 + b * NBUCKET + q];
        }
        P->bin_count[b] = run - P->bin_off[b];
    }
    P->bin_off[NBINS] = run;
    if (P->bin_off[NBINS] != P->U) return fail(MSP_ERR_DEVICE, "inconsistent unit statistics");
    if (P->U >= INT32_MAX) return fail(MSP_ERR_UNSUPPORTED, "too many work units");
    if (P->bin_count[BIN_INNER_W] > 0 && !o.b_transpose) MSP_CHECK(build_transpose(P, true));

    const int64_t U = P->U;
    // workspace sized by the units (and the one-phase staging)
    {
        msp_plan::Carve c;
        c.add(&P->seg_off_d, NBINS * NBUCKET);
        c.add(&P->seg_cursor, NBINS * NBUCKET);
        c.add(&P->unit_row, U);
        c.add(&P->unit_tile, U);
        c.add(&P->stg_off, U + 1);
        c.add(&P->cnt, U + 1);
        c.add(&P->bin_units, U);
        int64_t* part = nullptr;
        if (U + 1 > m + 1) c.add(&part, scan_partial_elems(U + 1));
        if (want_staging && o.phase == 1) {
            c.add(&P->stg_col, P->S);
            c.add_bytes(&P->stg_val, (size_t)(P->S > 0 ? P->S : 1) * out_bytes(semiring));
        }
        MSP_CHECK(P->alloc_carve(c));
        if (part) P->scan_partial = part;
    }
    MSP_HIP(hipMemcpyAsync(P->seg_off_d, P->seg_off, sizeof(int64_t) * NBINS * NBUCKET, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemsetAsync(P->seg_cursor, 0, sizeof(unsigned long long) * NBINS * NBUCKET, s));
    UnitArgs ua{};
    ua.op = op;
    ua.flops = P->flops;
    ua.unit_base = P->unit_base;
    ua.bin = P->bin;
    ua.seg_off = P->seg_off_d;
    ua.seg_cursor = P->seg_cursor;
    ua.unit_row = P->unit_row;
    ua.unit_tile = P->unit_tile;
    ua.stg_size = P->stg_off;
    ua.bin_units = P->bin_units;
    MSP_HIP(launch_units(ua, m, s));
    if (want_staging && o.phase == 1) MSP_HIP(launch_scan(P->stg_off, P->stg_off, U, P->scan_partial, s));
    return MSP_OK;
}

msp_status msp_plan_create(msp_plan** plan, const msp_csr* A, const msp_csr* B, const msp_csr* M,
                           int complement, msp_semiring semiring, const msp_options* opt, void* stream) {
    if (!plan) return fail(MSP_ERR_INVALID_ARGUMENT, "plan is NULL");
    *plan = nullptr;
    msp_plan* P = new (std::nothrow) msp_plan();
    if (!P) return fail(MSP_ERR_OUT_OF_MEMORY, "host allocation");
    const msp_status st = plan_create_impl(P, A, B, M, complement, semiring, opt, (hipStream_t)stream, true);
    if (st != MSP_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        P->release();
        delete P;
        return st;
    }
    *plan = P;
    return MSP_OK;
}

msp_status msp_plan_info(const msp_plan* P, msp_plan_info_t* info) {
    if (!P || !info) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    info->upper_bound = P->ub;
    info->products = (int64_t)P->stats[ST_FLOPS];
    info->units = P->U;
    info->staging = P->S;
    info->mask_nnz = (int64_t)P->stats[ST_MNNZ];
    info->kind_units[MSP_KIND_DENSE] = P->bin_count[BIN_DENSE_W] + P->bin_count[BIN_DENSE_B];
    info->kind_units[MSP_KIND_HASH] = P->bin_count[BIN_HASH_W] + P->bin_count[BIN_HASH_B];
    info->kind_units[MSP_KIND_MASKIDX] = P->bin_count[BIN_MASKIDX_W] + P->bin_count[BIN_MASKIDX_B];
    info->kind_units[MSP_KIND_INNER] = P->bin_count[BIN_INNER_W];
    for (int b = 0; b < 8; ++b) info->bin_units[b] = b < NBINS ? P->bin_count[b] : 0;
    return MSP_OK;
}

static NumArgs num_args(const msp_plan* P, int b) {
    NumArgs a{};
    a.op = P->op;
    a.unit_row = P->unit_row;
    a.unit_tile = P->unit_tile;
    a.units = P->bin_units + P->bin_off[b];
    a.nunits = P->bin_count[b];
    return a;
}

static msp_status check_out(const msp_plan* P, const msp_csr_out* C) {
    if (!C) return fail(MSP_ERR_INVALID_ARGUMENT, "C is NULL");
    if (C->nrows != P->op.m || C->ncols != P->op.n)
        return fail(MSP_ERR_DIMENSION_MISMATCH, "C must be A.nrows x B.ncols");
    if (!C->rowptr) return fail(MSP_ERR_INVALID_ARGUMENT, "C.rowptr is NULL");
    if (C->capacity < 0) return fail(MSP_ERR_INVALID_ARGUMENT, "negative capacity");
    if (C->capacity > 0 && (!C->colidx || !C->values))
        return fail(MSP_ERR_INVALID_ARGUMENT, "C.colidx / C.values is NULL");
    return MSP_OK;
}

msp_status msp_symbolic(msp_plan* P, int64_t* C_rowptr, int64_t* nnz_host, void* stream) {
    if (!P || !C_rowptr) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    for (int b = 0; b < NBINS; ++b) {
        if (!P->bin_count[b]) continue;
        NumArgs a = num_args(P, b);
        a.cnt = P->cnt;
        MSP_HIP(launch_numeric(P->sr, b, MODE_COUNT, a, s));
    }
    MSP_HIP(launch_scan(P->cnt, P->cnt, P->U, P->scan_partial, s));
    MSP_HIP(launch_rowptr_from_units(P->op.m, P->unit_base, P->cnt, C_rowptr, s));
    P->symbolic_done = true;
    if (nnz_host) {
        MSP_HIP(hipMemcpyAsync(nnz_host, C_rowptr + P->op.m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
    }
    return MSP_OK;
}

msp_status msp_numeric(msp_plan* P, msp_csr_out* C, void* stream) {
    if (!P) return fail(MSP_ERR_INVALID_ARGUMENT, "plan is NULL");
    MSP_CHECK(check_out(P, C));
    if (!P->symbolic_done) return fail(MSP_ERR_INVALID_ARGUMENT, "msp_numeric needs msp_symbolic first");
    hipStream_t s = (hipStream_t)stream;
    for (int b = 0; b < NBINS; ++b) {
        if (!P->bin_count[b]) continue;
        NumArgs a = num_args(P, b);
        a.out_off = P->cnt;
        a.out_col = C->colidx;
        a.out_val = C->values;
        MSP_HIP(launch_numeric(P->sr, b, MODE_DIRECT, a, s));
    }
    return MSP_OK;
}

// Optional per-stage HIP event timing (msp_execute_profiled).
struct StageTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    hipEvent_t open_ev = nullptr;
    int open_stage = -1;
    msp_status begin(int stage) {
        if (!on) return MSP_OK;
        hipEvent_t e;
        MSP_HIP(hipEventCreate(&e));
        MSP_HIP(hipEventRecord(e, s));
        open_ev = e;
        open_stage = stage;
        return MSP_OK;
    }
    msp_status end() {
        if (!on) return MSP_OK;
        hipEvent_t e;
        MSP_HIP(hipEventCreate(&e));
        MSP_HIP(hipEventRecord(e, s));
        marks.push_back({open_stage, {open_ev, e}});
        return MSP_OK;
    }
    msp_status collect(double* ms) {
        if (!on) return MSP_OK;
        MSP_HIP(hipStreamSynchronize(s));
        for (auto& mk : marks) {
            float t = 0.f;
            MSP_HIP(hipEventElapsedTime(&t, mk.second.first, mk.second.second));
            ms[mk.first] += (double)t;
        }
        return MSP_OK;
    }
    ~StageTimer() {
        for (auto& mk : marks) {
            (void)hipEventDestroy(mk.second.first);
            (void)hipEventDestroy(mk.second.second);
        }
    }
};

static msp_status execute_impl(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, hipStream_t s, StageTimer& tm) {
    if (P->opt.phase == 2) {
        int64_t nnz = 0;
        MSP_CHECK(tm.begin(MSP_STAGE_SYMBOLIC));
        for (int b = 0; b < NBINS; ++b) {
            if (!P->bin_count[b]) continue;
            NumArgs a = num_args(P, b);
            a.cnt = P->cnt;
            MSP_HIP(launch_numeric(P->sr, b, MODE_COUNT, a, s));
        }
        MSP_CHECK(tm.end());
        MSP_CHECK(tm.begin(MSP_STAGE_SCAN));
        MSP_HIP(launch_scan(P->cnt, P->cnt, P->U, P->scan_partial, s));
        MSP_CHECK(tm.end());
        MSP_CHECK(tm.begin(MSP_STAGE_ROWPTR));
        MSP_HIP(launch_rowptr_from_units(P->op.m, P->unit_base, P->cnt, C->rowptr, s));
        MSP_CHECK(tm.end());
        P->symbolic_done = true;
        MSP_HIP(hipMemcpyAsync(&nnz, C->rowptr + P->op.m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
        if (C->capacity < nnz) {
            if (nnz_host) *nnz_host = nnz;
            return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "capacity below nnz(C)");
        }
        for (int b = 0; b < NBINS; ++b) {
            if (!P->bin_count[b]) continue;
            NumArgs a = num_args(P, b);
            a.out_off = P->cnt;
            a.out_col = C->colidx;
            a.out_val = C->values;
            MSP_CHECK(tm.begin(b));
            MSP_HIP(launch_numeric(P->sr, b, MODE_DIRECT, a, s));
            MSP_CHECK(tm.end());
        }
        if (nnz_host) *nnz_host = nnz;
        return MSP_OK;
    }
    if (C->capacity < P->ub) {
        if (nnz_host) *nnz_host = P->ub;
        return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "one-phase output capacity below the upper bound");
    }
    if (!P->stg_col) return fail(MSP_ERR_INVALID_ARGUMENT, "plan has no one-phase staging");
    for (int b = 0; b < NBINS; ++b) {
        if (!P->bin_count[b]) continue;
        NumArgs a = num_args(P, b);
        a.out_off = P->stg_off;
        a.cnt = P->cnt;
        a.out_col = P->stg_col;
        a.out_val = P->stg_val;
        MSP_CHECK(tm.begin(b));
        MSP_HIP(launch_numeric(P->sr, b, MODE_STAGE, a, s));
        MSP_CHECK(tm.end());
    }
    MSP_CHECK(tm.begin(MSP_STAGE_SCAN));
    MSP_HIP(launch_scan(P->cnt, P->cnt, P->U, P->scan_partial, s));
    MSP_CHECK(tm.end());
    MSP_CHECK(tm.begin(MSP_STAGE_ROWPTR));
    MSP_HIP(launch_rowptr_from_units(P->op.m, P->unit_base, P->cnt, C->rowptr, s));
    MSP_CHECK(tm.end());
    CompactArgs ca{};
    ca.m = P->op.m;
    ca.U = P->U;
    ca.unit_base = P->unit_base;
    ca.stg_off = P->stg_off;
    ca.out_off = P->cnt;
    ca.stg_col = P->stg_col;
    ca.stg_val = P->stg_val;
    ca.val_bytes = out_bytes(P->sr);
    ca.C_rowptr = C->rowptr;
    ca.C_col = C->colidx;
    ca.C_val = C->values;
    MSP_CHECK(tm.begin(MSP_STAGE_COMPACT));
    MSP_HIP(launch_compact(ca, s));
    MSP_CHECK(tm.end());
    if (nnz_host) {
        MSP_HIP(hipMemcpyAsync(nnz_host, C->rowptr + P->op.m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
    }
    return MSP_OK;
}

msp_status msp_execute(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, void* stream) {
    if (!P) return fail(MSP_ERR_INVALID_ARGUMENT, "plan is NULL");
    MSP_CHECK(check_out(P, C));
    StageTimer none;
    return execute_impl(P, C, nnz_host, (hipStream_t)stream, none);
}

msp_status msp_execute_profiled(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, double* stage_ms, void* stream) {
    if (!P || !stage_ms) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    MSP_CHECK(check_out(P, C));
    StageTimer tm;
    tm.on = true;
    tm.s = (hipStream_t)stream;
    MSP_CHECK(execute_impl(P, C, nnz_host, tm.s, tm));
    return tm.collect(stage_ms);
}

msp_status msp_plan_row_bins(const msp_plan* P, int8_t* bins, void* stream) {
    if (!P || (!bins && P->op.m > 0)) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    if (P->op.m == 0) return MSP_OK;
    hipStream_t s = (hipStream_t)stream;
    MSP_HIP(hipMemcpyAsync(bins, P->bin, (size_t)P->op.m, hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    return MSP_OK;
}

void msp_plan_destroy(msp_plan* P) {
    if (!P) return;
    P->release();
    delete P;
}

msp_status msp_masked_spgemm(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                             msp_semiring semiring, const msp_options* opt, msp_csr_out* C, int64_t* nnz_host,
                             void* stream) {
    msp_plan* P = nullptr;
    MSP_CHECK(msp_plan_create(&P, A, B, M, complement, semiring, opt, stream));
    const msp_status st = msp_execute(P, C, nnz_host, stream);
    if (st == MSP_OK && !nnz_host) (void)hipStreamSynchronize((hipStream_t)stream);
    msp_plan_destroy(P);
    return st;
}

msp_status msp_upper_bound(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                           int64_t* upper_bound, void* stream) {
    if (!upper_bound) return fail(MSP_ERR_INVALID_ARGUMENT, "upper_bound is NULL");
    msp_plan* P = new (std::nothrow) msp_plan();
    if (!P) return fail(MSP_ERR_OUT_OF_MEMORY, "host allocation");
    msp_options o;
    msp_options_default(&o);
    const msp_status st = plan_create_impl(P, A, B, M, complement, MSP_PLUS_PAIR_I64, &o, (hipStream_t)stream,
                                           false);
    if (st == MSP_OK) *upper_bound = P->ub;
    (void)hipStreamSynchronize((hipStream_t)stream);
    P->release();
    delete P;
    return st;
}

msp_status msp_reduce(const void* values, int64_t n, msp_semiring semiring, void* result, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    if (n < 0 || !result || (n > 0 && !values)) return fail(MSP_ERR_INVALID_ARGUMENT, "bad reduce arguments");
    configure_pool();
    hipStream_t s = (hipStream_t)stream;
    void* partial = nullptr;
    const size_t bytes = sizeof(unsigned long long) * (size_t)reduce_partial_elems();
    bool pooled = true;
    hipError_t e = hipMallocAsync(&partial, bytes, s);
    if (e == hipErrorNotSupported) { pooled = false; e = hipMalloc(&partial, bytes); }
    MSP_HIP(e);
    const hipError_t le = launch_reduce(semiring, values, n, partial, result, s);
    if (pooled) (void)hipFreeAsync(partial, s);
    else { (void)hipStreamSynchronize(s); (void)hipFree(partial); }
    MSP_HIP(le);
    return MSP_OK;
}

}  // extern "C"
