// Host runtime of the C-ABI (include/msp.h): argument checks, workspace
// layout, kernel sequencing for the one-phase and two-phase paths (Section
// "Symbolic and Numeric Phases"), and batches of products that share one set
// of launches.
//
// A plan covers P >= 1 products on one semiring. Their rows are numbered
// globally (product p owns rows row_off_p .. row_off_p + m_p - 1) and their
// work units share one unit space, so that each kernel bin runs one launch
// over the units of all products; a unit finds its operands through a device
// table. A single product (msp_plan_create) is the case P = 1.
//
// The library allocates no device memory. A plan lays its arrays out in two
// caller-owned buffers: the plan workspace (sized from the operand shapes,
// held by the plan) and the execution workspace (sized from the binning,
// given to every call that runs the product).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <map>
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

}  // namespace

msp_status mspk::set_error(msp_status st, const char* msg) { return fail(st, msg); }

namespace {

// The integer a caller passed for an enumeration parameter. C callers may pass
// any int, and reading an out-of-range value through the C++ enumeration type
// is undefined, so the bits are copied out instead.
template <class E>
int enum_value(const E& e) {
    static_assert(sizeof(E) == sizeof(int), "C enumerations have the size of int");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

bool valid_sr(const msp_semiring& s) {
    const int v = enum_value(s);
    return v >= MSP_PLUS_TIMES_F64 && v <= MSP_PLUS_TIMES_I64;
}

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

msp_status check_triple(const msp_csr* A, const msp_csr* B, const msp_csr* M) {
    MSP_CHECK(check_csr(A, "A"));
    MSP_CHECK(check_csr(B, "B"));
    MSP_CHECK(check_csr(M, "M"));
    if (A->ncols != B->nrows || M->nrows != A->nrows || M->ncols != B->ncols)
        return fail(MSP_ERR_DIMENSION_MISMATCH, "need A.ncols == B.nrows, M.nrows == A.nrows, M.ncols == B.ncols");
    return MSP_OK;
}

// Lays out arrays one after another from `base`, each starting on a 256-byte
// boundary; with a null base it only adds up their sizes (the size queries
// and the checks use the same walk as the placement).
struct Layout {
    char* base = nullptr;
    size_t off = 0;
    void bytes(void** p, size_t n) {
        if (n == 0) n = 1;
        if (p) *p = base ? base + off : nullptr;
        off += (n + 255) & ~(size_t)255;
    }
    template <class T>
    void take(T** p, int64_t n) {
        bytes(reinterpret_cast<void**>(p), (size_t)(n > 0 ? n : 1) * sizeof(T));
    }
};

struct Product {
    Operands op{};
    int64_t row_off = 0;
    int64_t nnzB = 0;
    int64_t nnzA = 0;
    int64_t nnzM = 0;
    // B^T built by the plan for the inner kind (plan workspace)
    int64_t* BTrp = nullptr;
    int32_t* BTci = nullptr;
    void* BTv = nullptr;
    int64_t* bt_part = nullptr;
    unsigned long long* bt_cursor = nullptr;
    bool bt_counted = false, bt_scattered = false;
    uint16_t* bdeg = nullptr;  // B's row lengths, 2 bytes each (plan workspace), when B has many rows
    int64_t gblk0 = 0;         // first analysis block of this product
    int64_t ub = 0, flops = 0, units = 0, staging = 0, mnnz = 0;
    int64_t bin_units[NBINS] = {};
};

}  // namespace

struct msp_plan {
    hipStream_t stream = nullptr;  // stream of creation
    int sr = 0;
    msp_options opt{};
    std::vector<Product> prods;
    int64_t P = 0, R = 0, U = 0, S = 0, ub = 0;
    bool inner_any = false;       // the inner kind may run: pull costs and B^T
    bool plain_readback = false;  // read host values by plain copies (no page-locked buffers)
    // plan workspace: analysis (global rows)
    unsigned long long* stats_d = nullptr;  // [P * ST_COUNT]
    unsigned long long* part = nullptr;     // [ST_COUNT][gtot] statistics per analysis block
    unsigned long long* segtot = nullptr;   // [NSEG] units per segment over all products
    unsigned long long* err_d = nullptr;    // validation: nonzero when an operand is not a valid CSR
    int64_t* blk_off_d = nullptr;           // [P + 1] first analysis block of every product (batches)
    std::vector<int64_t> blk_off_h;         // the same on the host (kept while the plan lives)
    int64_t gtot = 0;                       // analysis blocks of all products
    std::vector<unsigned long long> stats;
    int64_t* flops = nullptr;
    int64_t* unit_base = nullptr;
    int8_t* bin = nullptr;
    int64_t* scan_partial = nullptr;
    int64_t* icost = nullptr;
    // units (global)
    int64_t bin_count[NBINS] = {};
    int64_t bin_off[NBINS + 1] = {};
    bool heap_fold = false;     // BIN_HEAP_L units run in the mask-indexed wave kernel's launch
    bool heap_lm_fold = false;  // BIN_HEAP_LM units run in the mask-indexed block kernel's launch
    bool heap_sort = false;     // BIN_HEAP_L units run in the one-wave sorting kernel
    bool narrow = false;        // the dense kernels read a 16-bit copy of B's column indices
    int64_t narrow_n = 0;       // entries of that copy (nnz(B) when narrow)
    uint16_t* bci16 = nullptr;  // that copy (execution workspace), made by every execution
    int64_t seg_off[NBINS * NBUCKET] = {};
    int64_t nsplit = 0;
    // execution workspace: valid for the workspace the units were last placed in
    const void* placed_ws = nullptr;
    bool placed_staging = false;
    unsigned long long* split_counter = nullptr;  // split rows placed so far
    int32_t* unit_row = nullptr;
    int32_t* unit_tile = nullptr;
    int32_t* unit_prob = nullptr;
    int64_t* stg_off = nullptr;
    int64_t* cnt = nullptr;
    int32_t* bin_units = nullptr;
    int64_t* xpart = nullptr;  // scan partials over the units
    int32_t* stg_col = nullptr;
    void* stg_val = nullptr;
    int32_t* unit_aux = nullptr;
    int32_t* split_first = nullptr;
    int32_t* split_nchunk = nullptr;
    unsigned int* gacc = nullptr;  // [nsplit] x (inserted bits, slots)
    // batch tables (plan workspace)
    Operands* ops_d = nullptr;
    ProdMeta* meta_d = nullptr;            // [P + 1] per-product entries of the batch launches
    int64_t* nnz_d = nullptr;              // [P] output counts gathered for msp_batch_nnz
    bool batch_launch = false;             // analysis and unit placement: one launch for all products
    std::vector<Operands> ops_h;           // host copies of the uploaded tables (kept while the plan lives)
    std::vector<ProdMeta> meta_h;
    std::vector<int64_t> ent_h;
    OutBind* outs_d = nullptr;
    int64_t* ent_off_d = nullptr;
    std::vector<OutBind> outs;
    bool bound = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;
    bool symbolic_done = false;
    int64_t sym_nnz = -1;  // nnz(C) when msp_symbolic read it back
    bool has_table = false;  // the caller's kind per row class (copied at creation)
    int8_t kind_table[MSP_KIND_CLASSES] = {};

    void release() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
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
    opt->maskidx_max = -1;
    opt->heap_flops = -1;
    opt->block_flops = -1;
    opt->split_flops = -1;
    opt->kind_table = nullptr;
}

const char* msp_status_string(msp_status s) {
    switch (enum_value(s)) {
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

int msp_version(void) { return 300; }

}  // extern "C"

// Checks the arguments of a plan over `probs` and fills the plan's options
// and products (host only: no GPU work).
static msp_status plan_setup(msp_plan* P, const msp_problem* probs, int64_t count, msp_semiring semiring,
                             const msp_options* opt) {
    if (count < 1) return fail(MSP_ERR_INVALID_ARGUMENT, "a plan needs at least one product");
    if (!probs) return fail(MSP_ERR_INVALID_ARGUMENT, "problems is NULL");
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    msp_options o;
    msp_options_default(&o);
    if (opt) o = *opt;
    if (o.phase == 0) o.phase = 1;
    if (o.phase != 1 && o.phase != 2) return fail(MSP_ERR_INVALID_ARGUMENT, "phase must be 1 or 2");
    if (count > 1 && o.phase != 1) return fail(MSP_ERR_UNSUPPORTED, "a batch runs one-phase only");
    if (o.force_kind < MSP_KIND_AUTO || o.force_kind > MSP_KIND_HEAP)
        return fail(MSP_ERR_INVALID_ARGUMENT, "unknown force_kind");
    if (o.inner_ratio < 0) return fail(MSP_ERR_INVALID_ARGUMENT, "inner_ratio must be >= 0");
    if (o.maskidx_max < 0) o.maskidx_max = DEFAULT_MASKIDX_MAX;
    if (o.block_flops < 0) o.block_flops = DEFAULT_BLOCK_FLOPS;
    if (o.split_flops < 0) o.split_flops = DEFAULT_SPLIT_FLOPS;
    if (o.heap_flops < 0) o.heap_flops = DEFAULT_HEAP_FLOPS;
    if (count > 1 && o.b_transpose) return fail(MSP_ERR_UNSUPPORTED, "b_transpose applies to a single product");
    P->has_table = o.kind_table != nullptr;
    bool table_inner = false;
    if (o.kind_table) {
        for (int c = 0; c < MSP_KIND_CLASSES; ++c) {
            const int8_t t = o.kind_table[c];
            if (t < MSP_KIND_AUTO || t > MSP_KIND_HEAP) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown kind in kind_table");
            P->kind_table[c] = t;
            table_inner = table_inner || t == MSP_KIND_INNER;
        }
        o.kind_table = nullptr;  // the plan keeps its own copy
    }
    int64_t R = 0;
    P->prods.assign((size_t)count, Product{});
    for (int64_t p = 0; p < count; ++p) {
        const msp_problem& q = probs[p];
        MSP_CHECK(check_triple(&q.A, &q.B, &q.M));
        if (q.complement != 0 && q.complement != 1)
            return fail(MSP_ERR_INVALID_ARGUMENT, "complement must be 0 or 1");
        if (q.complement && o.force_kind != MSP_KIND_AUTO && o.force_kind != MSP_KIND_DENSE &&
            o.force_kind != MSP_KIND_HEAP)
            return fail(MSP_ERR_UNSUPPORTED, "a complemented mask supports only the dense and heap kinds");
        Product& pr = P->prods[(size_t)p];
        Operands& op = pr.op;
        op.m = q.A.nrows; op.k = q.A.ncols; op.n = q.B.ncols;
        op.Arp = q.A.rowptr; op.Aci = q.A.colidx; op.Av = q.A.values;
        op.Brp = q.B.rowptr; op.Bci = q.B.colidx; op.Bv = q.B.values;
        op.Mrp = q.M.rowptr; op.Mci = q.M.colidx;
        op.complement = q.complement;
        pr.nnzA = q.A.nnz;
        pr.nnzB = q.B.nnz;
        pr.nnzM = q.M.nnz;
        pr.row_off = R;
        R += op.m;
    }
    if (R >= INT32_MAX) return fail(MSP_ERR_UNSUPPORTED, "too many rows in one plan");
    if (o.b_transpose) {
        MSP_CHECK(check_csr(o.b_transpose, "B^T"));
        const msp_csr& B = probs[0].B;
        if (o.b_transpose->nrows != B.ncols || o.b_transpose->ncols != B.nrows || o.b_transpose->nnz != B.nnz)
            return fail(MSP_ERR_DIMENSION_MISMATCH, "B^T must be B.ncols x B.nrows with nnz(B) entries");
    }
    P->sr = semiring;
    P->opt = o;
    P->P = count;
    P->R = R;
    P->inner_any = o.force_kind == MSP_KIND_INNER ||
                   (o.force_kind == MSP_KIND_AUTO && (o.inner_ratio > 0 || table_inner));
    return MSP_OK;
}

// The plan workspace: the analysis arrays over the global rows, the batch
// tables, and B^T of every product with a normal mask when the inner kind may
// run and the caller gave no B^T. Returns its size.
static size_t plan_layout(msp_plan* P, char* base) {
    Layout L{base};
    const int64_t count = P->P, R = P->R;
    P->blk_off_h.assign((size_t)count + 1, 0);
    for (int64_t p = 0; p < count; ++p) {
        Product& pr = P->prods[(size_t)p];
        pr.gblk0 = P->blk_off_h[(size_t)p];
        P->blk_off_h[(size_t)p + 1] = pr.gblk0 + analysis_blocks(pr.op.m);
    }
    P->gtot = P->blk_off_h[(size_t)count];
    L.take(&P->stats_d, count * ST_COUNT);
    L.take(&P->part, (int64_t)ST_COUNT * P->gtot);
    L.take(&P->segtot, NSEG);
    L.take(&P->err_d, 1);
    if (count > 1) L.take(&P->blk_off_d, count + 1);
    L.take(&P->flops, R);
    L.take(&P->unit_base, R + 1);
    L.take(&P->bin, R);
    L.take(&P->scan_partial, scan_partial_elems(R + 1));
    for (Product& pr : P->prods)  // B row pointers beyond 2 MB: gather 2-byte lengths instead
        if (pr.op.k > BDEG_MIN_ROWS && pr.nnzA > 0) L.take(&pr.bdeg, pr.op.k);
    if (P->inner_any) {  // pull cost per row, one product at a time (stream order)
        int64_t mmax = 0;
        for (const Product& pr : P->prods) mmax = std::max(mmax, pr.op.m);
        L.take(&P->icost, mmax);
    }
    if (count > 1) {
        L.take(&P->ops_d, count);
        L.take(&P->outs_d, count);
        L.take(&P->ent_off_d, count + 1);
        L.take(&P->meta_d, count + 1);
        L.take(&P->nnz_d, count);
    }
    if (P->inner_any && !P->opt.b_transpose) {
        const int vb = in_bytes(P->sr);
        for (Product& pr : P->prods) {
            if (pr.op.complement) continue;
            L.take(&pr.BTrp, pr.op.n + 1);
            L.take(&pr.bt_part, scan_partial_elems(pr.op.n));
            L.take(&pr.BTci, pr.nnzB);
            if (vb && pr.op.Bv) L.bytes(&pr.BTv, (size_t)(pr.nnzB > 0 ? pr.nnzB : 1) * vb);
            L.take(&pr.bt_cursor, pr.op.n);
        }
    }
    return L.off;
}

// The execution workspace: placement cursors, the unit lists, per-unit
// counts and staging offsets, their scan partials, the split rows'
// accumulators, and the one-phase staging when `staging`. Returns its size.
static size_t exec_layout(msp_plan* P, char* base, bool staging) {
    Layout L{base};
    const int64_t U = P->U;
    L.take(&P->split_counter, 1);
    L.take(&P->unit_row, U);
    L.take(&P->unit_tile, U);
    L.take(&P->unit_prob, U);
    L.take(&P->stg_off, U + 1);
    L.take(&P->cnt, U + 1);
    L.take(&P->bin_units, U);
    L.take(&P->unit_aux, U);
    L.take(&P->xpart, scan_partial_elems(U + 1));
    L.take(&P->split_first, P->nsplit);
    L.take(&P->split_nchunk, P->nsplit);
    if (P->narrow_n > 0) L.take(&P->bci16, P->narrow_n);
    else P->bci16 = nullptr;
    L.bytes(reinterpret_cast<void**>(&P->gacc), (size_t)(P->nsplit > 0 ? P->nsplit : 1) * split_acc_bytes(P->sr));
    if (staging) {
        L.take(&P->stg_col, P->S);
        L.bytes(&P->stg_val, (size_t)(P->S > 0 ? P->S : 1) * out_bytes(P->sr));
    } else {
        P->stg_col = nullptr;
        P->stg_val = nullptr;
    }
    return L.off;
}

static bool exec_staging(const msp_plan* P) { return P->opt.phase == 1; }

// Bytes of the execution workspace: a size-only walk of exec_layout on a copy
// of the sizes, which leaves the plan's placed pointers alone.
static size_t exec_size(const msp_plan* P, bool staging) {
    msp_plan tmp;
    tmp.U = P->U;
    tmp.S = P->S;
    tmp.nsplit = P->nsplit;
    tmp.sr = P->sr;
    tmp.narrow_n = P->narrow_n;
    return exec_layout(&tmp, nullptr, staging);
}

// B^T of product `pr`: column counts and their prefix sum (always), rows
// scattered (when `scatter`). Rows of B^T come out in no particular order.
static msp_status build_transpose(msp_plan* P, Product& pr, bool scatter) {
    const Operands& o = pr.op;
    hipStream_t s = P->stream;
    if (!pr.bt_counted) {
        MSP_HIP(launch_fill_i64(pr.BTrp, o.n + 1, 0, s));
        MSP_HIP(launch_colcount(o.Bci, pr.nnzB, pr.BTrp, s));
        MSP_HIP(launch_scan(pr.BTrp, pr.BTrp, o.n, pr.bt_part, s));
        pr.op.BTrp = pr.BTrp;
        pr.bt_counted = true;
    }
    if (scatter && !pr.bt_scattered) {
        const int vb = in_bytes(P->sr);
        MSP_HIP(launch_fill_i64(reinterpret_cast<int64_t*>(pr.bt_cursor), o.n, 0, s));
        MSP_HIP(launch_transpose_scatter(o.Brp, o.Bci, o.Bv, vb, o.k, pr.BTrp, pr.bt_cursor, pr.BTci, pr.BTv, s));
        pr.op.BTci = pr.BTci;
        pr.op.BTv = pr.BTv;
        pr.bt_scattered = true;
    }
    return MSP_OK;
}

// Page-locked, device-mapped host words for the small device-to-host reads
// (statistics and output counts), reused through a process-wide pool. A
// kernel writes them directly, so a read costs no copy-engine pass.
struct PinnedBuf {
    void* p = nullptr;    // host address
    void* dev = nullptr;  // the same memory as the device addresses it
    size_t cap = 0;
    static std::mutex& mu() {
        static std::mutex m;
        return m;
    }
    static std::multimap<size_t, void*>& pool() {
        static std::multimap<size_t, void*> free_list;
        return free_list;
    }
    msp_status get(size_t bytes) {
        {
            std::lock_guard<std::mutex> lk(mu());
            auto it = pool().lower_bound(bytes);
            if (it != pool().end()) {
                cap = it->first;
                p = it->second;
                pool().erase(it);
                return map_dev();
            }
        }
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        // mapped and coherent: kernels write into it directly, and the host reads it after a
        // stream synchronization
        if (hipHostMalloc(&p, c, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            p = nullptr;
            return fail(MSP_ERR_OUT_OF_MEMORY, "pinned host allocation");
        }
        cap = c;
        return map_dev();
    }
    msp_status map_dev() {
        if (hipHostGetDevicePointer(&dev, p, 0) != hipSuccess) {
            dev = nullptr;
            return fail(MSP_ERR_DEVICE, "no device address for page-locked host memory");
        }
        return MSP_OK;
    }
    ~PinnedBuf() {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu());
        pool().emplace(cap, p);
    }
};

// Reads one int64 from device memory after the stream's work (synchronizes).
static msp_status read_back_i64(const msp_plan* P, int64_t* dst, const int64_t* src, hipStream_t s) {
    if (P && P->plain_readback) {
        int64_t v = 0;
        MSP_HIP(hipMemcpyAsync(&v, src, sizeof(v), hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
        *dst = v;
        return MSP_OK;
    }
    PinnedBuf pin;
    MSP_CHECK(pin.get(sizeof(int64_t)));
    MSP_HIP(launch_peek(src, static_cast<int64_t*>(pin.dev), s));
    MSP_HIP(hipStreamSynchronize(s));
    std::memcpy(dst, pin.p, sizeof(int64_t));
    return MSP_OK;
}

static msp_status plan_create_impl(msp_plan* P, const msp_problem* probs, int64_t count, msp_semiring semiring,
                                   const msp_options* opt, void* ws, size_t ws_bytes, hipStream_t stream) {
    MSP_CHECK(plan_setup(P, probs, count, semiring, opt));
    const size_t need = plan_layout(P, nullptr);
    if (ws_bytes < need)
        return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "plan workspace of " + std::to_string(ws_bytes) +
                                                       " bytes is below the " + std::to_string(need) + " needed");
    if (!ws) return fail(MSP_ERR_INVALID_ARGUMENT, "plan workspace is NULL");
    plan_layout(P, static_cast<char*>(ws));
    const msp_options& o = P->opt;
    const int64_t R = P->R;
    P->stream = stream;
    hipStream_t s = stream;

    // the statistics and every product's row counts start at zero (one launch)
    MSP_HIP(launch_zero2(reinterpret_cast<int64_t*>(P->err_d), 1, P->flops, R, s));
    if (o.validate) {
        unsigned long long* err = P->err_d;
        for (int64_t p = 0; p < count; ++p) {
            const msp_problem& q = probs[p];
            MSP_HIP(launch_validate(q.A.rowptr, q.A.colidx, q.A.nrows, q.A.ncols, q.A.nnz, err, s));
            MSP_HIP(launch_validate(q.B.rowptr, q.B.colidx, q.B.nrows, q.B.ncols, q.B.nnz, err, s));
            MSP_HIP(launch_validate(q.M.rowptr, q.M.colidx, q.M.nrows, q.M.ncols, q.M.nnz, err, s));
        }
        if (o.b_transpose)
            MSP_HIP(launch_validate(o.b_transpose->rowptr, o.b_transpose->colidx, o.b_transpose->nrows,
                                    o.b_transpose->ncols, o.b_transpose->nnz, err, s));
        // validation must finish before the analysis trusts the row pointers
        unsigned long long e = 0;
        MSP_HIP(hipMemcpyAsync(&e, err, sizeof(e), hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
        if (e) return fail(MSP_ERR_INVALID_CSR, "an operand violates the CSR invariants");
    }
    for (int64_t p = 0; p < count; ++p) {
        Product& pr = P->prods[(size_t)p];
        if (pr.op.complement || !P->inner_any) continue;
        if (o.b_transpose) {
            pr.op.BTrp = o.b_transpose->rowptr;
            pr.op.BTci = o.b_transpose->colidx;
            pr.op.BTv = o.b_transpose->values;
        } else {
            MSP_CHECK(build_transpose(P, pr, o.force_kind == MSP_KIND_INNER));
        }
    }
    // a batch without pull costs: the row sums and the analysis of all products in one launch each
    P->batch_launch = count > 1 && !P->inner_any;
    if (P->batch_launch) {
        P->ops_h.resize((size_t)count);
        P->meta_h.assign((size_t)count + 1, ProdMeta{});
        int64_t chunks = 0;
        for (int64_t p = 0; p < count; ++p) {
            const Product& pr = P->prods[(size_t)p];
            P->ops_h[(size_t)p] = pr.op;
            P->meta_h[(size_t)p] = ProdMeta{pr.bdeg, pr.row_off, pr.gblk0, chunks, pr.nnzA};
            chunks += rowsum_chunks(pr.nnzA);
        }
        P->meta_h[(size_t)count] = ProdMeta{nullptr, R, P->gtot, chunks, 0};
        P->ent_h.assign((size_t)count + 1, 0);
        for (int64_t p = 0; p < count; ++p)
            P->ent_h[(size_t)p + 1] = P->ent_h[(size_t)p] + P->prods[(size_t)p].op.m + 1;
        // the tables go up before the plan's synchronization below, which also ends the copies' reads
        // of the host vectors
        MSP_HIP(hipMemcpyAsync(P->ops_d, P->ops_h.data(), sizeof(Operands) * count, hipMemcpyHostToDevice, s));
        MSP_HIP(hipMemcpyAsync(P->meta_d, P->meta_h.data(), sizeof(ProdMeta) * (count + 1), hipMemcpyHostToDevice,
                               s));
        MSP_HIP(hipMemcpyAsync(P->ent_off_d, P->ent_h.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice,
                               s));
        for (int64_t p = 0; p < count; ++p) {
            const Product& pr = P->prods[(size_t)p];
            if (pr.bdeg) MSP_HIP(launch_deg16(pr.op.Brp, pr.op.k, pr.bdeg, s));
        }
        AnalysisArgs aa{};
        aa.force_kind = o.force_kind;
        aa.inner_ratio = 0;
        aa.maskidx_max = o.maskidx_max;
        aa.block_flops = o.block_flops;
        aa.split_flops = o.split_flops;
        aa.heap_flops = o.heap_flops;
        aa.has_table = P->has_table && o.force_kind == MSP_KIND_AUTO;
        std::memcpy(aa.kind_table, P->kind_table, sizeof(aa.kind_table));
        aa.icost = nullptr;
        aa.flops = P->flops;
        aa.flops_zeroed = true;
        aa.tiles = P->unit_base;
        aa.bin = P->bin;
        aa.part = P->part;
        aa.gtot = P->gtot;
        MSP_HIP(launch_analysis_batch(aa, P->ops_d, P->meta_d, count, chunks, P->gtot, s));
    }
    for (int64_t p = 0; p < count && !P->batch_launch; ++p) {
        Product& pr = P->prods[(size_t)p];
        AnalysisArgs aa{};
        aa.op = pr.op;
        aa.row_off = pr.row_off;
        aa.force_kind = o.force_kind;
        aa.inner_ratio = (!pr.op.complement && P->inner_any) ? o.inner_ratio : 0;
        aa.maskidx_max = o.maskidx_max;
        aa.block_flops = o.block_flops;
        aa.split_flops = o.split_flops;
        aa.heap_flops = o.heap_flops;
        aa.has_table = P->has_table && o.force_kind == MSP_KIND_AUTO;
        std::memcpy(aa.kind_table, P->kind_table, sizeof(aa.kind_table));
        aa.colcnt_rp = pr.op.BTrp;
        aa.a_nnz = pr.nnzA;
        aa.m_nnz = pr.nnzM;
        aa.icost = (aa.inner_ratio > 0 && aa.colcnt_rp && o.force_kind == MSP_KIND_AUTO) ? P->icost : nullptr;
        aa.flops = P->flops;
        aa.flops_zeroed = true;
        aa.tiles = P->unit_base;
        aa.bin = P->bin;
        aa.bdeg = pr.bdeg;
        aa.part = P->part;
        aa.gtot = P->gtot;
        aa.gblk0 = pr.gblk0;
        if (pr.bdeg) MSP_HIP(launch_deg16(pr.op.Brp, pr.op.k, pr.bdeg, s));
        MSP_HIP(launch_analysis(aa, s));
    }
    MSP_HIP(launch_scan(P->unit_base, P->unit_base, R, P->scan_partial, s));
    {
        // the one synchronization of plan creation: the statistics size the unit arrays
        const size_t sb = sizeof(unsigned long long) * ST_COUNT * (size_t)count;
        P->stats.assign((size_t)(count * ST_COUNT), 0ull);
        if (count > 1)  // the host copy lives as long as the plan
            MSP_HIP(hipMemcpyAsync(P->blk_off_d, P->blk_off_h.data(), sizeof(int64_t) * (count + 1),
                                   hipMemcpyHostToDevice, s));
        if (P->plain_readback) {
            MSP_HIP(launch_segoff(P->part, P->gtot, P->blk_off_d, count, P->stats_d, nullptr, P->segtot, s));
            MSP_HIP(hipMemcpyAsync(P->stats.data(), P->stats_d, sb, hipMemcpyDeviceToHost, s));
            MSP_HIP(hipStreamSynchronize(s));
        } else {
            PinnedBuf pin;
            MSP_CHECK(pin.get(sb));
            MSP_HIP(launch_segoff(P->part, P->gtot, P->blk_off_d, count, P->stats_d,
                                  static_cast<unsigned long long*>(pin.dev), P->segtot, s));
            MSP_HIP(hipStreamSynchronize(s));
            std::memcpy(P->stats.data(), pin.p, sb);
        }
    }

    // totals; bins in order, inside a bin the flops buckets from the heaviest down
    std::vector<int64_t> segc(NBINS * NBUCKET, 0);
    int64_t heap_apart = 0, heap_lm_apart = 0;
    for (int64_t p = 0; p < count; ++p) {
        Product& pr = P->prods[(size_t)p];
        const unsigned long long* st = &P->stats[(size_t)(p * ST_COUNT)];
        pr.ub = (int64_t)st[ST_UB];
        pr.flops = (int64_t)st[ST_FLOPS];
        pr.units = (int64_t)st[ST_UNITS];
        pr.staging = (int64_t)st[ST_STAGING];
        pr.mnnz = (int64_t)st[ST_MNNZ];
        for (int b = 0; b < NBINS; ++b) {
            int64_t t = 0;
            for (int q = 0; q < NBUCKET; ++q) {
                t += (int64_t)st[ST_BIN0 + b * NBUCKET + q];
                segc[(size_t)(b * NBUCKET + q)] += (int64_t)st[ST_BIN0 + b * NBUCKET + q];
            }
            pr.bin_units[b] = t;
        }
        P->U += pr.units;
        P->S += pr.staging;
        P->ub += pr.ub;
        P->nsplit += (int64_t)st[ST_SPLITROWS];
        heap_apart += (int64_t)st[ST_HEAP_APART];
        heap_lm_apart += (int64_t)st[ST_HEAPLM_APART];
    }
    int64_t run = 0;
    for (int x = 0; x < NBINS; ++x) {  // the layout of the unit list (the device computed the same)
        const int b = bin_at(x);
        P->bin_off[b] = run;
        for (int q = NBUCKET - 1; q >= 0; --q) {
            P->seg_off[b * NBUCKET + q] = run;
            run += segc[(size_t)(b * NBUCKET + q)];
        }
        P->bin_count[b] = run - P->bin_off[b];
    }
    P->bin_off[NBINS] = run;
    if (run != P->U) return fail(MSP_ERR_DEVICE, "inconsistent unit statistics");
    P->heap_fold = o.force_kind == MSP_KIND_AUTO && P->bin_count[BIN_HEAP_L] > 0 &&
                   P->bin_count[BIN_HEAP_L] <= HEAP_FOLD_MAX && heap_apart == 0;
    P->heap_lm_fold = o.force_kind == MSP_KIND_AUTO && P->bin_count[BIN_HEAP_LM] > 0 &&
                      P->bin_count[BIN_HEAP_LM] <= HEAP_LM_FOLD_MAX && heap_lm_apart == 0;
    // A small heap bin that no mask-indexed launch takes (complemented rows) is as slow as its
    // longest lane's serial merge; when each of its rows has fewer than 256 products, the
    // one-wave sorting kernel runs them side by side instead.
    P->heap_sort = o.force_kind == MSP_KIND_AUTO && !P->heap_fold && P->bin_count[BIN_HEAP_L] > 0 &&
                   P->bin_count[BIN_HEAP_L] <= HEAP_FOLD_MAX &&
                   P->seg_off[BIN_HEAP_L * NBUCKET + ESC_LIGHT_FROM_BUCKET] == P->bin_off[BIN_HEAP_L];
    // The one-tile dense kernels of a single product over at most 512 columns re-read B's rows
    // once per entry of A that selects them: when their products (a lower bound from the flops
    // buckets) come to NARROW_REUSE times nnz(B) or more, each execution first copies B's column
    // indices to 16 bits, halving the bytes of the column stream.
    if (P->P == 1 && P->prods[0].op.n <= DENSE_W_COLS && P->prods[0].nnzB > 0) {
        int64_t dense_flops = 0;
        for (int b : {BIN_DENSE_W, BIN_DENSE_BN, BIN_DENSE_SPLIT})
            for (int q = 0; q < NBUCKET; ++q)
                dense_flops += segc[(size_t)(b * NBUCKET + q)] * (q == 0 ? 1 : (int64_t(1) << (2 * q)));
        P->narrow = dense_flops >= NARROW_REUSE * P->prods[0].nnzB;
    }
    P->narrow_n = P->narrow ? P->prods[0].nnzB : 0;
    if (P->U >= INT32_MAX) return fail(MSP_ERR_UNSUPPORTED, "too many work units");
    for (int64_t p = 0; p < count; ++p) {
        Product& pr = P->prods[(size_t)p];
        if (pr.bin_units[BIN_INNER_W] > 0 && !o.b_transpose) MSP_CHECK(build_transpose(P, pr, true));
    }
    if (count > 1 && !P->batch_launch) {  // the operand table (B^T may have been built since) and the row offsets
        P->ops_h.resize((size_t)count);
        P->ent_h.assign((size_t)count + 1, 0);
        for (int64_t p = 0; p < count; ++p) {
            P->ops_h[(size_t)p] = P->prods[(size_t)p].op;
            P->ent_h[(size_t)p + 1] = P->ent_h[(size_t)p] + P->prods[(size_t)p].op.m + 1;
        }
        MSP_HIP(hipMemcpyAsync(P->ops_d, P->ops_h.data(), sizeof(Operands) * count, hipMemcpyHostToDevice, s));
        MSP_HIP(hipMemcpyAsync(P->ent_off_d, P->ent_h.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice,
                               s));
        MSP_HIP(hipStreamSynchronize(s));  // the copies have read the host vectors
    }
    return MSP_OK;
}

// Places the work units in the execution workspace `ws`: every row's units
// into its (bin, flops bucket) segment, their staging sizes and, when
// `staging`, the staging offsets (a prefix sum). Kernels only.
static msp_status place_units(msp_plan* P, void* ws, size_t ws_bytes, bool staging, hipStream_t s) {
    const size_t need = exec_layout(P, nullptr, staging);
    if (ws_bytes < need)
        return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "execution workspace of " + std::to_string(ws_bytes) +
                                                       " bytes is below the " + std::to_string(need) + " needed");
    if (!ws) return fail(MSP_ERR_INVALID_ARGUMENT, "execution workspace is NULL");
    exec_layout(P, static_cast<char*>(ws), staging);
    P->placed_ws = nullptr;
    // the split-row counter starts at zero
    MSP_HIP(launch_fill_i64(reinterpret_cast<int64_t*>(P->split_counter), 1, 0, s));
    for (int64_t p = 0; p < (P->batch_launch ? 1 : P->P); ++p) {
        Product& pr = P->prods[(size_t)p];
        if (pr.op.m == 0 && !P->batch_launch) continue;
        UnitArgs ua{};
        ua.op = pr.op;
        ua.row_off = pr.row_off;
        ua.prob = (int32_t)p;
        ua.flops = P->flops;
        ua.unit_base = P->unit_base;
        ua.bin = P->bin;
        ua.part = P->part;
        ua.gtot = P->gtot;
        ua.gblk0 = pr.gblk0;
        ua.segtot = P->segtot;
        ua.unit_row = P->unit_row;
        ua.unit_tile = P->unit_tile;
        ua.unit_prob = P->unit_prob;
        ua.stg_size = P->stg_off;
        ua.bin_units = P->bin_units;
        ua.split_counter = P->split_counter;
        ua.unit_aux = P->unit_aux;
        ua.split_first = P->split_first;
        ua.split_nchunk = P->split_nchunk;
        if (P->batch_launch)  // every product's units in one launch (per-product fields from the tables)
            MSP_HIP(launch_units_batch(ua, P->ops_d, P->meta_d, P->P, P->gtot, s));
        else
            MSP_HIP(launch_units(ua, pr.op.m, s));
    }
    if (staging) MSP_HIP(launch_scan(P->stg_off, P->stg_off, P->U, P->xpart, s));
    P->placed_ws = ws;
    P->placed_staging = staging;
    return MSP_OK;
}

static msp_status create_common(msp_plan** plan, const msp_problem* probs, int64_t count, msp_semiring semiring,
                                const msp_options* opt, void* ws, size_t ws_bytes, void* stream,
                                bool plain_readback = false) {
    if (!plan) return fail(MSP_ERR_INVALID_ARGUMENT, "plan is NULL");
    *plan = nullptr;
    msp_plan* P = new (std::nothrow) msp_plan();
    if (!P) return fail(MSP_ERR_OUT_OF_MEMORY, "host allocation");
    P->plain_readback = plain_readback;
    const msp_status st = plan_create_impl(P, probs, count, semiring, opt, ws, ws_bytes, (hipStream_t)stream);
    if (st != MSP_OK) {
        // kernels enqueued before the error may still use the caller's workspace
        (void)hipStreamSynchronize((hipStream_t)stream);
        P->release();
        delete P;
        return st;
    }
    *plan = P;
    return MSP_OK;
}

static msp_status workspace_size_common(const msp_problem* probs, int64_t count, msp_semiring semiring,
                                        const msp_options* opt, size_t* bytes) {
    if (!bytes) return fail(MSP_ERR_INVALID_ARGUMENT, "bytes is NULL");
    msp_plan tmp;
    MSP_CHECK(plan_setup(&tmp, probs, count, semiring, opt));
    *bytes = plan_layout(&tmp, nullptr);
    return MSP_OK;
}

static NumArgs num_args(const msp_plan* P, int b) {
    NumArgs a{};
    a.op = P->prods[0].op;
    a.ops = P->P > 1 ? P->ops_d : nullptr;
    a.unit_prob = P->unit_prob;
    a.unit_row = P->unit_row;
    a.unit_tile = P->unit_tile;
    a.units = P->bin_units + P->bin_off[b];
    a.nunits = P->bin_count[b];
    a.unit_aux = P->unit_aux;
    a.split_first = P->split_first;
    a.split_nchunk = P->split_nchunk;
    a.nsplit = P->nsplit;
    a.gset = P->gacc;
    a.gval = P->gacc + (size_t)P->nsplit * (DENSE_B_COLS / 32);
    for (const Product& pr : P->prods) a.max_n = std::max(a.max_n, pr.op.n);
    if (P->narrow) a.op.Bci16 = P->bci16;
    return a;
}

// Split rows: clear their global accumulators before the numeric kernels.
static msp_status split_clear(msp_plan* P, hipStream_t s) {
    if (P->nsplit <= 0) return MSP_OK;
    MSP_HIP(launch_fill_u32(P->gacc, (int64_t)(P->nsplit * split_acc_bytes(P->sr) / 4), s));
    return MSP_OK;
}

// Split rows: ordered emission after all numeric kernels.
static msp_status split_emit(msp_plan* P, int mode, const NumArgs& base, hipStream_t s) {
    if (P->nsplit <= 0) return MSP_OK;
    NumArgs a = base;
    MSP_HIP(launch_split_emit(P->sr, mode, a, s));
    return MSP_OK;
}

static msp_status check_out(const Product& pr, const msp_csr_out* C) {
    if (!C) return fail(MSP_ERR_INVALID_ARGUMENT, "C is NULL");
    if (C->nrows != pr.op.m || C->ncols != pr.op.n) return fail(MSP_ERR_DIMENSION_MISMATCH, "C must be A.nrows x B.ncols");
    if (!C->rowptr) return fail(MSP_ERR_INVALID_ARGUMENT, "C.rowptr is NULL");
    if (C->capacity < 0) return fail(MSP_ERR_INVALID_ARGUMENT, "negative capacity");
    if (C->capacity > 0 && (!C->colidx || !C->values))
        return fail(MSP_ERR_INVALID_ARGUMENT, "C.colidx / C.values is NULL");
    return MSP_OK;
}

static OutBind bind_of(const msp_plan* P, const msp_csr_out* C, int64_t p) {
    const Product& pr = P->prods[(size_t)p];
    OutBind ob{};
    ob.rowptr = C->rowptr;
    ob.col = C->colidx;
    ob.val = C->values;
    ob.row_off = pr.row_off;
    ob.nrows = pr.op.m;
    // units of earlier products come first in the global unit numbering
    int64_t first = 0;
    for (int64_t q = 0; q < p; ++q) first += P->prods[(size_t)q].units;
    ob.unit_first = first;
    return ob;
}

// Optional per-stage HIP event timing (msp_execute_profiled).
// Per-thread, per-device pool of timing events (created once, reused).
static std::vector<hipEvent_t>& event_pool() {
    thread_local std::map<int, std::vector<hipEvent_t>> pools;
    int dev = 0;
    (void)hipGetDevice(&dev);
    return pools[dev];
}

// A timing session (msp_timing_*): the event pairs of any number of
// executions, read out together by msp_timing_collect. Its events are its own.
struct msp_timing {
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    std::vector<hipEvent_t> spare;  // events free for reuse
    std::vector<hipEvent_t> all;    // every event created, destroyed with the session
    int device = 0;
    uint32_t stages = 0;            // bit s set: stage s is timed
};

// Stage times from events attached to the stage's own kernel launches
// (hipExtLaunchKernel): begin() arms a start/stop pair, end() disarms it.
// With a session the pairs go to the session and are read later; otherwise
// collect() reads them after synchronizing the stream.
struct StageTimer {
    bool on = false;
    hipStream_t s = nullptr;
    msp_timing* sess = nullptr;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    std::vector<hipEvent_t> held;  // taken from the pool, returned at destruction
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    int open_stage = -1;
    msp_status take(hipEvent_t* e) {
        if (sess) {
            if (sess->spare.empty()) {
                MSP_HIP(hipEventCreate(e));
                sess->all.push_back(*e);
            } else {
                *e = sess->spare.back();
                sess->spare.pop_back();
            }
            return MSP_OK;
        }
        auto& pool = event_pool();
        if (pool.empty()) {
            // the events of a whole execution are created at once, before the first of them is
            // recorded: creating one between a stage's start and stop events would count the
            // host's creation time in that stage
            for (int x = 0; x < 2 * MSP_NSTAGES; ++x) {
                hipEvent_t f = nullptr;
                MSP_HIP(hipEventCreate(&f));
                pool.push_back(f);
            }
        }
        *e = pool.back();
        pool.pop_back();
        held.push_back(*e);
        return MSP_OK;
    }
    msp_status begin(int stage) {
        if (!on) return MSP_OK;
        if (sess && !((sess->stages >> stage) & 1u)) {  // not a stage of this session
            open_stage = -1;
            return MSP_OK;
        }
        MSP_CHECK(take(&ev_start));
        MSP_CHECK(take(&ev_stop));
        open_stage = stage;
        timing_arm(ev_start, ev_stop);
        return MSP_OK;
    }
    msp_status end() {
        if (!on || open_stage < 0) return MSP_OK;
        if (timing_disarm()) {
            (sess ? sess->marks : marks).push_back({open_stage, {ev_start, ev_stop}});
        } else if (sess) {  // nothing was launched: the pair is free again
            sess->spare.push_back(ev_start);
            sess->spare.push_back(ev_stop);
        }
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
        (void)timing_disarm();
        auto& pool = event_pool();
        for (hipEvent_t e : held) pool.push_back(e);
    }
};

// Numeric kernels of every non-empty bin, in bin order on `s`, in `mode`,
// with `a` giving the outputs. A folded heap bin runs as part of its
// mask-indexed neighbour's launch: BIN_HEAP_L's units directly follow the
// wave bin's, BIN_HEAP_LM's directly precede the block bin's.
static msp_status launch_bins(msp_plan* P, int mode, const NumArgs& a, hipStream_t s, StageTimer* tm) {
    if (P->narrow) {  // the 16-bit copy of B's column indices that the dense kernels read
        if (tm) MSP_CHECK(tm->begin(MSP_STAGE_PLACE));
        MSP_HIP(launch_narrow_cols(P->prods[0].op.Bci, P->bci16, P->prods[0].nnzB, s));
        if (tm) MSP_CHECK(tm->end());
    }
    for (int b = 0; b < NBINS; ++b) {
        if ((P->heap_fold && b == BIN_HEAP_L) || (P->heap_lm_fold && b == BIN_HEAP_LM)) continue;
        const int64_t after = P->heap_fold && b == BIN_MASKIDX_W ? P->bin_count[BIN_HEAP_L] : 0;
        const int64_t before = P->heap_lm_fold && b == BIN_MASKIDX_B ? P->bin_count[BIN_HEAP_LM] : 0;
        if (!P->bin_count[b] && !after && !before) continue;
        NumArgs ab = a;
        ab.units = P->bin_units + P->bin_off[b] - before;
        ab.nunits = P->bin_count[b] + after + before;
        if (tm) MSP_CHECK(tm->begin(b));
        // the mask-indexed block bin's heaviest units (its first buckets) in a wider launch
        const int64_t wide = b == BIN_MASKIDX_B && MASKIDX_B_WIDE_BUCKET > 0
                                 ? P->seg_off[b * NBUCKET + MASKIDX_B_WIDE_BUCKET - 1] - P->bin_off[b]
                                 : 0;
        if (wide > 0) {
            NumArgs aw = a;
            aw.units = P->bin_units + P->bin_off[b];
            aw.nunits = wide;
            MSP_HIP(launch_numeric(P->sr, LAUNCH_MASKIDX_B_WIDE, mode, aw, s));
            if (before > 0) {  // the folded heap units that precede the bin
                NumArgs ah = a;
                ah.units = P->bin_units + P->bin_off[b] - before;
                ah.nunits = before;
                MSP_HIP(launch_numeric(P->sr, b, mode, ah, s));
            }
            ab.units = P->bin_units + P->bin_off[b] + wide;
            ab.nunits = P->bin_count[b] - wide;
        }
        if (b == BIN_ESC) {
            // the sorting bin's lighter units (its last buckets) in smaller workgroups
            const int64_t e_end = P->bin_off[b] + P->bin_count[b];
            const int64_t e_mid = P->seg_off[b * NBUCKET + ESC_MID_FROM_BUCKET];
            const int64_t e_light = P->seg_off[b * NBUCKET + ESC_LIGHT_FROM_BUCKET];
            ab.nunits = e_mid - P->bin_off[b];
            NumArgs am = a, al = a;
            am.units = P->bin_units + e_mid;
            am.nunits = e_light - e_mid;
            al.units = P->bin_units + e_light;
            al.nunits = e_end - e_light;
            if (am.nunits > 0) MSP_HIP(launch_numeric(P->sr, LAUNCH_ESC_MID, mode, am, s));
            if (al.nunits > 0) MSP_HIP(launch_numeric(P->sr, LAUNCH_ESC_LIGHT, mode, al, s));
            if (ab.nunits <= 0) {
                if (tm) MSP_CHECK(tm->end());
                continue;
            }
        }
        MSP_HIP(launch_numeric(P->sr, P->heap_sort && b == BIN_HEAP_L ? LAUNCH_ESC_LIGHT : b, mode, ab, s));
        if (tm) MSP_CHECK(tm->end());
    }
    return MSP_OK;
}

// The one-phase sequence over all products: numeric into staging, prefix sum
// of the unit counts, row pointers, compaction. Kernels only (no allocation,
// no memset, no synchronization), so it can be captured in a HIP graph. The
// units must be placed (with staging) in the execution workspace.
static msp_status run_one_phase(msp_plan* P, const OutBind& one, hipStream_t s, StageTimer& tm) {
    if (!P->placed_ws || !P->placed_staging) return fail(MSP_ERR_INVALID_ARGUMENT, "no one-phase workspace placed");
    MSP_CHECK(split_clear(P, s));
    NumArgs a = num_args(P, 0);
    a.out_off = P->stg_off;
    a.cnt = P->cnt;
    a.out_col = P->stg_col;
    a.out_val = P->stg_val;
    MSP_CHECK(launch_bins(P, MODE_STAGE, a, s, &tm));
    MSP_CHECK(tm.begin(MSP_STAGE_SPLIT_EMIT));
    MSP_CHECK(split_emit(P, MODE_STAGE, a, s));
    MSP_CHECK(tm.end());
    MSP_CHECK(tm.begin(MSP_STAGE_SCAN));
    MSP_HIP(launch_scan(P->cnt, P->cnt, P->U, P->xpart, s));
    MSP_CHECK(tm.end());
    const OutBind* outs = P->P > 1 ? P->outs_d : nullptr;
    const int64_t entries = P->P > 1 ? P->R + P->P : P->prods[0].op.m + 1;
    MSP_CHECK(tm.begin(MSP_STAGE_ROWPTR));
    MSP_HIP(launch_rowptr(P->P, entries, P->ent_off_d, outs, one, P->unit_base, P->cnt, s));
    MSP_CHECK(tm.end());
    CompactArgs ca{};
    ca.U = P->U;
    ca.stg_off = P->stg_off;
    ca.out_off = P->cnt;
    ca.unit_prob = P->unit_prob;
    ca.stg_col = P->stg_col;
    ca.stg_val = P->stg_val;
    ca.val_bytes = out_bytes(P->sr);
    ca.one = one;
    ca.outs = outs;
    MSP_CHECK(tm.begin(MSP_STAGE_COMPACT));
    MSP_HIP(launch_compact(ca, s));
    MSP_CHECK(tm.end());
    return MSP_OK;
}

static msp_status symbolic_impl(msp_plan* P, int64_t* C_rowptr, int64_t* nnz_host, void* ws, size_t ws_bytes,
                                hipStream_t s, StageTimer& tm) {
    const Product& pr = P->prods[0];
    P->symbolic_done = false;
    P->sym_nnz = -1;
    MSP_CHECK(tm.begin(MSP_STAGE_PLACE));
    MSP_CHECK(place_units(P, ws, ws_bytes, false, s));
    MSP_CHECK(tm.end());
    MSP_CHECK(tm.begin(MSP_STAGE_SYMBOLIC));
    MSP_CHECK(split_clear(P, s));
    {
        NumArgs a = num_args(P, 0);
        a.cnt = P->cnt;
        MSP_CHECK(launch_bins(P, MODE_COUNT, a, s, nullptr));
    }
    {
        NumArgs a = num_args(P, 0);
        a.cnt = P->cnt;
        MSP_CHECK(split_emit(P, MODE_COUNT, a, s));
    }
    MSP_CHECK(tm.end());
    MSP_CHECK(tm.begin(MSP_STAGE_SCAN));
    MSP_HIP(launch_scan(P->cnt, P->cnt, P->U, P->xpart, s));
    MSP_CHECK(tm.end());
    OutBind one{};
    one.rowptr = C_rowptr;
    one.nrows = pr.op.m;
    MSP_CHECK(tm.begin(MSP_STAGE_ROWPTR));
    MSP_HIP(launch_rowptr(1, pr.op.m + 1, nullptr, nullptr, one, P->unit_base, P->cnt, s));
    MSP_CHECK(tm.end());
    P->symbolic_done = true;
    if (nnz_host) {
        MSP_CHECK(read_back_i64(P, nnz_host, C_rowptr + pr.op.m, s));
        P->sym_nnz = *nnz_host;
    }
    return MSP_OK;
}

// Two-phase numeric step; the workspace must be the one msp_symbolic placed
// the units in, and C must hold nnz(C).
static msp_status numeric_impl(msp_plan* P, msp_csr_out* C, const void* ws, hipStream_t s, StageTimer& tm) {
    if (!P->symbolic_done) return fail(MSP_ERR_INVALID_ARGUMENT, "msp_numeric needs msp_symbolic first");
    if (!ws || ws != P->placed_ws || P->placed_staging)
        return fail(MSP_ERR_INVALID_ARGUMENT, "msp_numeric needs the execution workspace of msp_symbolic");
    if (C->capacity < P->ub) {
        int64_t nnz = P->sym_nnz;
        if (nnz < 0) {  // the count after the scan of the unit counts
            MSP_CHECK(read_back_i64(P, &nnz, P->cnt + P->U, s));
            P->sym_nnz = nnz;
        }
        if (C->capacity < nnz) return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "capacity below nnz(C)");
    }
    MSP_CHECK(split_clear(P, s));
    NumArgs a = num_args(P, 0);
    a.out_off = P->cnt;
    a.out_col = C->colidx;
    a.out_val = C->values;
    MSP_CHECK(launch_bins(P, MODE_DIRECT, a, s, &tm));
    MSP_CHECK(tm.begin(MSP_STAGE_SPLIT_EMIT));
    MSP_CHECK(split_emit(P, MODE_DIRECT, a, s));
    MSP_CHECK(tm.end());
    return MSP_OK;
}

static msp_status execute_impl(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, void* ws, size_t ws_bytes,
                               hipStream_t s, StageTimer& tm) {
    if (P->P != 1) return fail(MSP_ERR_INVALID_ARGUMENT, "msp_execute takes a single-product plan; use msp_batch_*");
    const Product& pr = P->prods[0];
    MSP_CHECK(check_out(pr, C));
    if (P->opt.phase == 2) {
        int64_t nnz = 0;
        MSP_CHECK(symbolic_impl(P, C->rowptr, &nnz, ws, ws_bytes, s, tm));
        if (C->capacity < nnz) {
            if (nnz_host) *nnz_host = nnz;
            return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "capacity below nnz(C)");
        }
        MSP_CHECK(numeric_impl(P, C, ws, s, tm));
        if (nnz_host) *nnz_host = nnz;
        return MSP_OK;
    }
    if (C->capacity < P->ub) {
        if (nnz_host) *nnz_host = P->ub;
        return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "one-phase output capacity below the upper bound");
    }
    MSP_CHECK(tm.begin(MSP_STAGE_PLACE));
    MSP_CHECK(place_units(P, ws, ws_bytes, true, s));
    MSP_CHECK(tm.end());
    const OutBind one = bind_of(P, C, 0);
    MSP_CHECK(run_one_phase(P, one, s, tm));
    if (nnz_host) MSP_CHECK(read_back_i64(P, nnz_host, C->rowptr + pr.op.m, s));
    return MSP_OK;
}

static msp_problem single_problem(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement) {
    msp_problem pb{};
    pb.A = *A;
    pb.B = *B;
    pb.M = *M;
    pb.complement = complement;
    return pb;
}

// The workspace of msp_masked_spgemm_noalloc: a fixed array in device memory
// that each GPU the library runs on holds until the process ends. In host
// code its name is only a host-side stand-in; the array's device address on
// a GPU comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[MSP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// The scratch array's device address on the current device.
static msp_status scratch_address(void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    MSP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MSP_ERR_UNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return from_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                   "hipGetSymbolAddress(scratch)");
        addr[dev] = p;
    }
    *out = addr[dev];
    return MSP_OK;
}

// The one-shot product in one workspace: the plan workspace, then the
// execution workspace.
static msp_status one_shot(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                           msp_semiring semiring, const msp_options* opt, msp_csr_out* C, int64_t* nnz_host,
                           void* ws, size_t ws_bytes, size_t* ws_needed, hipStream_t s, bool plain_readback) {
    if (!A || !B || !M) return fail(MSP_ERR_INVALID_ARGUMENT, "A, B and M must not be NULL");
    const msp_problem pb = single_problem(A, B, M, complement);
    size_t pneed = 0;
    MSP_CHECK(workspace_size_common(&pb, 1, semiring, opt, &pneed));
    if (ws_bytes < pneed) {
        if (ws_needed) *ws_needed = pneed;
        return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "workspace of " + std::to_string(ws_bytes) +
                                                       " bytes is below the plan's " + std::to_string(pneed));
    }
    msp_plan* P = nullptr;
    MSP_CHECK(create_common(&P, &pb, 1, semiring, opt, ws, pneed, s, plain_readback));
    const size_t xneed = exec_layout(P, nullptr, exec_staging(P));
    msp_status st = MSP_OK;
    if (ws_bytes - pneed < xneed) {
        if (ws_needed) *ws_needed = pneed + xneed;
        st = fail(MSP_ERR_INSUFFICIENT_CAPACITY, "workspace of " + std::to_string(ws_bytes) + " bytes is below the " +
                                                     std::to_string(pneed + xneed) + " needed");
    } else {
        if (ws_needed) *ws_needed = pneed + xneed;
        StageTimer none;
        st = execute_impl(P, C, nnz_host, static_cast<char*>(ws) + pneed, ws_bytes - pneed, s, none);
    }
    // the caller may reuse the workspace when this returns
    const hipError_t e = hipStreamSynchronize(s);
    msp_plan_destroy(P);
    if (st == MSP_OK) MSP_HIP(e);
    return st;
}

extern "C" {

msp_status msp_plan_workspace_size(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                                   msp_semiring semiring, const msp_options* opt, size_t* bytes) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    if (!A || !B || !M) return fail(MSP_ERR_INVALID_ARGUMENT, "A, B and M must not be NULL");
    const msp_problem pb = single_problem(A, B, M, complement);
    return workspace_size_common(&pb, 1, semiring, opt, bytes);
}

msp_status msp_batch_workspace_size(const msp_problem* problems, int64_t count, msp_semiring semiring,
                                    const msp_options* opt, size_t* bytes) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    return workspace_size_common(problems, count, semiring, opt, bytes);
}

msp_status msp_plan_create(msp_plan** plan, const msp_csr* A, const msp_csr* B, const msp_csr* M,
                           int complement, msp_semiring semiring, const msp_options* opt, void* workspace,
                           size_t workspace_bytes, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    if (!A || !B || !M) return fail(MSP_ERR_INVALID_ARGUMENT, "A, B and M must not be NULL");
    const msp_problem pb = single_problem(A, B, M, complement);
    return create_common(plan, &pb, 1, semiring, opt, workspace, workspace_bytes, stream);
}

msp_status msp_workspace_size(const msp_plan* P, size_t* bytes) {
    if (!P || !bytes) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    *bytes = exec_size(P, exec_staging(P));
    return MSP_OK;
}

msp_status msp_plan_info(const msp_plan* P, msp_plan_info_t* info) { return msp_batch_info(P, -1, info); }

msp_status msp_symbolic(msp_plan* P, int64_t* C_rowptr, int64_t* nnz_host, void* workspace, size_t workspace_bytes,
                        void* stream) {
    if (!P || !C_rowptr) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    if (P->P != 1) return fail(MSP_ERR_INVALID_ARGUMENT, "msp_symbolic takes a single-product plan");
    StageTimer none;
    return symbolic_impl(P, C_rowptr, nnz_host, workspace, workspace_bytes, (hipStream_t)stream, none);
}

msp_status msp_numeric(msp_plan* P, msp_csr_out* C, void* workspace, size_t workspace_bytes, void* stream) {
    if (!P) return fail(MSP_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (P->P != 1) return fail(MSP_ERR_INVALID_ARGUMENT, "msp_numeric takes a single-product plan");
    MSP_CHECK(check_out(P->prods[0], C));
    size_t need = 0;
    MSP_CHECK(msp_workspace_size(P, &need));
    if (P->opt.phase == 1) need = exec_size(P, false);  // a one-phase plan's size includes staging
                                                         // that the two-phase steps leave unused
    if (workspace_bytes < need) return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "execution workspace too small");
    StageTimer none;
    return numeric_impl(P, C, workspace, (hipStream_t)stream, none);
}

msp_status msp_execute(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, void* workspace, size_t workspace_bytes,
                       void* stream) {
    if (!P) return fail(MSP_ERR_INVALID_ARGUMENT, "plan is NULL");
    StageTimer none;
    return execute_impl(P, C, nnz_host, workspace, workspace_bytes, (hipStream_t)stream, none);
}

msp_status msp_execute_profiled(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, void* workspace,
                                size_t workspace_bytes, double* stage_ms, void* stream) {
    if (!P || !stage_ms) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    StageTimer tm;
    tm.on = true;
    tm.s = (hipStream_t)stream;
    MSP_CHECK(execute_impl(P, C, nnz_host, workspace, workspace_bytes, tm.s, tm));
    return tm.collect(stage_ms);
}

msp_status msp_timing_create(msp_timing** timing, int32_t executions, uint32_t stages) {
    if (!timing) return fail(MSP_ERR_INVALID_ARGUMENT, "timing is NULL");
    if (executions < 0) return fail(MSP_ERR_INVALID_ARGUMENT, "executions must be >= 0");
    msp_timing* T = new (std::nothrow) msp_timing();
    if (!T) return fail(MSP_ERR_OUT_OF_MEMORY, "timing session");
    (void)hipGetDevice(&T->device);
    T->stages = stages ? stages : (uint32_t)((1ull << MSP_NSTAGES) - 1);
    // events for `executions` executions are created now, outside any timed region
    const int64_t n = 2 * (int64_t)MSP_NSTAGES * executions;
    for (int64_t x = 0; x < n; ++x) {
        hipEvent_t e = nullptr;
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) {
            msp_timing_destroy(T);
            return fail(MSP_ERR_DEVICE, "hipEventCreate for the timing session");
        }
        T->all.push_back(e);
        T->spare.push_back(e);
    }
    *timing = T;
    return MSP_OK;
}

void msp_timing_destroy(msp_timing* T) {
    if (!T) return;
    for (hipEvent_t e : T->all) (void)hipEventDestroy(e);
    delete T;
}

msp_status msp_execute_timed(msp_plan* P, msp_csr_out* C, int64_t* nnz_host, void* workspace, size_t workspace_bytes,
                             msp_timing* T, void* stream) {
    if (!P || !T) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    int dev = 0;
    MSP_HIP(hipGetDevice(&dev));
    if (dev != T->device) return fail(MSP_ERR_INVALID_ARGUMENT, "the timing session belongs to another device");
    StageTimer tm;
    tm.on = true;
    tm.s = (hipStream_t)stream;
    tm.sess = T;
    return execute_impl(P, C, nnz_host, workspace, workspace_bytes, tm.s, tm);
}

msp_status msp_timing_collect(msp_timing* T, double* stage_ms) {
    if (!T || !stage_ms) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    for (auto& mk : T->marks) {
        MSP_HIP(hipEventSynchronize(mk.second.second));
        float t = 0.f;
        MSP_HIP(hipEventElapsedTime(&t, mk.second.first, mk.second.second));
        stage_ms[mk.first] += (double)t;
        T->spare.push_back(mk.second.first);
        T->spare.push_back(mk.second.second);
    }
    T->marks.clear();
    return MSP_OK;
}

msp_status msp_plan_row_bins(const msp_plan* P, int8_t* bins, void* stream) {
    if (!P || (!bins && P->R > 0)) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    if (P->R == 0) return MSP_OK;
    hipStream_t s = (hipStream_t)stream;
    MSP_HIP(hipMemcpyAsync(bins, P->bin, (size_t)P->R, hipMemcpyDeviceToHost, s));
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
                             void* workspace, size_t workspace_bytes, size_t* ws_needed, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    return one_shot(A, B, M, complement, semiring, opt, C, nnz_host, workspace, workspace_bytes, ws_needed,
                    (hipStream_t)stream, false);
}

msp_status msp_masked_spgemm_noalloc(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                                     msp_semiring semiring, const msp_options* opt, msp_csr_out* C,
                                     int64_t* nnz_host, size_t* ws_needed, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    void* ws = nullptr;
    MSP_CHECK(scratch_address(&ws));
    size_t need = 0;
    // plain copies for the host reads: no page-locked host memory either
    const msp_status st = one_shot(A, B, M, complement, semiring, opt, C, nnz_host, ws, MSP_NOALLOC_SCRATCH_BYTES,
                                   &need, (hipStream_t)stream, true);
    if (ws_needed) *ws_needed = need;
    if (st == MSP_ERR_INSUFFICIENT_CAPACITY && need > MSP_NOALLOC_SCRATCH_BYTES)
        return fail(st, "the product needs " + std::to_string(need) + " bytes of workspace (or more), above the " +
                            std::to_string((size_t)MSP_NOALLOC_SCRATCH_BYTES) +
                            " bytes of the fixed scratch; use msp_masked_spgemm with a workspace");
    return st;
}

msp_status msp_upper_bound(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                           int64_t* upper_bound, void* workspace, size_t workspace_bytes, void* stream) {
    if (!upper_bound) return fail(MSP_ERR_INVALID_ARGUMENT, "upper_bound is NULL");
    if (!A || !B || !M) return fail(MSP_ERR_INVALID_ARGUMENT, "A, B and M must not be NULL");
    const msp_problem pb = single_problem(A, B, M, complement);
    msp_plan* P = nullptr;
    MSP_CHECK(create_common(&P, &pb, 1, MSP_PLUS_PAIR_I64, nullptr, workspace, workspace_bytes, stream));
    *upper_bound = P->ub;
    msp_plan_destroy(P);
    return MSP_OK;
}

static msp_status reduce_impl(const void* values, int64_t n, const int64_t* n_dev, msp_semiring semiring,
                              void* result, void* ws, size_t ws_bytes, void* stream);

msp_status msp_reduce_workspace_size(size_t* bytes) {
    if (!bytes) return fail(MSP_ERR_INVALID_ARGUMENT, "bytes is NULL");
    *bytes = sizeof(unsigned long long) * (size_t)reduce_partial_elems();
    return MSP_OK;
}

msp_status msp_reduce(const void* values, int64_t n, msp_semiring semiring, void* result, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    return reduce_impl(values, n, nullptr, semiring, result, workspace, workspace_bytes, stream);
}

msp_status msp_reduce_csr(const int64_t* rowptr, int64_t nrows, const void* values, int64_t capacity,
                          msp_semiring semiring, void* result, void* workspace, size_t workspace_bytes,
                          void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    if (!rowptr || nrows < 0) return fail(MSP_ERR_INVALID_ARGUMENT, "bad row pointers");
    return reduce_impl(values, capacity, rowptr + nrows, semiring, result, workspace, workspace_bytes, stream);
}

static msp_status reduce_impl(const void* values, int64_t n, const int64_t* n_dev, msp_semiring semiring,
                              void* result, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    if (n < 0 || !result || (n > 0 && !values)) return fail(MSP_ERR_INVALID_ARGUMENT, "bad reduce arguments");
    size_t need = 0;
    MSP_CHECK(msp_reduce_workspace_size(&need));
    if (ws_bytes < need) return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "reduce workspace too small");
    if (!ws) return fail(MSP_ERR_INVALID_ARGUMENT, "reduce workspace is NULL");
    MSP_HIP(launch_reduce(semiring, values, n, n_dev, ws, result, (hipStream_t)stream));
    return MSP_OK;
}

// ------------------------------------------------------------------- batches

msp_status msp_batch_create(msp_plan** batch, const msp_problem* problems, int64_t count, msp_semiring semiring,
                            const msp_options* opt, void* workspace, size_t workspace_bytes, void* stream) {
    if (!valid_sr(semiring)) return fail(MSP_ERR_INVALID_ARGUMENT, "unknown semiring");
    return create_common(batch, problems, count, semiring, opt, workspace, workspace_bytes, stream);
}

int64_t msp_batch_count(const msp_plan* P) { return P ? P->P : 0; }

msp_status msp_batch_info(const msp_plan* P, int64_t p, msp_plan_info_t* info) {
    if (!P || !info) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    if (p < -1 || p >= P->P) return fail(MSP_ERR_INVALID_ARGUMENT, "product index out of range");
    std::memset(info, 0, sizeof(*info));
    for (int64_t q = 0; q < P->P; ++q) {
        if (p >= 0 && q != p) continue;
        const Product& pr = P->prods[(size_t)q];
        info->upper_bound += pr.ub;
        info->products += pr.flops;
        info->units += pr.units;
        info->staging += pr.staging;
        info->mask_nnz += pr.mnnz;
        info->kind_units[MSP_KIND_DENSE] += pr.bin_units[BIN_DENSE_W] + pr.bin_units[BIN_DENSE_B] +
                                            pr.bin_units[BIN_DENSE_BN] + pr.bin_units[BIN_DENSE_SPLIT];
        info->kind_units[MSP_KIND_HASH] += pr.bin_units[BIN_HASH_W] + pr.bin_units[BIN_HASH_B];
        info->kind_units[MSP_KIND_MASKIDX] +=
            pr.bin_units[BIN_MASKIDX_W] + pr.bin_units[BIN_MASKIDX_B] + pr.bin_units[BIN_MASKIDX_P];
        info->kind_units[MSP_KIND_INNER] += pr.bin_units[BIN_INNER_W];
        info->kind_units[MSP_KIND_HEAP] += pr.bin_units[BIN_HEAP_L] + pr.bin_units[BIN_HEAP_LM];
        info->kind_units[MSP_KIND_HEAP + 1] += pr.bin_units[BIN_ESC];
        for (int b = 0; b < NBINS; ++b) info->bin_units[b] += pr.bin_units[b];
    }
    return MSP_OK;
}

msp_status msp_batch_bind(msp_plan* P, const msp_csr_out* C, void* workspace, size_t workspace_bytes, void* stream) {
    if (!P || !C) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument");
    if (P->opt.phase != 1) return fail(MSP_ERR_UNSUPPORTED, "a batch runs one-phase only");
    std::vector<OutBind> outs((size_t)P->P);
    for (int64_t p = 0; p < P->P; ++p) {
        const Product& pr = P->prods[(size_t)p];
        MSP_CHECK(check_out(pr, &C[p]));
        if (C[p].capacity < pr.ub) return fail(MSP_ERR_INSUFFICIENT_CAPACITY, "output capacity below its upper bound");
        outs[(size_t)p] = bind_of(P, &C[p], p);
    }
    // a captured graph refers to the previous outputs and workspace
    if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
    if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
    P->bound = false;
    hipStream_t s = (hipStream_t)stream;
    MSP_CHECK(place_units(P, workspace, workspace_bytes, true, s));
    if (P->P > 1)
        MSP_HIP(hipMemcpyAsync(P->outs_d, outs.data(), sizeof(OutBind) * P->P, hipMemcpyHostToDevice, s));
    MSP_HIP(hipStreamSynchronize(s));
    P->outs = std::move(outs);
    P->bound = true;
    return MSP_OK;
}

msp_status msp_batch_execute(msp_plan* P, void* stream) {
    if (!P || !P->bound) return fail(MSP_ERR_INVALID_ARGUMENT, "batch outputs are not bound");
    StageTimer none;
    return run_one_phase(P, P->outs[0], (hipStream_t)stream, none);
}

msp_status msp_batch_execute_timed(msp_plan* P, msp_timing* T, void* stream) {
    if (!P || !P->bound) return fail(MSP_ERR_INVALID_ARGUMENT, "batch outputs are not bound");
    if (!T) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL timing session");
    int dev = 0;
    MSP_HIP(hipGetDevice(&dev));
    if (dev != T->device) return fail(MSP_ERR_INVALID_ARGUMENT, "the timing session belongs to another device");
    StageTimer tm;
    tm.on = true;
    tm.s = (hipStream_t)stream;
    tm.sess = T;
    return run_one_phase(P, P->outs[0], tm.s, tm);
}

msp_status msp_batch_graph_launch(msp_plan* P, void* stream) {
    if (!P || !P->bound) return fail(MSP_ERR_INVALID_ARGUMENT, "batch outputs are not bound");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(MSP_ERR_INVALID_ARGUMENT, "graph capture needs a non-default stream");
    if (P->gexec && P->graph_stream != s) {
        (void)hipGraphExecDestroy(P->gexec);
        (void)hipGraphDestroy(P->graph);
        P->gexec = nullptr;
        P->graph = nullptr;
    }
    if (!P->gexec) {
        MSP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        StageTimer none;
        const msp_status st = run_one_phase(P, P->outs[0], s, none);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(s, &g);
        if (st != MSP_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        MSP_HIP(ee);
        P->graph = g;
        MSP_HIP(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
        P->graph_stream = s;
    }
    MSP_HIP(hipGraphLaunch(P->gexec, s));
    return MSP_OK;
}

msp_status msp_batch_nnz(const msp_plan* P, int64_t* nnz, void* stream) {
    if (!P || !nnz || !P->bound) return fail(MSP_ERR_INVALID_ARGUMENT, "NULL argument or unbound batch");
    hipStream_t s = (hipStream_t)stream;
    if (P->P > 1) {  // one gather kernel and one copy for all products
        MSP_HIP(launch_batch_nnz(P->outs_d, P->P, P->nnz_d, s));
        MSP_HIP(hipMemcpyAsync(nnz, P->nnz_d, sizeof(int64_t) * P->P, hipMemcpyDeviceToHost, s));
    } else {
        const OutBind& ob = P->outs[0];
        MSP_HIP(hipMemcpyAsync(&nnz[0], ob.rowptr + ob.nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    MSP_HIP(hipStreamSynchronize(s));
    return MSP_OK;
}

}  // extern "C"
