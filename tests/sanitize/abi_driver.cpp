// Sanitizer run of the C-ABI library's host-side checks (built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side by
// tests/test_sanitizers.py): argument errors, dimension rules, CSR shape
// checks, workspace size queries and short workspaces, which all return
// before any device work, so no GPU is needed. Exit status 0 = all good.
#include <cstdio>
#include <cstring>

#include "msp.h"

static int failures = 0;
#define EXPECT(cond)                                                           \
    do {                                                                       \
        if (!(cond)) {                                                         \
            std::fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, msp_last_error()); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static msp_csr csr(int64_t r, int64_t c, int64_t nnz = 0) {
    msp_csr x{};
    x.nrows = r;
    x.ncols = c;
    x.nnz = nnz;
    x.rowptr = reinterpret_cast<const int64_t*>(8);   // never dereferenced on these paths
    x.colidx = nnz ? reinterpret_cast<const int32_t*>(8) : nullptr;
    x.values = nullptr;
    return x;
}

int main() {
    msp_options o;
    msp_options_default(&o);
    EXPECT(o.phase == 1 && o.force_kind == MSP_KIND_AUTO);
    for (int s = -1; s < 10; ++s) EXPECT(msp_status_string((msp_status)s) != nullptr);
    EXPECT(msp_version() > 0);

    msp_plan* h = nullptr;
    msp_csr A = csr(4, 5), B = csr(5, 6), M = csr(4, 6), Bbad = csr(7, 6);
    EXPECT(msp_plan_create(&h, nullptr, &B, &M, 0, MSP_PLUS_TIMES_F64, nullptr, nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    EXPECT(msp_plan_create(&h, &A, &Bbad, &M, 0, MSP_PLUS_TIMES_F64, nullptr, nullptr, 0, nullptr) ==
           MSP_ERR_DIMENSION_MISMATCH);
    EXPECT(msp_plan_create(&h, &A, &B, &M, 0, (msp_semiring)9, nullptr, nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    for (int kind = 1; kind <= 3; ++kind) {
        o.force_kind = kind;
        EXPECT(msp_plan_create(&h, &A, &B, &M, 1, MSP_PLUS_TIMES_F64, &o, nullptr, 0, nullptr) == MSP_ERR_UNSUPPORTED);
    }
    o.force_kind = 7;
    EXPECT(msp_plan_create(&h, &A, &B, &M, 0, MSP_PLUS_TIMES_F64, &o, nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    msp_options_default(&o);
    o.phase = 3;
    EXPECT(msp_plan_create(&h, &A, &B, &M, 0, MSP_PLUS_TIMES_F64, &o, nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    msp_csr Anull = csr(4, 5, 3);
    Anull.colidx = nullptr;
    EXPECT(msp_plan_create(&h, &Anull, &B, &M, 0, MSP_PLUS_TIMES_F64, nullptr, nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    EXPECT(h == nullptr);

    // size queries: shapes only; a big row count grows the plan workspace
    size_t s_small = 0, s_big = 0, s = 0;
    msp_csr sA = csr(100, 50, 10), sB = csr(50, 60, 10), sM = csr(100, 60, 10);
    msp_csr bA = csr(1000000, 50, 10), bM = csr(1000000, 60, 10), wB = csr(50, 300000, 10);
    EXPECT(msp_plan_workspace_size(&sA, &sB, &sM, 0, MSP_PLUS_TIMES_F64, nullptr, &s_small) == MSP_OK);
    EXPECT(msp_plan_workspace_size(&bA, &sB, &bM, 0, MSP_PLUS_TIMES_F64, nullptr, &s_big) == MSP_OK);
    EXPECT(s_big > s_small + 1000000 * 17);
    msp_csr tallB = csr(400000, 60, 10), tallA = csr(100, 400000, 10);
    EXPECT(msp_plan_workspace_size(&tallA, &tallB, &sM, 0, MSP_PLUS_TIMES_F64, nullptr, &s) == MSP_OK);
    EXPECT(s >= 2 * 400000);  // 2-byte row lengths of a B with many rows
    msp_csr wM = csr(100, 300000, 10);
    msp_options_default(&o);
    o.force_kind = MSP_KIND_INNER;
    EXPECT(msp_plan_workspace_size(&sA, &wB, &wM, 0, MSP_PLUS_TIMES_F64, &o, &s) == MSP_OK);
    EXPECT(s > 300000 * 8);  // B^T row pointers
    msp_options_default(&o);
    EXPECT(msp_plan_workspace_size(&sA, &sB, &sM, 0, MSP_PLUS_TIMES_F64, nullptr, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    EXPECT(msp_plan_create(&h, &sA, &sB, &sM, 0, MSP_PLUS_TIMES_F64, nullptr, reinterpret_cast<void*>(256),
                           s_small - 1, nullptr) == MSP_ERR_INSUFFICIENT_CAPACITY);
    size_t need = 0;
    int64_t cnt[2] = {0, 0};
    msp_csr_out out{};
    out.nrows = 100;
    out.ncols = 60;
    EXPECT(msp_masked_spgemm(&sA, &sB, &sM, 0, MSP_PLUS_TIMES_F64, nullptr, &out, cnt, nullptr, 0, &need, nullptr) ==
           MSP_ERR_INSUFFICIENT_CAPACITY);
    EXPECT(need == s_small);
    EXPECT(msp_masked_spgemm(nullptr, &sB, &sM, 0, MSP_PLUS_TIMES_F64, nullptr, &out, cnt, nullptr, 0, &need,
                             nullptr) == MSP_ERR_INVALID_ARGUMENT);

    // batches: sizes add up; argument errors
    msp_problem pr[3];
    std::memset(pr, 0, sizeof(pr));
    for (auto& q : pr) { q.A = sA; q.B = sB; q.M = sM; }
    EXPECT(msp_batch_workspace_size(pr, 3, MSP_PLUS_TIMES_F64, nullptr, &s) == MSP_OK);
    EXPECT(s > s_small);
    EXPECT(msp_batch_workspace_size(pr, 0, MSP_PLUS_TIMES_F64, nullptr, &s) == MSP_ERR_INVALID_ARGUMENT);
    pr[1].B = Bbad;
    EXPECT(msp_batch_workspace_size(pr, 3, MSP_PLUS_TIMES_F64, nullptr, &s) == MSP_ERR_DIMENSION_MISMATCH);

    // reductions and timing sessions
    EXPECT(msp_reduce_workspace_size(&s) == MSP_OK && s > 0);
    EXPECT(msp_reduce(reinterpret_cast<void*>(8), 4, MSP_PLUS_TIMES_F64, reinterpret_cast<void*>(8),
                      reinterpret_cast<void*>(256), s - 1, nullptr) == MSP_ERR_INSUFFICIENT_CAPACITY);
    EXPECT(msp_reduce(nullptr, -1, MSP_PLUS_TIMES_F64, reinterpret_cast<void*>(8), nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    EXPECT(msp_reduce_csr(nullptr, 5, nullptr, 0, MSP_PLUS_PAIR_I64, nullptr, nullptr, 0, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    msp_timing* t = nullptr;
    EXPECT(msp_timing_create(nullptr, 0, 0) == MSP_ERR_INVALID_ARGUMENT);
    EXPECT(msp_timing_create(&t, -1, 0) == MSP_ERR_INVALID_ARGUMENT);
    msp_timing_destroy(nullptr);
    EXPECT(msp_execute_timed(nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr) == MSP_ERR_INVALID_ARGUMENT);

    // iterated products need an allocator
    msp_csr G = csr(4, 4);
    int64_t n = 0;
    int32_t src[1] = {0};
    EXPECT(msp_ktruss(&G, 3, reinterpret_cast<int64_t*>(8), nullptr, nullptr, &n, nullptr, nullptr, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    EXPECT(msp_bc_batch(&G, src, 1, reinterpret_cast<double*>(8), nullptr, nullptr, nullptr) ==
           MSP_ERR_INVALID_ARGUMENT);
    msp_plan_destroy(nullptr);

    if (failures) std::fprintf(stderr, "%d ABI checks failed\n", failures);
    else std::printf("ABI sanitizer run: ok\n");
    return failures != 0;
}
