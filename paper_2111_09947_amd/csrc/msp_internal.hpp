// Internal interface between the host runtime (msp_api.cpp) and the kernels
// (msp_kernels.hip). Not installed; the public interface is include/msp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "msp.h"

namespace mspk {

// Work-unit bins. A unit is a row of C, or one tile of a heavy row: a chunk
// of the row's mask entries (mask-keyed kinds) or a column window (dense).
enum Bin : int {  // same numbering as MSP_BIN_* in msp.h
    BIN_DENSE_W = 0,    // one wave, dense state over <= DENSE_W_COLS columns
    BIN_DENSE_B = 1,    // one block, dense state over a DENSE_B_COLS column tile
    BIN_HASH_W = 2,     // one wave, hash table of <= HASH_W_CAP mask entries
    BIN_HASH_B = 3,     // one block, hash table of <= HASH_B_CAP mask entries
    BIN_MASKIDX_W = 4,  // one wave, binary search over <= MASKIDX_W_CAP mask entries
    BIN_MASKIDX_B = 5,  // one block, binary search over <= MASKIDX_B_CAP mask entries
    BIN_INNER_W = 6,    // one wave, dot products for <= INNER_CAP mask entries
    BIN_DENSE_BN = 7,   // one block, dense state over <= DENSE_W_COLS columns (product-heavy rows)
    BIN_DENSE_SPLIT = 8,  // one block per chunk of A's row, dense state over <= DENSE_B_COLS
                          // columns, merged into a per-row accumulator in global memory
    BIN_HEAP_L = 9,     // one lane per row, k-way merge of <= HEAP_CAP rows of B by a heap in LDS
                        // (normal masks of <= MASKIDX_W_CAP entries, and complemented masks)
    BIN_HEAP_LM = 10,   // the same for normal masks of more than MASKIDX_W_CAP entries
    BIN_MASKIDX_P = 11,  // eight lanes per row, eight rows per wave: short normal mask rows
                         // (<= PACK_MASK entries), few products (<= PACK_FLOPS), short rows of A
    BIN_ESC = 12,        // one block per row: complemented rows of matrices wider than DENSE_B_COLS
                         // with more than heap_flops and <= ESC_MAX products: expand, sort, fold
    NBINS = 13
};

constexpr int DENSE_W_COLS = 512;
constexpr int DENSE_B_COLS = 4096;
constexpr int HASH_W_CAP = 256;
constexpr int HASH_B_CAP = 512;
constexpr int MASKIDX_W_CAP = 256;
// Keys per tile of the mask-indexed block kind. Its lookups are binary
// searches over the tile's keys in LDS, so the kernel is bound by LDS latency
// rather than by issue: 2048 keys keep a workgroup's LDS (keys, values, flags,
// filter, candidate rings) at 36-47 KB, three or four workgroups per CU, which hides
// that latency better than two workgroups of 4096-key tiles. Smaller tiles
// help hub rows a little more but leave rows of a few thousand mask entries
// and few products in a heap launch of their own (a folded heap unit must fit
// one tile).
#ifndef MSP_MASKIDX_B_CAP
#define MSP_MASKIDX_B_CAP 2048
#endif
constexpr int MASKIDX_B_CAP = MSP_MASKIDX_B_CAP;
constexpr int INNER_CAP = 256;
// The packed mask-indexed bin (automatic choice only): a row fits it with a
// normal mask row of at most PACK_MASK entries, at most PACK_FLOPS products
// and at most PACK_ALEN entries in its row of A. Such rows take PACK_G lanes
// each; a wave per row would leave most of its 64 lanes idle on them (an
// Erdos-Renyi row of degree 8 has 64 products and 8 mask entries).
#ifndef MSP_PACK_G
#define MSP_PACK_G 8
#endif
constexpr int PACK_G = MSP_PACK_G;
constexpr int PACK_MASK = 16;
constexpr int PACK_ALEN = 32;
constexpr int64_t PACK_FLOPS = 256;
// Complemented rows of matrices wider than one dense tile (DENSE_B_COLS
// columns) would make the dense kind stream the row once per 4096-column tile.
// A row of more than heap_flops and at most ESC_MAX products is expanded into
// LDS, sorted by column, folded and filtered against its mask row instead
// (automatic choice only); lighter rows, and heavier ones that fit it, take
// the heap.
constexpr int64_t ESC_MAX = 4096;
// Rows of at least ESC_WAVE_MAX products take the four-wave sorting shape,
// whose LDS sort costs more than restreaming the row over fewer than
// ESC_BLOCK_MIN_TILES dense tiles: those rows keep the dense tiles.
constexpr int64_t ESC_WAVE_MAX = 1024;
constexpr int64_t ESC_BLOCK_MIN_TILES = 10;
// Dense kernels read a 16-bit copy of B's column indices when their products
// come to at least this many times nnz(B) (single products, n <= 512).
constexpr int64_t NARROW_REUSE = 4;
constexpr int INNER_ACAP = 1024;  // A row (column indices) staged in LDS up to this length
constexpr int BLOCK_NW = 4;       // waves per block for the block kinds
#ifndef MSP_MASKIDX_B_NW
#define MSP_MASKIDX_B_NW 4
#endif
constexpr int MASKIDX_B_NW = MSP_MASKIDX_B_NW;  // waves per block of the mask-indexed block kind
// The mask-indexed block bin's heaviest units (rows of at least
// 4^MASKIDX_B_WIDE_BUCKET products, 0: none) run in a launch of their own
// with MASKIDX_B_WIDE_NW waves per unit: such rows have many batches of A
// entries for the waves to claim, and the extra waves hide the latency of
// the search lookups. Lighter units would leave the extra waves idle.
#ifndef MSP_MASKIDX_B_WIDE_BUCKET
#define MSP_MASKIDX_B_WIDE_BUCKET 8
#endif
constexpr int MASKIDX_B_WIDE_BUCKET = MSP_MASKIDX_B_WIDE_BUCKET;
constexpr int MASKIDX_B_WIDE_NW = 8;
constexpr int LAUNCH_MASKIDX_B_WIDE = NBINS;  // launch id (not a bin) of that kernel
// The sorting bin's units of fewer than 4^5 products run in a launch of one
// wave per unit with room for 1024 products, and those of fewer than 4^4 in
// one of a wave per unit with room for 256.
constexpr int ESC_MID_FROM_BUCKET = 4;
constexpr int ESC_LIGHT_FROM_BUCKET = 3;
constexpr int LAUNCH_ESC_MID = NBINS + 1;
constexpr int LAUNCH_ESC_LIGHT = NBINS + 2;
constexpr int HEAP_CAP = 8;       // heap kind: iterators per row (entries of the row of A)
constexpr int64_t HEAP_MAX_FLOPS = (int64_t(1) << 24) - 1;  // heap keys hold a B row's remaining length in 24 bits
constexpr int64_t HEAP_LONG_MASK_RATIO = 8;  // auto HEAP also when the mask row has >= this many entries per product
constexpr int64_t HEAP_LONG_MASK_FLOPS = 2;  // ... and the row has at most this many times heap_flops products
// An automatic heap bin of at most this many units, all of them rows that the
// neighbouring mask-indexed kernel can take with the same staging (BIN_HEAP_L:
// the wave kernel, normal masks of at most MASKIDX_W_CAP entries; BIN_HEAP_LM:
// the block kernel, at most MASKIDX_B_CAP entries, one tile), runs in that
// kernel's launch instead of a launch of its own: a small heap launch costs
// its latency-bound tail (a lane walks its row serially, a long mask row
// costs a binary search per product) and saves less than that. The block
// kernel spends time per mask entry, so long-mask bins fold only when small.
constexpr int64_t HEAP_FOLD_MAX = 32768;
constexpr int64_t HEAP_LM_FOLD_MAX = 4096;

// Position x of the unit list holds the units of bin bin_at(x): the bins in
// numeric order, except that the two heap bins sit between the mask-indexed
// wave and block bins (wave, heap, heap with long masks, block), so that each
// heap bin and its mask-indexed neighbour form one contiguous range of units;
// the packed and the sorting bins come last.
__host__ __device__ inline int bin_at(int x) {
    return x >= BIN_MASKIDX_P ? x
           : x <= BIN_MASKIDX_W ? x
           : x == BIN_MASKIDX_W + 1 ? (int)BIN_HEAP_L
           : x == BIN_MASKIDX_W + 2 ? (int)BIN_HEAP_LM
           : x - 2;
}
constexpr int DEFAULT_MASKIDX_MAX = 8;       // auto: binary search up to this mask size, hash above
constexpr int64_t DEFAULT_BLOCK_FLOPS = 8192;  // rows with more products run on a whole block
// ... except dense-kind rows of matrices with at most DENSE_W_COLS columns,
// which take a block only above this many times block_flops products: the
// one-wave tile of 512 columns needs no block barriers and its per-row setup
// is small, and on the 512-source BFS step one wave per row measured faster
// up to the split threshold (6.20 against 6.39 ms a step with int32 path
// counts, 5.57 against 5.96 ms boolean).
constexpr int64_t DENSE_NARROW_BLOCK_MULT = 32;
constexpr int DEFAULT_HEAP_FLOPS = 32;           // auto: HEAP for fitting rows with at most this many products
constexpr int64_t DEFAULT_SPLIT_FLOPS = 262144;  // dense rows with more products split over several blocks
// Units of a bin are ordered by the product count of their row, heaviest
// first (bucket b holds rows with 4^b <= flops < 4^(b+1)), so that the
// longest units start first and do not form the tail of the launch.
constexpr int NBUCKET = 12;
static_assert(NBUCKET == MSP_ROW_BUCKETS, "row classes use the flops buckets");

// Device statistics written by the analysis kernel (one sync reads them).
enum Stat : int {
    ST_FLOPS = 0,
    ST_UB = 1,
    ST_UNITS = 2,
    ST_STAGING = 3,
    ST_MNNZ = 4,
    ST_MAXFLOPS = 5,
    ST_BIN0 = 6,                 // ST_BIN0 + b * NBUCKET + bucket: units of bin b in a flops bucket
    ST_SPLITROWS = ST_BIN0 + NBINS * NBUCKET,  // rows split over several blocks
    ST_HEAP_APART = ST_SPLITROWS + 1,      // BIN_HEAP_L rows the mask-indexed wave kernel cannot take
    ST_HEAPLM_APART = ST_HEAP_APART + 1,   // BIN_HEAP_LM rows the mask-indexed block kernel cannot take
    ST_COUNT = ST_HEAPLM_APART + 1
};

enum Mode : int { MODE_COUNT = 0, MODE_STAGE = 1, MODE_DIRECT = 2 };

struct Operands {
    int64_t m, k, n;
    const int64_t* Arp; const int32_t* Aci; const void* Av;
    const int64_t* Brp; const int32_t* Bci; const void* Bv;
    const int64_t* Mrp; const int32_t* Mci;
    const int64_t* BTrp; const int32_t* BTci; const void* BTv;  // B^T (inner kind)
    const uint16_t* Bci16;  // B's column indices in 16 bits (single products, n <= 65536), or null
    int complement;
};

struct AnalysisArgs {
    Operands op;
    int64_t row_off;           // first global row of this product
    int force_kind;
    int inner_ratio;
    int maskidx_max;
    int64_t block_flops;
    int64_t split_flops;
    int64_t heap_flops;        // auto: HEAP for fitting rows with at most this many products (0 = never)
    int has_table;             // auto: kind_table holds a kind per row class
    int8_t kind_table[MSP_KIND_CLASSES];
    const int64_t* colcnt_rp;  // row pointers of B^T (column counts of B) or null
    int64_t a_nnz;             // nnz(A), nnz(M)
    int64_t m_nnz;
    int64_t* icost;            // [m] pull cost per row (auto INNER choice) or null
    int64_t* flops;            // [R] global rows
    bool flops_zeroed;         // flops of this product's rows are zero already
    int64_t* tiles;            // [R+1], number of units per row (scanned later)
    int8_t* bin;               // [R]
    const uint16_t* bdeg;      // [k] row lengths of B saturated at 0xFFFF (or null: read B's row pointers)
    // every analysis block writes its statistics to part[x * gtot + gblk0 + block] (no atomics)
    unsigned long long* part;  // [ST_COUNT][gtot]
    int64_t gtot;              // analysis blocks of all products of the plan
    int64_t gblk0;             // first analysis block of this product
};

// Blocks of one product's analysis (and unit placement): one per chunk of
// 256 rows up to ANA_MAXB (8 per CU), each walking every ANA_MAXB-th chunk;
// the two kernels split the rows identically, so that the placement can use
// the analysis's per-block counts.
constexpr int ANA_ROWS = 256;
constexpr int64_t ANA_MAXB = 2048;
__host__ __device__ inline int64_t analysis_blocks(int64_t m) {
    const int64_t b = (m + ANA_ROWS - 1) / ANA_ROWS;
    return b < ANA_MAXB ? b : ANA_MAXB;
}
constexpr int NSEG = NBINS * NBUCKET;  // (bin, flops bucket) segments of the unit list
// Per-product entries of a batch's analysis launches (a device table of
// count + 1 entries; the last holds the totals), so that the row sums, the
// analysis and the unit placement run as one launch each for all products.
struct ProdMeta {
    const uint16_t* bdeg;  // B's 2-byte row lengths, or null
    int64_t row_off;       // first global row
    int64_t blk0;          // first analysis block
    int64_t chunk0;        // first row-sum chunk
    int64_t a_nnz;         // nnz(A)
};
// When B has more rows than this, its row pointers (8 bytes a row) exceed
// 2 MB, half of one XCD's L2: the product count per row then gathers B's row
// lengths from a 2-byte copy instead.
constexpr int64_t BDEG_MIN_ROWS = 262144;

struct UnitArgs {
    Operands op;
    int64_t row_off;           // first global row of this product
    int32_t prob;              // product index
    const int64_t* flops;
    const int64_t* unit_base;  // [R+1] exclusive scan of tiles over global rows
    const int8_t* bin;
    // per analysis block and segment, the block's first position inside the segment (exclusive
    // prefix over the blocks of all products, in place of the analysis's counts) ...
    const unsigned long long* part;  // [ST_COUNT][gtot]
    int64_t gtot;
    int64_t gblk0;             // first analysis block of this product
    const unsigned long long* segtot;  // [NSEG] ... and every segment's total over all products
    int32_t* unit_row;         // local row within the product
    int32_t* unit_tile;
    int32_t* unit_prob;        // product of the unit
    int64_t* stg_size;         // [U+1] staging entries per unit (scanned later)
    int32_t* bin_units;
    // split rows
    unsigned long long* split_counter;
    int32_t* unit_aux;         // split row index of a split unit
    int32_t* split_first;      // first unit of each split row
    int32_t* split_nchunk;     // chunks (units) of each split row
};

struct NumArgs {
    Operands op;               // operands when ops == nullptr (single product)
    const Operands* ops;       // per-product operands (device), or nullptr
    const int32_t* unit_prob;  // product of each unit (with ops)
    const int32_t* unit_row;
    const int32_t* unit_tile;
    const int32_t* units;      // this bin's units
    int64_t nunits;
    const int64_t* out_off;    // staging offsets (STAGE) or final offsets (DIRECT)
    int64_t* cnt;              // per-unit output counts (COUNT, STAGE)
    int32_t* out_col;
    void* out_val;
    // split rows
    const int32_t* unit_aux;
    const int32_t* split_first;
    const int32_t* split_nchunk;
    int64_t nsplit;
    int64_t split_off;         // first split row of this launch (split emission)
    unsigned int* gset;        // [nsplit][DENSE_B_COLS / 32] inserted bits
    void* gval;                // [nsplit][DENSE_B_COLS] accumulator slots
    int64_t max_n;             // the largest column count of the launch's products (sort-key width)
};

// Per-product output binding (device table entry when batched).
struct OutBind {
    int64_t* rowptr;
    int32_t* col;
    void* val;
    int64_t row_off;     // first global row
    int64_t nrows;
    int64_t unit_first;  // first global unit (= unit_base[row_off])
};

struct CompactArgs {
    int64_t U;
    const int64_t* stg_off;    // [U+1]
    const int64_t* out_off;    // [U+1] (scanned counts)
    const int32_t* unit_prob;  // [U] (batched) or nullptr
    const int32_t* stg_col;
    const void* stg_val;
    int val_bytes;
    OutBind one;               // single product
    const OutBind* outs;       // per product (device) or nullptr
};

// ---- launchers (msp_kernels.hip). All enqueue on `s` and return the launch error.
hipError_t launch_validate(const int64_t* rp, const int32_t* ci, int64_t nrows, int64_t ncols, int64_t nnz,
                           unsigned long long* err, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
// Zeroes a[0, na) and b[0, nb) in one launch.
hipError_t launch_zero2(int64_t* a, int64_t na, int64_t* b, int64_t nb, hipStream_t s);
hipError_t launch_analysis(const AnalysisArgs& a, hipStream_t s);
hipError_t launch_units(const UnitArgs& a, int64_t m, hipStream_t s);
// nnz(C_p) of every product of a bound batch into dst[count] (device).
hipError_t launch_batch_nnz(const OutBind* outs, int64_t count, int64_t* dst, hipStream_t s);
// Row-sum chunks of a row of A with nnz entries (one workgroup each).
int64_t rowsum_chunks(int64_t nnz);
// The row sums and the analysis of all products of a batch, one launch each:
// `a` holds the fields common to the products (no pull costs: icost null,
// inner_ratio 0); ops and meta are device tables of count and count + 1
// entries; chunks and blocks are the totals (meta[count].chunk0, .blk0).
hipError_t launch_analysis_batch(const AnalysisArgs& a, const Operands* ops, const ProdMeta* meta, int64_t count,
                                 int64_t chunks, int64_t blocks, hipStream_t s);
// The unit placement of all products of a batch in one launch (`a` without
// its per-product fields).
hipError_t launch_units_batch(const UnitArgs& a, const Operands* ops, const ProdMeta* meta, int64_t count,
                              int64_t blocks, hipStream_t s);
__host__ __device__ inline int flops_bucket(int64_t flops) {
    int b = 0;
    while (b < NBUCKET - 1 && flops >= (int64_t(4) << (2 * b))) ++b;
    return b;
}
// Exclusive scan of n int64 (in may equal out); writes n + 1 outputs.
// `partial` needs scan_partial_elems(n) int64.
int64_t scan_partial_elems(int64_t n);
hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* partial, hipStream_t s);
hipError_t launch_numeric(int semiring, int bin, int mode, const NumArgs& a, hipStream_t s);
// Ordered emission of the split rows' global accumulators (after all numeric kernels).
hipError_t launch_split_emit(int semiring, int mode, const NumArgs& a, hipStream_t s);
// Bytes of the global accumulator per split row.
size_t split_acc_bytes(int semiring);
hipError_t launch_fill_u32(unsigned int* p, int64_t n, hipStream_t s);
hipError_t launch_narrow_cols(const int32_t* in, uint16_t* out, int64_t n, hipStream_t s);
hipError_t launch_compact(const CompactArgs& a, hipStream_t s);
// Row pointers of every product: C_p.rowptr[i] = out_off[unit_base[row_off_p + i]] - out_off[unit_first_p].
// `outs` (device, P entries) or `one` (P == 1); `ent_off` (device, P + 1) = row_off_p + p.
hipError_t launch_rowptr(int64_t P, int64_t total_entries, const int64_t* ent_off, const OutBind* outs,
                         const OutBind& one, const int64_t* unit_base, const int64_t* out_off, hipStream_t s);
// B^T construction: column counts -> scan -> scatter (rows of B^T unsorted).
hipError_t launch_colcount(const int32_t* ci, int64_t nnz, int64_t* cnt, hipStream_t s);
hipError_t launch_transpose_scatter(const int64_t* rp, const int32_t* ci, const void* v, int val_bytes,
                                    int64_t nrows, const int64_t* trp, unsigned long long* cursor,
                                    int32_t* tci, void* tv, hipStream_t s);
// Deterministic (+)-reduction into one value.
int64_t reduce_partial_elems();
// (+)-reduction of n values, or of min(*n_dev, n) when n_dev (device) is given.
hipError_t launch_reduce(int semiring, const void* vals, int64_t n, const int64_t* n_dev, void* partial, void* result,
                         hipStream_t s);

// Reduces the analysis blocks' statistics (part, [ST_COUNT][gtot]): per
// product p (blocks blk_off[p] .. blk_off[p+1], or all gtot blocks when
// count == 1 and blk_off is null) into stats[p * ST_COUNT + x] and, unless it
// is null, host_stats (device-visible page-locked host memory); every
// segment's total over all blocks into segtot; and, in place, every
// segment's counts into exclusive prefix sums over the blocks.
hipError_t launch_segoff(unsigned long long* part, int64_t gtot, const int64_t* blk_off, int64_t count,
                         unsigned long long* stats, unsigned long long* host_stats, unsigned long long* segtot,
                         hipStream_t s);
// deg[r] = min(rp[r + 1] - rp[r], 0xFFFF) for r < nrows.
hipError_t launch_deg16(const int64_t* rp, int64_t nrows, uint16_t* deg, hipStream_t s);
// *host_dst = *src, with host_dst device-visible page-locked host memory.
hipError_t launch_peek(const int64_t* src, int64_t* host_dst, hipStream_t s);

// Records `msg` as the thread's last error (msp_last_error) and returns `st`.
msp_status set_error(msp_status st, const char* msg);

// Device buffers of the iterated applications (betweenness centrality,
// k-truss), taken from the caller's allocator; every buffer still held is
// released, in stream order, when the holder goes out of scope.
struct DevMem {
    const msp_allocator* a;
    hipStream_t s;
    std::vector<void*> ptrs;
    DevMem(const msp_allocator* alloc, hipStream_t st) : a(alloc), s(st) {}
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    msp_status bytes(void** p, size_t n) {
        void* q = a->alloc(a->ctx, n > 0 ? n : 1, (void*)s);
        if (!q) return set_error(MSP_ERR_OUT_OF_MEMORY, "the caller's allocator returned no memory");
        ptrs.push_back(q);
        *p = q;
        return MSP_OK;
    }
    template <class T>
    msp_status get(T** p, int64_t count) {
        return bytes(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(count > 0 ? count : 1));
    }
    void release(const void* p) {
        for (size_t x = 0; x < ptrs.size(); ++x)
            if (ptrs[x] == p) {
                a->release(a->ctx, ptrs[x], (void*)s);
                ptrs.erase(ptrs.begin() + (std::ptrdiff_t)x);
                return;
            }
    }
    ~DevMem() {
        for (size_t x = ptrs.size(); x-- > 0;) a->release(a->ctx, ptrs[x], (void*)s);
    }
};

// Stage timing: between timing_arm(start, stop) and timing_disarm(), the
// launches of this thread record `start` at the beginning of the first kernel
// and `stop` at the end of the last one. timing_disarm() returns whether any
// kernel was launched (otherwise the events were not recorded).
void timing_arm(hipEvent_t start, hipEvent_t stop);
bool timing_disarm();

int out_bytes(int semiring);   // output value width
int in_bytes(int semiring);    // input value width (0: values ignored)

}  // namespace mspk
