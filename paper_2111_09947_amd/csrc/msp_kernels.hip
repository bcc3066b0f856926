// HIP kernels (gfx950, wave64) of the masked SpGEMM hot path C = M .* (A B).
//
// Path (one product):
//   analysis   per row: products flops_i = sum_k nnz(B(k,:)), mask count,
//              exact output bound, accumulator kind and tiling
//   units      expand rows into work units (row or row tile) and place them
//              in per-kind bins
//   scan       prefix sums (unit bases, staging offsets, output offsets)
//   numeric    one kernel per non-empty bin: the accumulator kinds
//   compaction one-phase staging -> final CSR
//   reduce     optional (+)-reduction of the output values
//
// The row-wise push formulation (Section "Push-Based algorithms") streams,
// for row i, every stored A(i,k) and the stanza B(k,:). Here a wavefront
// flattens the stanzas of up to 64 A entries into one product sequence so
// that all 64 lanes read consecutive B entries regardless of stanza lengths;
// a product's B value is loaded only when the mask admits its column (the
// lazy insert of the accumulator interface, Section "Accumulator").
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "msp_device.hpp"
#include "msp_internal.hpp"

namespace mspk {

// Kernel-attached timing. While a stage is armed (timing_arm), every launch
// goes through hipExtLaunchKernel with the stage's events: the first launch
// of the stage records `start` when it begins and every launch records `stop`
// when it ends, so the pair spans exactly the stage's kernels. No marker
// packets are inserted between kernels, unlike separate event records.
namespace {
thread_local hipEvent_t tl_start = nullptr;
thread_local hipEvent_t tl_stop = nullptr;
thread_local bool tl_launched = false;
}  // namespace

void timing_arm(hipEvent_t start, hipEvent_t stop) {
    tl_start = start;
    tl_stop = stop;
    tl_launched = false;
}

bool timing_disarm() {
    const bool launched = tl_launched;
    tl_start = tl_stop = nullptr;
    tl_launched = false;
    return launched;
}

}  // namespace mspk

// Every launch goes through this macro (inside a function returning
// hipError_t). A dispatch that would hold 2^32 work-items or more is refused
// with an error instead of being issued (the dispatch packet's grid size is a
// 32-bit count of work-items).
#define MSP_LAUNCH(K, G, B, SH, S, ...)                                                                    \
    do {                                                                                                 \
        if ((uint64_t)dim3(G).x * (uint64_t)dim3(B).x >= (uint64_t(1) << 32))                           \
            return hipErrorInvalidConfiguration;                                                         \
        if (::mspk::tl_stop) {                                                                           \
            hipExtLaunchKernelGGL(K, G, B, SH, S, ::mspk::tl_launched ? nullptr : ::mspk::tl_start,      \
                                  ::mspk::tl_stop, 0u, __VA_ARGS__);                                      \
            ::mspk::tl_launched = true;                                                                  \
        } else {                                                                                         \
            hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                             \
        }                                                                                                \
    } while (0)

namespace mspk {

int out_bytes(int sr) {
    switch (sr) {
    case MSP_PLUS_TIMES_F64: return 8;
    case MSP_PLUS_PAIR_I64: return 8;
    case MSP_LOR_LAND_BOOL: return 1;
    case MSP_PLUS_TIMES_I32: return 4;
    case MSP_PLUS_TIMES_I64: return 8;
    default: return 0;
    }
}

int in_bytes(int sr) {
    switch (sr) {
    case MSP_PLUS_TIMES_F64: return 8;
    case MSP_PLUS_PAIR_I64: return 0;
    case MSP_LOR_LAND_BOOL: return 1;
    case MSP_PLUS_TIMES_I32: return 4;
    case MSP_PLUS_TIMES_I64: return 8;
    default: return 0;
    }
}

static inline unsigned grid_for(int64_t n, int per_block, int64_t cap = 1 << 20) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------- validation

__global__ void k_validate(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, int64_t nrows,
                           int64_t ncols, int64_t nnz, unsigned long long* err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nrows) return;
    if (i == nrows) {
        if (rp[nrows] != nnz || rp[0] != 0) atomicOr(err, 1ull);
        return;
    }
    const int64_t a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || b > nnz) { atomicOr(err, 1ull); return; }
    int64_t prev = -1;
    for (int64_t p = a; p < b; ++p) {
        const int64_t c = ci[p];
        if (c <= prev || c >= ncols) { atomicOr(err, 1ull); return; }
        prev = c;
    }
}

hipError_t launch_validate(const int64_t* rp, const int32_t* ci, int64_t nrows, int64_t ncols, int64_t nnz,
                           unsigned long long* err, hipStream_t s) {
    MSP_LAUNCH(k_validate, dim3(grid_for(nrows + 1, 256, INT32_MAX)), dim3(256), 0, s, rp, ci, nrows,
                       ncols, nnz, err);
    return hipGetLastError();
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        p[x] = v;
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    MSP_LAUNCH(k_fill_i64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ analysis

constexpr int ANA_T = 256;             // threads per block (analysis and row sums)
constexpr int RS_PER = 8;              // nonzeros per thread in a row-sum block
constexpr int RS_CHUNK = RS_PER * ANA_T;
__device__ __forceinline__ int rs_idx(int e) { return e + (e >> 3); }  // pad: fewer LDS bank conflicts

// Largest r in [0, nrows) with rp[r] <= c (rp[0] = 0 <= c), by a 64-ary
// search of one wave: every round narrows the range 64-fold.
__device__ int64_t row_of(const int64_t* __restrict__ rp, int64_t nrows, int64_t c) {
    int64_t lo = 0, hi = nrows - 1;  // rp[lo] <= c, answer <= hi
    while (lo < hi) {
        const int64_t step = (hi - lo + WAVE) / WAVE;  // >= 1
        const int64_t r = lo + (int64_t)lane() * step;
        const bool ok = r <= hi && rp[r] <= c;
        const int cnt = __popcll(__ballot(ok));        // lane 0 (r = lo) always holds
        const int64_t nlo = lo + (int64_t)(cnt - 1) * step;
        hi = min(hi, nlo + step - 1);
        lo = nlo;
    }
    return lo;
}

// out[r] += sum over the stored entries (r, c) of rp/ci of (grp[c+1] - grp[c])
// for every row r, with `out` zeroed beforehand. Work is split by nonzeros,
// not rows, so a block of very long rows costs the same as any other: block b
// takes the entries [b * RS_CHUNK, (b+1) * RS_CHUNK), gathers the lengths
// into LDS, prefix-sums them, and every row overlapping the range adds its
// overlap (a plain store when the row lies wholly in the range, an atomic add
// when it spans blocks).
// The last product p with key(p) <= x, for a key that does not decrease over
// the count + 1 entries of a batch table, starts at 0 and ends above x:
// the product of a batch launch's workgroup x (empty products are skipped).
template <class K>
__device__ __forceinline__ int64_t product_of(int64_t count, int64_t x, K key) {
    int64_t lo = 0, hi = count;  // key(lo) <= x < key(hi)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (key(mid) <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// BATCHED: one launch for all products of a batch; workgroup b takes chunk
// b - meta[p].chunk0 of product p (the arguments before `ops` are unused).
template <bool BATCHED>
__global__ __launch_bounds__(ANA_T) void k_rowsum(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  int64_t nrows, int64_t nnz, const int64_t* __restrict__ grp,
                                                  const uint16_t* __restrict__ gdeg, int64_t* __restrict__ out,
                                                  const Operands* ops, const ProdMeta* meta, int64_t count) {
    __shared__ int64_t lds[RS_CHUNK + RS_CHUNK / 8];
    __shared__ int64_t tmp[ANA_T / WAVE];
    __shared__ int64_t rows[2];
    const int tid = threadIdx.x;
    int64_t chunk = blockIdx.x;
    if constexpr (BATCHED) {
        const int64_t p = product_of(count, chunk, [&](int64_t q) { return meta[q].chunk0; });
        const Operands& o = ops[p];
        rp = o.Arp;
        ci = o.Aci;
        nrows = o.m;
        grp = o.Brp;
        nnz = meta[p].a_nnz;
        gdeg = meta[p].bdeg;
        out += meta[p].row_off;
        chunk -= meta[p].chunk0;
    }
    const int64_t c0 = chunk * RS_CHUNK;
    const int64_t c1 = min(c0 + (int64_t)RS_CHUNK, nnz);
    const int w = tid / WAVE;
    if (w < 2) {  // wave 0 finds the row of the first entry, wave 1 that of the last
        const int64_t r = row_of(rp, nrows, w == 0 ? c0 : c1 - 1);
        if (lane() == 0) rows[w] = r;
    }
    int32_t col[RS_PER];
#pragma unroll
    for (int x = 0; x < RS_PER; ++x) {
        const int64_t p = c0 + tid + x * ANA_T;
        col[x] = p < c1 ? ci[p] : -1;
    }
    int64_t gv[RS_PER];
    if (gdeg) {  // 2-byte lengths (a quarter of the row pointers' footprint in cache); 0xFFFF: look it up
#pragma unroll
        for (int x = 0; x < RS_PER; ++x) gv[x] = col[x] >= 0 ? (int64_t)gdeg[col[x]] : 0;
#pragma unroll
        for (int x = 0; x < RS_PER; ++x)
            if (gv[x] == 0xFFFF) gv[x] = grp[col[x] + 1] - grp[col[x]];
    } else {
#pragma unroll
        for (int x = 0; x < RS_PER; ++x) gv[x] = col[x] >= 0 ? grp[col[x] + 1] - grp[col[x]] : 0;
    }
#pragma unroll
    for (int x = 0; x < RS_PER; ++x) lds[rs_idx(tid + x * ANA_T)] = gv[x];
    __syncthreads();
    int64_t loc[RS_PER];
    int64_t run = 0;
#pragma unroll
    for (int j = 0; j < RS_PER; ++j) {
        run += lds[rs_idx(tid * RS_PER + j)];
        loc[j] = run;
    }
    int64_t tot;
    const int64_t off = block_excl_scan<ANA_T / WAVE>(run, tmp, tot);
#pragma unroll
    for (int j = 0; j < RS_PER; ++j) lds[rs_idx(tid * RS_PER + j)] = loc[j] + off;  // inclusive prefix
    __syncthreads();
    const int64_t ra = rows[0], rb = rows[1];
    for (int64_t r = ra + tid; r <= rb; r += ANA_T) {
        const int64_t rs = rp[r], re = rp[r + 1];
        const int64_t a = max(rs, c0), b = min(re, c1);
        if (a >= b) continue;
        const int64_t v = lds[rs_idx((int)(b - c0 - 1))] - (a > c0 ? lds[rs_idx((int)(a - c0 - 1))] : 0);
        if (rs >= c0 && re <= c1) out[r] = v;
        else atomicAdd(reinterpret_cast<unsigned long long*>(&out[r]), (unsigned long long)v);
    }
}

__device__ __forceinline__ int64_t cdiv(int64_t x, int64_t y) { return (x + y - 1) / y; }

// Accumulator kind and tiling of one row (auto or forced). alen = nnz(A(i,:)).
__device__ void classify(int64_t mnnz, int64_t flops, int64_t alen, int64_t n, int comp, int force, int inner_ratio,
                        int maskidx_max, int64_t block_flops, int64_t split_flops, int64_t heap_flops,
                        int64_t icost, const int8_t* table, int& bin, int64_t& tiles) {
    // the heap holds one iterator per entry of A's row; other rows take the automatic choice
    const bool heap_fits = alen <= HEAP_CAP && flops <= HEAP_MAX_FLOPS;
    // a light row with a short normal mask row fits eight lanes of a wave (automatic choice only)
    const bool pack_fits = !comp && mnnz <= PACK_MASK && flops <= PACK_FLOPS && alen <= PACK_ALEN;
    bool pack = false;
    int kind = force == MSP_KIND_HEAP && !heap_fits ? (int)MSP_KIND_AUTO : force;
    const bool forced = kind != MSP_KIND_AUTO;  // a forced kind keeps its own kernels
    // a tuned kind for the row's class (products bucket x mask-length bucket), where it fits the row
    if (kind == MSP_KIND_AUTO && table) {
        const int t = table[flops_bucket(flops) * NBUCKET + flops_bucket(mnnz)];
        const bool fits = t >= 0 && t <= MSP_KIND_HEAP && (!comp || t == MSP_KIND_DENSE || t == MSP_KIND_HEAP) &&
                          (t != MSP_KIND_HEAP || heap_fits);
        if (fits) kind = t;
    }
    const bool chosen = forced || kind != MSP_KIND_AUTO;  // forced or tabled
    // Auto: light rows with a short normal mask row take eight lanes each in the packed
    // mask-indexed kernel. Other very light rows are merged one row per lane (a wave-wide kind
    // would leave most of its lanes idle on them), and so are somewhat heavier rows whose mask
    // row is much longer than their product count (the other kinds spend time per mask entry).
    // Matrices of at most 512 columns keep the one-wave dense tile. Under a complemented mask
    // light rows of a wider one go to the heap. Rows of one wider than a 4096-column tile, which
    // the dense kind would restream once per tile, are expanded and sorted when they have at most
    // ESC_MAX products, and otherwise go to the heap where they fit it.
    if (kind == MSP_KIND_AUTO && heap_fits && heap_flops > 0 && n > DENSE_W_COLS && !pack_fits) {
        const bool light = flops <= heap_flops;
        if (comp ? (light || (n > DENSE_B_COLS && flops > ESC_MAX))
                 : (light || (flops <= HEAP_LONG_MASK_FLOPS * heap_flops && mnnz >= HEAP_LONG_MASK_RATIO * flops)))
            kind = MSP_KIND_HEAP;
    }
    if (comp && kind != MSP_KIND_HEAP) kind = MSP_KIND_DENSE;
    const bool heavy = flops > block_flops;
    if (kind == MSP_KIND_AUTO) {
        // Every mask-keyed lookup is behind the membership filter, so a light row is looked up
        // by search in the smaller (higher-occupancy) kernel; a heavy row with a mid-size mask
        // has more candidates per lookup round and takes the hash table of a workgroup.
        if (inner_ratio > 0 && icost * (int64_t)inner_ratio < flops) kind = MSP_KIND_INNER;
        else if (n <= DENSE_W_COLS) kind = MSP_KIND_DENSE;
        else if (pack_fits) { kind = MSP_KIND_MASKIDX; pack = true; }
        else if (mnnz <= maskidx_max || (mnnz <= MASKIDX_W_CAP && !heavy)) kind = MSP_KIND_MASKIDX;
        else if (mnnz <= HASH_B_CAP) kind = MSP_KIND_HASH;
        else kind = MSP_KIND_MASKIDX;
    }
    const bool split = split_flops > 0 && flops > split_flops && alen > 1;
    switch (kind) {
    case MSP_KIND_DENSE:
        tiles = 1;
        if (n <= DENSE_B_COLS && split) { bin = BIN_DENSE_SPLIT; tiles = min(cdiv(flops, split_flops), alen); }
        else if (n <= DENSE_W_COLS) bin = flops > DENSE_NARROW_BLOCK_MULT * block_flops ? BIN_DENSE_BN : BIN_DENSE_W;
        else if (comp && !chosen && n > DENSE_B_COLS && flops <= ESC_MAX &&
                 (flops < ESC_WAVE_MAX || cdiv(n, DENSE_B_COLS) >= ESC_BLOCK_MIN_TILES)) {
            bin = BIN_ESC;
            tiles = 1;
        }
        else { bin = BIN_DENSE_B; tiles = cdiv(n, DENSE_B_COLS); }
        break;
    case MSP_KIND_HASH:
        if (mnnz <= HASH_W_CAP && !heavy) { bin = BIN_HASH_W; tiles = 1; }
        else { bin = BIN_HASH_B; tiles = cdiv(mnnz, HASH_B_CAP); }
        break;
    case MSP_KIND_MASKIDX:
        if (pack) { bin = BIN_MASKIDX_P; tiles = 1; }
        else if (mnnz <= MASKIDX_W_CAP && !heavy) { bin = BIN_MASKIDX_W; tiles = 1; }
        else { bin = BIN_MASKIDX_B; tiles = cdiv(mnnz, MASKIDX_B_CAP); }
        break;
    case MSP_KIND_HEAP:
        bin = !comp && mnnz > MASKIDX_W_CAP ? BIN_HEAP_LM : BIN_HEAP_L; tiles = 1;
        break;
    default:
        bin = BIN_INNER_W; tiles = cdiv(mnnz, INNER_CAP);
        break;
    }
}

// Staging entries of tile t of row i: min(admitted columns of the tile, products).
__device__ int64_t unit_staging(const Operands& o, int64_t i, int bin, int64_t t, int64_t tiles, int64_t mnnz,
                                int64_t flops) {
    int64_t adm = 0;
    switch (bin) {
    case BIN_DENSE_W: case BIN_DENSE_BN:
        adm = o.complement ? o.n - mnnz : mnnz;
        break;
    case BIN_DENSE_SPLIT:  // the first chunk emits the whole row
        adm = t == 0 ? (o.complement ? o.n - mnnz : mnnz) : 0;
        break;
    case BIN_DENSE_B: {
        const int64_t c0 = t * DENSE_B_COLS, c1 = min(c0 + (int64_t)DENSE_B_COLS, o.n);
        int64_t mt = mnnz;
        if (tiles > 1) {
            const int64_t p0 = lower_bound_g(o.Mci, o.Mrp[i], o.Mrp[i + 1], c0);
            mt = lower_bound_g(o.Mci, p0, o.Mrp[i + 1], c1) - p0;
        }
        adm = o.complement ? (c1 - c0) - mt : mt;
        break;
    }
    case BIN_HEAP_L: case BIN_HEAP_LM: case BIN_ESC: adm = o.complement ? o.n - mnnz : mnnz; break;
    case BIN_HASH_W: case BIN_MASKIDX_W: case BIN_MASKIDX_P: adm = mnnz; break;
    case BIN_HASH_B: adm = min((int64_t)HASH_B_CAP, mnnz - t * HASH_B_CAP); break;
    case BIN_MASKIDX_B: adm = min((int64_t)MASKIDX_B_CAP, mnnz - t * MASKIDX_B_CAP); break;
    default: adm = min((int64_t)INNER_CAP, mnnz - t * INNER_CAP); break;
    }
    return min(adm, flops);
}

// The rows of one analysis block: rows blk * ANA_T.., then every nblk-th chunk
// of ANA_T rows, classified and counted into the block's statistics sst.
__device__ __forceinline__ void analysis_rows(const AnalysisArgs& a, const Operands& o, int64_t row_off, int64_t blk,
                                              int64_t nblk, const int8_t* table, unsigned long long* sst) {
    for (int64_t r0 = blk * ANA_T; r0 < o.m; r0 += nblk * ANA_T) {
        const int64_t r1 = min(r0 + ANA_T, o.m);
        const int64_t i = r0 + threadIdx.x;
        // products per row (and the pull cost), summed beforehand by k_rowsum
        const int64_t flops = i < r1 ? a.flops[row_off + i] : 0;
        const int64_t icost = (i < r1 && a.icost) ? a.icost[i] : 0;
        int64_t ub = 0, tiles = 0, stg = 0, mnnz = 0;
        int seg = -1;
        if (i < r1) {
            mnnz = o.Mrp[i + 1] - o.Mrp[i];
            const int64_t adm = o.complement ? o.n - mnnz : mnnz;
            ub = min(adm, flops);
            int bin = -1;
            if (ub > 0) {
                classify(mnnz, flops, o.Arp[i + 1] - o.Arp[i], o.n, o.complement, a.force_kind, a.inner_ratio,
                         a.maskidx_max, a.block_flops, a.split_flops, a.heap_flops, icost,
                         table, bin, tiles);
                if (bin == BIN_DENSE_SPLIT) atomicAdd(&sst[ST_SPLITROWS], 1ull);
                if (bin == BIN_HEAP_L && o.complement) atomicAdd(&sst[ST_HEAP_APART], 1ull);
                if (bin == BIN_HEAP_LM && mnnz > MASKIDX_B_CAP) atomicAdd(&sst[ST_HEAPLM_APART], 1ull);
                for (int64_t t = 0; t < tiles; ++t) stg += unit_staging(o, i, bin, t, tiles, mnnz, flops);
                seg = bin * NBUCKET + flops_bucket(flops);
            }
            a.tiles[row_off + i] = tiles;
            a.bin[row_off + i] = (int8_t)bin;
        }
        // per-segment unit counts: one LDS atomic per distinct segment per wave
        bool pending = seg >= 0;
        while (true) {
            const uint64_t pm = __ballot(pending);
            if (pm == 0) break;
            const int leader = __builtin_ctzll(pm);
            const int sg = __shfl(seg, leader, WAVE);
            const bool mine = pending && seg == sg;
            const int64_t cnt = wave_sum(mine ? tiles : 0);
            if (lane() == leader) atomicAdd(&sst[ST_BIN0 + sg], (unsigned long long)cnt);
            pending = pending && !mine;
        }
        // sums: wave reductions, then one LDS atomic per wave
        const int64_t v_flops = wave_sum(flops);
        const int64_t v_ub = wave_sum(ub), v_tiles = wave_sum(tiles), v_stg = wave_sum(stg);
        const int64_t v_mnnz = wave_sum(mnnz);
        int64_t v_max = flops;
#pragma unroll
        for (int d = WAVE / 2; d >= 1; d >>= 1) v_max = max(v_max, (int64_t)__shfl_xor(v_max, d, WAVE));
        if (lane() == 0) {
            atomicAdd(&sst[ST_FLOPS], (unsigned long long)v_flops);
            atomicAdd(&sst[ST_UB], (unsigned long long)v_ub);
            atomicAdd(&sst[ST_UNITS], (unsigned long long)v_tiles);
            atomicAdd(&sst[ST_STAGING], (unsigned long long)v_stg);
            atomicAdd(&sst[ST_MNNZ], (unsigned long long)v_mnnz);
            atomicMax(&sst[ST_MAXFLOPS], (unsigned long long)v_max);
        }
    }
}

// Each block walks the chunks of 256 rows blk, blk + nblk, ... of its product
// (nblk = analysis_blocks(m)) and writes its own statistics, so no two blocks
// update one address: k_segoff adds them up. BATCHED: one launch for all
// products of a batch, workgroup g taking block g - meta[p].blk0 of product p.
template <bool BATCHED>
__global__ __launch_bounds__(ANA_T) void k_analysis(AnalysisArgs a, const Operands* ops, const ProdMeta* meta,
                                                    int64_t count) {
    static_assert(ANA_T == ANA_ROWS, "one row per thread and chunk");
    static_assert(MSP_KIND_CLASSES % 4 == 0 && MSP_KIND_CLASSES / 4 <= ANA_T, "the kind table: whole words");
    __shared__ unsigned long long sst[ST_COUNT];
    __shared__ uint32_t table_w[MSP_KIND_CLASSES / 4];
    for (int x = threadIdx.x; x < ST_COUNT; x += ANA_T) sst[x] = 0;
    // the kind table moves to LDS word by word with constant indices: indexing the argument
    // block with a lane-dependent index would copy all of it to per-lane scratch memory
    if (a.has_table) {
#pragma unroll
        for (int x = 0; x < MSP_KIND_CLASSES / 4; ++x) {
            uint32_t w;
            __builtin_memcpy(&w, &a.kind_table[4 * x], 4);
            if (threadIdx.x == x) table_w[x] = w;
        }
    }
    __syncthreads();
    const int8_t* table = a.has_table ? reinterpret_cast<const int8_t*>(table_w) : nullptr;
    int64_t g;  // the block's column of the statistics table
    if constexpr (BATCHED) {
        g = blockIdx.x;
        const int64_t p = product_of(count, g, [&](int64_t q) { return meta[q].blk0; });
        analysis_rows(a, ops[p], meta[p].row_off, g - meta[p].blk0, meta[p + 1].blk0 - meta[p].blk0, table, sst);
    } else {
        g = a.gblk0 + blockIdx.x;
        analysis_rows(a, a.op, a.row_off, blockIdx.x, gridDim.x, table, sst);
    }
    __syncthreads();
    // this block's statistics, every one of them (the buffer is not cleared beforehand)
    for (int x = threadIdx.x; x < ST_COUNT; x += ANA_T) a.part[(int64_t)x * a.gtot + g] = sst[x];
}

// deg[r] = min(rp[r + 1] - rp[r], 0xFFFF)
__global__ void k_deg16(const int64_t* __restrict__ rp, int64_t nrows, uint16_t* __restrict__ deg) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x)
        deg[r] = (uint16_t)min(rp[r + 1] - rp[r], (int64_t)0xFFFF);
}

hipError_t launch_deg16(const int64_t* rp, int64_t nrows, uint16_t* deg, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    MSP_LAUNCH(k_deg16, dim3(grid_for(nrows, 256, 4096)), dim3(256), 0, s, rp, nrows, deg);
    return hipGetLastError();
}



__global__ void k_zero2(int64_t* a, int64_t na, int64_t* b, int64_t nb) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < na + nb; x += (int64_t)gridDim.x * blockDim.x) {
        if (x < na) a[x] = 0;
        else b[x - na] = 0;
    }
}

hipError_t launch_zero2(int64_t* a, int64_t na, int64_t* b, int64_t nb, hipStream_t s) {
    if (na + nb <= 0) return hipSuccess;
    MSP_LAUNCH(k_zero2, dim3(grid_for(na + nb, 256, 4096)), dim3(256), 0, s, a, na, b, nb);
    return hipGetLastError();
}

hipError_t launch_analysis(const AnalysisArgs& a, hipStream_t s) {
    if (a.op.m <= 0) return hipSuccess;
    // products per row: sum over A(i,:) of nnz(B(k,:)); pull cost: sum over M(i,:) of nnz(B(:,j))
    hipError_t e = a.flops_zeroed ? hipSuccess : launch_fill_i64(a.flops + a.row_off, a.op.m, 0, s);
    if (e != hipSuccess) return e;
    const Operands* no_ops = nullptr;
    const ProdMeta* no_meta = nullptr;
    if (a.a_nnz > 0)
        MSP_LAUNCH(k_rowsum<false>, dim3(grid_for(a.a_nnz, RS_CHUNK, INT32_MAX)), dim3(ANA_T), 0, s, a.op.Arp, a.op.Aci,
                   a.op.m, a.a_nnz, a.op.Brp, a.bdeg, a.flops + a.row_off, no_ops, no_meta, (int64_t)0);
    if (a.icost) {
        e = launch_fill_i64(a.icost, a.op.m, 0, s);
        if (e != hipSuccess) return e;
        if (a.m_nnz > 0)
            MSP_LAUNCH(k_rowsum<false>, dim3(grid_for(a.m_nnz, RS_CHUNK, INT32_MAX)), dim3(ANA_T), 0, s, a.op.Mrp,
                       a.op.Mci, a.op.m, a.m_nnz, a.colcnt_rp, (const uint16_t*)nullptr, a.icost, no_ops, no_meta,
                       (int64_t)0);
    }
    MSP_LAUNCH(k_analysis<false>, dim3(analysis_blocks(a.op.m)), dim3(ANA_T), 0, s, a, no_ops, no_meta, (int64_t)0);
    return hipGetLastError();
}

int64_t rowsum_chunks(int64_t nnz) { return nnz > 0 ? (nnz + RS_CHUNK - 1) / RS_CHUNK : 0; }

hipError_t launch_analysis_batch(const AnalysisArgs& a, const Operands* ops, const ProdMeta* meta, int64_t count,
                                 int64_t chunks, int64_t blocks, hipStream_t s) {
    if (a.icost || a.inner_ratio) return hipErrorInvalidValue;  // pull costs: one product at a time
    if (chunks > INT32_MAX || blocks > INT32_MAX) return hipErrorInvalidValue;
    if (chunks > 0)
        MSP_LAUNCH(k_rowsum<true>, dim3((unsigned)chunks), dim3(ANA_T), 0, s, (const int64_t*)nullptr,
                   (const int32_t*)nullptr, (int64_t)0, (int64_t)0, (const int64_t*)nullptr, (const uint16_t*)nullptr,
                   a.flops, ops, meta, count);
    if (blocks > 0) MSP_LAUNCH(k_analysis<true>, dim3((unsigned)blocks), dim3(ANA_T), 0, s, a, ops, meta, count);
    return hipGetLastError();
}

// One block per statistic x over the analysis blocks' values part[x][0, gtot):
// the total (the maximum for ST_MAXFLOPS) of every product's blocks, and for
// a segment count also the total over all blocks and, in place, the
// exclusive prefix sums over the blocks in order (products one after
// another): the first position of each block's units inside the segment.
constexpr int SEG_T = 256;
__global__ __launch_bounds__(SEG_T) void k_segoff(unsigned long long* __restrict__ part, int64_t gtot,
                                                  const int64_t* __restrict__ blk_off, int64_t count,
                                                  unsigned long long* __restrict__ stats,
                                                  unsigned long long* host_stats, unsigned long long* segtot) {
    __shared__ unsigned long long red[SEG_T / WAVE];
    const int x = blockIdx.x;
    unsigned long long* row = part + (int64_t)x * gtot;
    const bool is_max = x == ST_MAXFLOPS;
    const int w = threadIdx.x / WAVE;
    if (count == 1) {  // one product: the whole block adds up its blocks
        unsigned long long v = 0;
        for (int64_t g = threadIdx.x; g < gtot; g += SEG_T) v = is_max ? max(v, row[g]) : v + row[g];
#pragma unroll
        for (int d = WAVE / 2; d >= 1; d >>= 1) {
            const unsigned long long o = __shfl_xor(v, d, WAVE);
            v = is_max ? max(v, o) : v + o;
        }
        if (lane() == 0) red[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int k = 0; k < SEG_T / WAVE; ++k) t = is_max ? max(t, red[k]) : t + red[k];
            stats[x] = t;
            if (host_stats) host_stats[x] = t;
        }
    } else {  // a batch: one wave per product (most products have few blocks)
        for (int64_t p = w; p < count; p += SEG_T / WAVE) {
            const int64_t g0 = blk_off[p], g1 = blk_off[p + 1];
            unsigned long long v = 0;
            for (int64_t g = g0 + lane(); g < g1; g += WAVE) v = is_max ? max(v, row[g]) : v + row[g];
#pragma unroll
            for (int d = WAVE / 2; d >= 1; d >>= 1) {
                const unsigned long long o = __shfl_xor(v, d, WAVE);
                v = is_max ? max(v, o) : v + o;
            }
            if (lane() == 0) {
                stats[p * ST_COUNT + x] = v;
                if (host_stats) host_stats[p * ST_COUNT + x] = v;
            }
        }
    }
    __syncthreads();  // every read of `row` above comes before the prefix below rewrites it
    if (x < ST_BIN0 || x >= ST_BIN0 + NSEG) return;
    // segment counts -> exclusive prefix over all blocks, chunk by chunk
    unsigned long long carry = 0;
    for (int64_t base = 0; base < gtot; base += SEG_T) {
        const int64_t g = base + threadIdx.x;
        const unsigned long long v = g < gtot ? row[g] : 0ull;
        unsigned long long incl = v;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const unsigned long long o = __shfl_up(incl, d, WAVE);
            if (lane() >= d) incl += o;
        }
        if (lane() == WAVE - 1) red[w] = incl;
        __syncthreads();
        unsigned long long before = 0, total = 0;
        for (int k = 0; k < SEG_T / WAVE; ++k) {
            before += k < w ? red[k] : 0ull;
            total += red[k];
        }
        if (g < gtot) row[g] = carry + before + incl - v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) segtot[x - ST_BIN0] = carry;
}

hipError_t launch_segoff(unsigned long long* part, int64_t gtot, const int64_t* blk_off, int64_t count,
                         unsigned long long* stats, unsigned long long* host_stats, unsigned long long* segtot,
                         hipStream_t s) {
    MSP_LAUNCH(k_segoff, dim3(ST_COUNT), dim3(SEG_T), 0, s, part, gtot, blk_off, count, stats, host_stats, segtot);
    return hipGetLastError();
}

// The output count of every product of a batch, nnz(C_p) = rowptr_p[nrows_p],
// gathered into one device array (one copy to the host instead of one per product).
__global__ void k_batch_nnz(const OutBind* __restrict__ outs, int64_t count, int64_t* __restrict__ dst) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += (int64_t)gridDim.x * blockDim.x)
        dst[p] = outs[p].rowptr[outs[p].nrows];
}

hipError_t launch_batch_nnz(const OutBind* outs, int64_t count, int64_t* dst, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    MSP_LAUNCH(k_batch_nnz, dim3(grid_for(count, 256, 1024)), dim3(256), 0, s, outs, count, dst);
    return hipGetLastError();
}

// One int64 from device memory into a device-visible page-locked host word.
__global__ void k_peek(const int64_t* __restrict__ src, int64_t* dst) { *dst = *src; }

hipError_t launch_peek(const int64_t* src, int64_t* host_dst, hipStream_t s) {
    MSP_LAUNCH(k_peek, dim3(1), dim3(1), 0, s, src, host_dst);
    return hipGetLastError();
}

// --------------------------------------------------------------------- units

// Same blocks and row chunks as k_analysis. A block's units of segment s go
// to positions segment start + the block's prefix (from k_segoff) + a rank
// taken with an LDS atomic; the counts match the analysis's, so the ranges
// of the blocks tile every segment exactly. units_rows places the units of
// the rows of analysis block blk (of nblk) of one product (g: the block's
// column of the statistics table).
__device__ __forceinline__ void units_rows(const UnitArgs& a, const Operands& o, int64_t m, int64_t row_off,
                                           int32_t prob, int64_t g, int64_t blk, int64_t nblk) {
    __shared__ unsigned int hist[NSEG];
    __shared__ int64_t sbase[NSEG];
    for (int x = threadIdx.x; x < NSEG; x += blockDim.x) hist[x] = 0;
    if (threadIdx.x < WAVE) {  // segment starts: bins in order, inside a bin the buckets from the heaviest down
        constexpr int PER = (NSEG + WAVE - 1) / WAVE;  // consecutive list positions per lane
        int64_t v[PER];
        int sg[PER];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int x = (int)threadIdx.x * PER + k;  // position in the unit list's segment order
            sg[k] = x < NSEG ? bin_at(x / NBUCKET) * NBUCKET + (NBUCKET - 1 - x % NBUCKET) : -1;
            v[k] = sg[k] >= 0 ? (int64_t)a.segtot[sg[k]] : 0;
            sum += v[k];
        }
        int64_t run = wave_incl_scan(sum) - sum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (sg[k] >= 0) sbase[sg[k]] = run;
            run += v[k];
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < NSEG; x += blockDim.x) sbase[x] += (int64_t)a.part[(int64_t)(ST_BIN0 + x) * a.gtot + g];
    __syncthreads();
    for (int64_t r0 = blk * ANA_ROWS; r0 < m; r0 += nblk * ANA_ROWS) {
        const int64_t i = r0 + threadIdx.x;
        if (i >= m) continue;
        const int64_t gr = row_off + i;
        const int64_t base = a.unit_base[gr];
        const int64_t tiles = a.unit_base[gr + 1] - base;
        if (tiles <= 0) continue;
        const int bin = a.bin[gr];
        const int64_t mnnz = o.Mrp[i + 1] - o.Mrp[i];
        const int64_t flops = a.flops[gr];
        for (int64_t t = 0; t < tiles; ++t) {
            a.unit_row[base + t] = (int32_t)i;
            a.unit_tile[base + t] = (int32_t)t;
            a.unit_prob[base + t] = prob;
            a.stg_size[base + t] = unit_staging(o, i, bin, t, tiles, mnnz, flops);
        }
        const int seg = bin * NBUCKET + flops_bucket(flops);
        const int64_t pos = sbase[seg] + (int64_t)atomicAdd(&hist[seg], (unsigned int)tiles);
        for (int64_t t = 0; t < tiles; ++t) a.bin_units[pos + t] = (int32_t)(base + t);
        if (bin == BIN_DENSE_SPLIT) {
            const int32_t sidx = (int32_t)atomicAdd(a.split_counter, 1ull);
            a.split_first[sidx] = (int32_t)base;
            a.split_nchunk[sidx] = (int32_t)tiles;
            for (int64_t t = 0; t < tiles; ++t) a.unit_aux[base + t] = sidx;
        }
    }
}

// BATCHED: one launch for all products of a batch, workgroup g taking block
// g - meta[p].blk0 of product p (a's op, row_off, prob, gblk0 and m unused).
template <bool BATCHED>
__global__ __launch_bounds__(ANA_ROWS) void k_units(UnitArgs a, int64_t m, const Operands* ops, const ProdMeta* meta,
                                                    int64_t count) {
    if constexpr (BATCHED) {
        const int64_t g = blockIdx.x;
        const int64_t p = product_of(count, g, [&](int64_t q) { return meta[q].blk0; });
        const Operands& o = ops[p];
        units_rows(a, o, o.m, meta[p].row_off, (int32_t)p, g, g - meta[p].blk0, meta[p + 1].blk0 - meta[p].blk0);
    } else {
        units_rows(a, a.op, m, a.row_off, a.prob, a.gblk0 + blockIdx.x, blockIdx.x, gridDim.x);
    }
}

hipError_t launch_units(const UnitArgs& a, int64_t m, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    MSP_LAUNCH(k_units<false>, dim3(analysis_blocks(m)), dim3(ANA_ROWS), 0, s, a, m, (const Operands*)nullptr,
               (const ProdMeta*)nullptr, (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_units_batch(const UnitArgs& a, const Operands* ops, const ProdMeta* meta, int64_t count,
                              int64_t blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    MSP_LAUNCH(k_units<true>, dim3((unsigned)blocks), dim3(ANA_ROWS), 0, s, a, (int64_t)0, ops, meta, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------- scan

constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

int64_t scan_partial_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const int64_t* __restrict__ in, int64_t n,
                                                        int64_t* __restrict__ partial) {
    __shared__ int64_t t[SCAN_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_I; ++j) {
        const int64_t e = base + threadIdx.x + (int64_t)j * SCAN_T;
        if (e < n) s += in[e];
    }
    s = wave_sum(s);
    if (lane() == 0) t[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t v = 0;
        for (int w = 0; w < SCAN_T / WAVE; ++w) v += t[w];
        partial[blockIdx.x] = v;
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_partials(int64_t* partial, int64_t nb) {
    __shared__ int64_t tmp[SCAN_T / WAVE];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
        const int64_t idx = b0 + threadIdx.x;
        const int64_t v = idx < nb ? partial[idx] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<SCAN_T / WAVE>(v, tmp, tot);
        if (idx < nb) partial[idx] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_down(const int64_t* in, int64_t* out, int64_t n,
                                                      const int64_t* __restrict__ partial) {
    __shared__ int64_t tmp[SCAN_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    int64_t v[SCAN_I];
    int64_t run = 0;
#pragma unroll
    for (int j = 0; j < SCAN_I; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        run += v[j];
    }
    int64_t tot;
    const int64_t ex = block_excl_scan<SCAN_T / WAVE>(run, tmp, tot);
    int64_t acc = partial[blockIdx.x] + ex;
#pragma unroll
    for (int j = 0; j < SCAN_I; ++j) {
        if (base + j < n) out[base + j] = acc;
        acc += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1) out[n] = partial[blockIdx.x] + tot;
}

// k_scan_down for up to SCAN_FUSE_TILES tiles, taking the raw tile sums: each
// block adds up the sums of the tiles before it (at most SCAN_FUSE_TILES
// reads), which saves the launch of k_scan_partials.
constexpr int64_t SCAN_FUSE_TILES = 1024;

__global__ __launch_bounds__(SCAN_T) void k_scan_down_fused(const int64_t* in, int64_t* out, int64_t n,
                                                            const int64_t* __restrict__ tile_sum) {
    __shared__ int64_t tmp[SCAN_T / WAVE];
    __shared__ int64_t red[SCAN_T / WAVE];
    int64_t o = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SCAN_T) o += tile_sum[b];
    o = wave_sum(o);
    if (lane() == 0) red[threadIdx.x / WAVE] = o;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    int64_t v[SCAN_I];
    int64_t run = 0;
#pragma unroll
    for (int j = 0; j < SCAN_I; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        run += v[j];
    }
    int64_t tot;
    const int64_t ex = block_excl_scan<SCAN_T / WAVE>(run, tmp, tot);  // its barriers also order `red`
    int64_t off = 0;
#pragma unroll
    for (int w = 0; w < SCAN_T / WAVE; ++w) off += red[w];
    int64_t acc = off + ex;
#pragma unroll
    for (int j = 0; j < SCAN_I; ++j) {
        if (base + j < n) out[base + j] = acc;
        acc += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1) out[n] = off + tot;
}

// A short scan in one workgroup of 1024 threads, one chunk of SCAN1_CHUNK
// entries after another with a running carry: one launch instead of two for
// the small unit lists of small products. Each chunk is read whole before any
// of it is written, so in may equal out.
constexpr int SCAN1_T = 1024, SCAN1_CHUNK = SCAN1_T * SCAN_I;
constexpr int64_t SCAN1_MAX = 4 * (int64_t)SCAN1_CHUNK;

__global__ __launch_bounds__(SCAN1_T) void k_scan_single(const int64_t* in, int64_t* out, int64_t n) {
    __shared__ int64_t tmp[SCAN1_T / WAVE];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += SCAN1_CHUNK) {
        const int64_t base = c0 + (int64_t)threadIdx.x * SCAN_I;
        int64_t v[SCAN_I];
        int64_t run = 0;
#pragma unroll
        for (int j = 0; j < SCAN_I; ++j) {
            v[j] = (base + j < n) ? in[base + j] : 0;
            run += v[j];
        }
        int64_t tot;
        const int64_t ex = block_excl_scan<SCAN1_T / WAVE>(run, tmp, tot);  // every thread has read its entries
        int64_t acc = carry + ex;
#pragma unroll
        for (int j = 0; j < SCAN_I; ++j) {
            if (base + j < n) out[base + j] = acc;
            acc += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* partial, hipStream_t s) {
    if (n <= 0) return launch_fill_i64(out, 1, 0, s);
    if (n <= SCAN1_MAX) {
        MSP_LAUNCH(k_scan_single, dim3(1), dim3(SCAN1_T), 0, s, in, out, n);
        return hipGetLastError();
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    MSP_LAUNCH(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n, partial);
    if (nb <= SCAN_FUSE_TILES) {
        MSP_LAUNCH(k_scan_down_fused, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, (const int64_t*)partial);
        return hipGetLastError();
    }
    MSP_LAUNCH(k_scan_partials, dim3(1), dim3(SCAN_T), 0, s, partial, nb);
    MSP_LAUNCH(k_scan_down, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, (const int64_t*)partial);
    return hipGetLastError();
}

// ------------------------------------------------------- product streaming

// Products per lane per step of the product stream: each lane keeps this
// many independent B loads in flight, a wave covers 64 * STREAM_U products.
// Minimum waves per SIMD the compiler must leave room for (register
// budget) in the multi-wave (block) and one-wave numeric kernels.
#ifndef MSP_MINW_BLOCK
#define MSP_MINW_BLOCK 1
#endif
#ifndef MSP_MINW_WAVE
#define MSP_MINW_WAVE 1
#endif
#ifndef MSP_STREAM_U
#define MSP_STREAM_U 8
#endif
constexpr int STREAM_U = MSP_STREAM_U;

// An int32 in global memory (addresses rebuilt from integers keep their
// address space, so the loads stay global rather than flat).
typedef __attribute__((address_space(1))) const int32_t gint32_t;
typedef __attribute__((address_space(1))) const uint16_t guint16_t;

// B's column indices as the dense kernels read them: int32, or the 16-bit
// copy that an execution makes when B has at most 65536 columns.
template <class CI>
__device__ __forceinline__ const CI* bcols(const Operands& o) {
    static_assert(std::is_same<CI, int32_t>::value || std::is_same<CI, uint16_t>::value, "int32 or uint16 columns");
    if constexpr (std::is_same<CI, uint16_t>::value) return o.Bci16;
    else return o.Bci;
}

// First position p in [lo, hi) with a[p] >= key (a sorted ascending).
template <class CI>
__device__ __forceinline__ int64_t lower_bound_c(const CI* __restrict__ a, int64_t lo, int64_t hi, int64_t key) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// B's values are parallel to its column indices: the value of the product
// whose column index (of CW bytes) sits at byte address cb is at
// Bv + (cb - Bci) / CW * w for values of w bytes. With a per-operand constant
// this is one shift-add.
template <int W, int CW = 4>
struct ValAddr {
    static_assert(W == 8 || W == 4 || W == 1, "value widths 1, 4 or 8");
    static_assert(CW == 4 || CW == 2, "column widths 4 or 2");
    static constexpr int L = (W == 8 ? 3 : W == 4 ? 2 : 0) - (CW == 4 ? 2 : 1);  // log2(W / CW)
    // byte address scaled by W / CW (exact: Bci and cb are CW-byte aligned)
    __device__ static uint64_t scale(uint64_t x) {
        if constexpr (L >= 0) return x << L;
        else return x >> (-L);
    }
    uint64_t d;
    __device__ ValAddr(const void* Bv, const void* Bci) : d((uint64_t)Bv - scale((uint64_t)Bci)) {}
    __device__ uint64_t at(uint64_t cb) const { return scale(cb) + d; }
};

// Per-wave LDS for one batch of up to 64 A entries: for the s-th stanza with
// a nonzero length (in A order), its start in the flattened product
// sequence, the shift from flattened position to B position, and A's value;
// plus the start bitmap of the current window.
template <class T>
struct StanzaLds {
    int64_t start[WAVE];
    uint64_t ptr[WAVE];  // byte address that flattened position 0 would have in B's column indices
    typename T::in_t a[T::needs_values ? WAVE : 1];  // semirings that ignore values keep none
    unsigned long long S[STREAM_U];
};


// Streams every product (k, j) of the A entries [pa0, pa1) of one row: for each stored A(i,k) and each
// stored B(k,j) with lo <= j <= hi (when `window`). The products reach the
// caller one window at a time: f(j, s, cb, act) gets STREAM_U products per
// lane, where for slot u, cb[u] is the byte address of B(k,j)'s column index,
// j[u] the column and s[u] indexes st.a for A(i,k); slots past the last
// product have act[u] == false and meaningless j, s, cb. Handing over a whole window lets the caller
// issue the LDS (and value) reads of all its slots before waiting for any.
// Work split among the nw waves of a unit: without `claim`, every wave walks
// every batch of 64 A entries and wave `wv` takes the windows wv, wv + nw,
// ... of 64 * STREAM_U products of each batch. With `claim` (an LDS counter
// that starts at 0), the waves take whole batches instead, the next free one
// each time, and each walks all windows of its batches: a row with many
// batches then does each batch's loads and window searches once, not once per
// wave. batch_end() runs after the last window of every batch the wave
// walks, while st.a and st.ptr still describe that batch.
//
// Lane-to-stanza mapping of a window: every stanza that starts inside the
// window sets bit (start - window base) of a 64 * STREAM_U-bit map; the
// stanza of the product at offset 64u + lane is then
//   (#stanzas starting before the window)
//   + popcount(map bits 0 .. 64u + lane) - 1.
// The STREAM_U loads of a lane are issued back to back before any of them is
// consumed, so a wave keeps STREAM_U stanza reads outstanding.
template <class T, class CI = int32_t, class F, class E>
__device__ __forceinline__ void stream_products(const Operands& o, int64_t pa0, int64_t pa1, bool window, int32_t lo,
                                                int32_t hi, int wv, int nw, StanzaLds<T>& st, F&& f, E&& batch_end,
                                                int* claim = nullptr) {
    const int ln = lane();
    constexpr int64_t WIN = (int64_t)WAVE * STREAM_U;
    const int w0 = claim ? 0 : wv, ws = claim ? 1 : nw;  // this wave's windows of a batch: w0, w0 + ws, ...
    for (int64_t next = pa0;;) {
        int64_t pb;
        if (claim) {
            const int b = ln == 0 ? atomicAdd(claim, 1) : 0;
            pb = pa0 + (int64_t)__builtin_amdgcn_readfirstlane(b) * WAVE;
        } else {
            pb = next;
            next += WAVE;
        }
        if (pb >= pa1) break;
        const int64_t p = pb + ln;
        int64_t b0 = 0, b1 = 0;
        typename T::in_t a = T::one();
        if (p < pa1) {
            const int32_t k = o.Aci[p];
            b0 = o.Brp[k];
            b1 = o.Brp[k + 1];
            if (T::needs_values) a = T::load(o.Av, p);
            if (window) {
                b0 = lower_bound_c(bcols<CI>(o), b0, b1, lo);
                b1 = lower_bound_c(bcols<CI>(o), b0, b1, (int64_t)hi + 1);
            }
        }
        const int64_t len = b1 - b0;
        const uint64_t nzm = __ballot(len > 0);
        if (nzm == 0) continue;
        const int nz = __popcll(nzm);
        const int64_t incl = wave_incl_scan(len);
        const int64_t total = __shfl(incl, WAVE - 1, WAVE);
        if (len > 0) {
            const int sl = rank_below(nzm);
            st.start[sl] = incl - len;
            st.ptr[sl] = (uint64_t)(bcols<CI>(o) + b0) - sizeof(CI) * (uint64_t)(incl - len);
            if constexpr (T::needs_values) st.a[sl] = a;
        }
        wave_lds_sync();
        const int64_t my_start = ln < nz ? st.start[ln] : INT64_MAX;
        for (int64_t base = (int64_t)w0 * WIN; base < total; base += (int64_t)ws * WIN) {
            const int before = __popcll(__ballot(my_start < base));
            const int64_t rel = my_start - base;
            if (rel >= 0 && rel < WIN) atomicOr(&st.S[rel >> 6], 1ull << (rel & 63));
            wave_lds_sync();
            // the window's start bitmap is uniform: move it to scalar registers
            uint64_t Sw[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                const unsigned long long v = st.S[u];
                // readfirstlane returns int: go through uint32_t so that bit 31 does not sign-extend
                const uint32_t vh = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
                const uint32_t vl = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
                Sw[u] = ((uint64_t)vh << 32) | (uint64_t)vl;
            }
            wave_lds_sync();
            if (ln < STREAM_U) st.S[ln] = 0ull;
            const int lim = (int)min(total - base, WIN);  // products left in this window
            // stanza of the product at window offset 64u + lane:
            //   (#stanzas starting before it) + (#starts at offsets <= 64u + lane) - 1,
            // which lies in [0, nz): stanza 0 starts at position 0
            int sidx[STREAM_U];
            int cum = before - 1;
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                sidx[u] = cum + (int)(Sw[u] & 1ull) + rank_below(Sw[u] >> 1);
                cum += __popcll(Sw[u]);
            }
            // the product at flattened position x of stanza s sits at byte st.ptr[s] + x * sizeof(CI)
            // (slot u adds 64u entries: an immediate offset of the load)
            using gci_t = typename std::conditional<sizeof(CI) == 2, guint16_t, gint32_t>::type;
            const uint64_t pos4 = sizeof(CI) * (uint64_t)(base + ln);
            const gci_t* bp[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) bp[u] = reinterpret_cast<const gci_t*>(st.ptr[sidx[u]] + pos4);
            uint64_t cb[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) cb[u] = (uint64_t)(bp[u] + u * WAVE);
            // a full window (every slot holds a product) and the batch's last, partial one take
            // separate straight-line copies of the window's work
            auto run = [&](auto full) {
                constexpr bool FULL = decltype(full)::value;
                bool act[STREAM_U];
#pragma unroll
                for (int u = 0; u < STREAM_U; ++u) act[u] = FULL || u * WAVE + ln < lim;
                int32_t j[STREAM_U];
#pragma unroll
                for (int u = 0; u < STREAM_U; ++u) j[u] = (FULL || act[u]) ? (int32_t)bp[u][u * WAVE] : 0;
                f(j, sidx, cb, act);
            };
            if (lim == WIN) run(std::integral_constant<bool, true>{});
            else run(std::integral_constant<bool, false>{});
            wave_lds_sync();
        }
        batch_end();
        wave_lds_sync();
    }
}

// A unit of NW > 1 waves claims whole batches when its A row has at least
// this many batches of 64 entries per wave (0: never). Fewer batches than
// that are shared window by window, which balances rows whose products sit
// in a few long rows of B.
#ifndef MSP_BATCH_SPLIT_MIN
#define MSP_BATCH_SPLIT_MIN 2
#endif
template <int NW>
__device__ __forceinline__ int* batch_claim(int* counter, int64_t alen) {
    return (NW > 1 && MSP_BATCH_SPLIT_MIN > 0 && alen >= (int64_t)MSP_BATCH_SPLIT_MIN * NW * WAVE) ? counter
                                                                                                  : nullptr;
}

// Folds the admitted products of one window into the LDS accumulator: slot
// u goes to vals[slot[u]] when slot[u] >= 0 (-1: not admitted). B values are
// loaded only for admitted products; all loads of the window are issued
// before the first LDS update.
template <class T, bool FLAGS, bool COUNT, class CI = int32_t>
__device__ __forceinline__ void window_accumulate(const int* slot, const int* s, const uint64_t* cb,
                                                  const Operands& o, const StanzaLds<T>& st,
                                                  typename T::acc_t* vals, uint8_t* flags) {
    typename T::in_t b[STREAM_U];
    if (!COUNT) {
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) b[u] = T::one();
        if (T::needs_values && o.Bv) {  // one uniform test per window (iso-valued B: all ones)
            const ValAddr<T::vbytes, (int)sizeof(CI)> va(o.Bv, bcols<CI>(o));
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u)
                if (slot[u] >= 0) b[u] = T::load_at(va.at(cb[u]));
        }
    }
#pragma unroll
    for (int u = 0; u < STREAM_U; ++u) {
        if (slot[u] >= 0) {
            if (FLAGS) flags[slot[u]] = 1;
            if constexpr (!COUNT) {
                typename T::in_t av = T::one();
                if constexpr (T::needs_values) av = st.a[s[u]];
                T::lds_add(&vals[slot[u]], T::term(av, b[u]));
            }
        }
    }
}

// Ordered compaction over [0, len) for the NW waves of one unit (unit-local
// thread index ut): calls write(idx, position) for every idx with keep(idx),
// positions in idx order.
template <int NW, class K, class W>
__device__ __forceinline__ int64_t ordered_emit(int len, int64_t* tmp, int ut, K keep, W write) {
    int64_t running = 0;
    for (int base = 0; base < len; base += NW * WAVE) {
        const int idx = base + ut;
        const bool kp = idx < len && keep(idx);
        const uint64_t bm = __ballot(kp);
        int64_t before = 0, total = __popcll(bm);
        if (NW > 1) {
            const int w = ut / WAVE;
            if (lane() == 0) tmp[w] = total;
            __syncthreads();
            total = 0;
#pragma unroll
            for (int x = 0; x < NW; ++x) {
                const int64_t c = tmp[x];
                before += (x < w) ? c : 0;
                total += c;
            }
            __syncthreads();
        }
        if (kp) write(idx, running + before + rank_below(bm));
        running += total;
    }
    return running;
}

// ordered_emit for at most MAXLEN entries with one block barrier instead of
// two per round of NW * 64 entries: every wave ballots all of its rounds
// first (the masks stay in scalar registers) and publishes its per-round
// counts to `cnt` (LDS, MAXLEN / 64 entries); after the one barrier each
// thread adds up the counts before its (round, wave) and writes its entries
// in the same order, with the same coalesced stores, as ordered_emit.
template <int NW, int MAXLEN, class K, class W>
__device__ __forceinline__ int64_t ordered_emit_1b(int len, int32_t* cnt, int ut, K keep, W write) {
    constexpr int UT = NW * WAVE;
    constexpr int MAXR = (MAXLEN + UT - 1) / UT;
    static_assert(NW > 1 && MAXR <= 8, "for block units of at most eight rounds");
    const int w = ut / WAVE;
    uint64_t bm[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        const int idx = r * UT + ut;
        bm[r] = __ballot(idx < len && keep(idx));
        if (lane() == 0) cnt[r * NW + w] = __popcll(bm[r]);
    }
    __syncthreads();
    int64_t base = 0;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        int before = 0, round = 0;
#pragma unroll
        for (int x = 0; x < NW; ++x) {
            const int c = cnt[r * NW + x];
            before += x < w ? c : 0;
            round += c;
        }
        if ((bm[r] >> lane()) & 1ull) write(r * UT + ut, base + before + rank_below(bm[r]));
        base += round;
    }
    return base;
}

// Barrier among the waves that work on one unit: the whole block when a unit
// spans NW > 1 waves, only the wave itself otherwise (several independent
// one-wave units may share a block).
template <int NW>
__device__ __forceinline__ void unit_sync() {
    if (NW > 1) __syncthreads();
    else wave_lds_sync();
}

// ------------------------------------------------- dense-state accumulator
// A column tile [c0, c0 + wt) of row i held densely in LDS: admitted bitmap
// (normal: set from the mask row; complemented: all set, then cleared from
// the mask row), values and (where the value cannot tell) inserted flags.
// Emission scans the tile in column order, so rows come out sorted for both
// mask modes.
template <int SR, int MODE, int NW, int W, int WPB, bool BATCH, class CI = int32_t>
__global__ __launch_bounds__(NW * WPB * WAVE, NW > 1 ? (W <= DENSE_W_COLS && !SRT<SR>::sep_flag ? 5 : MSP_MINW_BLOCK)
                                                    : MSP_MINW_WAVE) void k_dense(NumArgs g) {
    static_assert(NW == 1 || WPB == 1, "a block holds one multi-wave unit or several one-wave units");
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    constexpr bool COUNT = MODE == MODE_COUNT;
    constexpr bool FLAGS = COUNT || T::sep_flag;
    constexpr int NWORDS = W / 32;
    constexpr int UT = NW * WAVE;  // threads per unit
    __shared__ uint32_t allowed_[WPB][NWORDS];
    __shared__ acc_t vals_[WPB][COUNT ? 1 : W];
    __shared__ uint8_t flags_[WPB][FLAGS ? W : 1];
    __shared__ StanzaLds<T> st[WPB * NW];
    __shared__ int64_t tmp[NW];
    // the wave index is the same on every lane: keep it (and what derives from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int gi = wave / NW, wv = wave % NW, ut = threadIdx.x % UT;
    const int64_t uix = (int64_t)blockIdx.x * WPB + gi;
    if (uix >= g.nunits) return;  // only one-wave units can leave early (WPB > 1 implies NW == 1)
    uint32_t* allowed = allowed_[gi];
    acc_t* vals = vals_[gi];
    uint8_t* flags = flags_[gi];
    // the unit is the same for every lane of the wave
    const int u = __builtin_amdgcn_readfirstlane(g.units[uix]);
    const Operands& o = BATCH ? g.ops[__builtin_amdgcn_readfirstlane(g.unit_prob[u])] : g.op;
    const int64_t i = g.unit_row[u];
    // the one-wave-tile bins hold only rows of matrices with n <= DENSE_W_COLS: one tile at column 0
    constexpr bool ONE_TILE = W == DENSE_W_COLS;
    const int64_t c0 = ONE_TILE ? 0 : (int64_t)g.unit_tile[u] * W;
    const int wt = (int)min((int64_t)W, o.n - c0);
    const bool tiled = !ONE_TILE && o.n > W;
    for (int x = ut; x < NWORDS; x += UT) {
        const int lo = x * 32;
        const uint32_t valid = (lo + 32 <= wt) ? 0xFFFFFFFFu : (lo >= wt ? 0u : ((1u << (wt - lo)) - 1u));
        allowed[x] = o.complement ? valid : 0u;
    }
    if (!COUNT) for (int x = ut; x < W; x += UT) vals[x] = T::identity();
    if (FLAGS) for (int x = ut; x < W; x += UT) flags[x] = 0;
    if (lane() < STREAM_U) st[wave].S[lane()] = 0ull;
    unit_sync<NW>();
    int64_t m0 = o.Mrp[i], m1 = o.Mrp[i + 1];
    if (tiled) {
        m0 = lower_bound_g(o.Mci, m0, m1, c0);
        m1 = lower_bound_g(o.Mci, m0, m1, c0 + wt);
    }
    for (int64_t p = m0 + ut; p < m1; p += UT) {
        const int c = o.Mci[p] - (int)c0;
        const uint32_t bit = 1u << (c & 31);
        if (o.complement) atomicAnd(&allowed[c >> 5], ~bit);
        else atomicOr(&allowed[c >> 5], bit);
    }
    unit_sync<NW>();
    StanzaLds<T>& S = st[wave];
    // the waves share every batch's windows: claiming whole batches measured slower with the
    // 512-column tile (the waves' concurrent LDS updates of the same few columns) and no faster
    // with the 4096-column one
    stream_products<T, CI>(o, o.Arp[i], o.Arp[i + 1], tiled, (int32_t)c0, (int32_t)(c0 + wt - 1), wv, NW, S,
                       [&](const int32_t* j, const int* s, const uint64_t* cb, const bool* act) {
                           int c[STREAM_U];
                           uint32_t w[STREAM_U];
#pragma unroll
                           for (int u = 0; u < STREAM_U; ++u) {
                               c[u] = act[u] ? j[u] - (int)c0 : 0;  // column 0 of the tile always exists
                               w[u] = allowed[c[u] >> 5];
                           }
                           // the tile column of an admitted product, -1 otherwise
#pragma unroll
                           for (int u = 0; u < STREAM_U; ++u)
                               c[u] = act[u] && __builtin_amdgcn_ubfe(w[u], (uint32_t)c[u], 1) ? c[u] : -1;
                           window_accumulate<T, FLAGS, COUNT, CI>(c, s, cb, o, S, vals, flags);
                       },
                       [] {});
    unit_sync<NW>();
    const int64_t ob = COUNT ? 0 : g.out_off[u];
    typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
    const int64_t total = ordered_emit<NW>(
        wt, tmp, ut,
        [&](int c) { return FLAGS ? (flags[c] != 0) : T::is_set(vals[c]); },
        [&](int c, int64_t pos) {
            if (!COUNT) {
                g.out_col[ob + pos] = (int32_t)(c0 + c);
                ov[ob + pos] = T::finish(vals[c]);
            }
        });
    if (ut == 0 && MODE != MODE_DIRECT) g.cnt[u] = total;
}

// ------------------------------------------------------------- split rows
// A dense-kind row with very many products is cut into chunks of its A row;
// each chunk (one unit, one 256-thread block) accumulates its products in an
// LDS tile as k_dense does, then merges the tile into the row's accumulator
// in global memory with atomics (inserted bits, and values with the
// semiring's (+)); a second kernel emits every split row in column order.
// Integer semirings stay exact; FP64 sums are reordered (within tolerance).
template <int SR, int MODE, bool BATCH, int LW, class CI = int32_t>
__global__ __launch_bounds__(BLOCK_NW * WAVE, MSP_MINW_BLOCK) void k_dense_split(NumArgs g) {
    // LW: the LDS tile (n <= LW); the global accumulator of a split row keeps DENSE_B_COLS columns
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    constexpr int W = LW;
    constexpr int NW = BLOCK_NW;
    constexpr bool COUNT = MODE == MODE_COUNT;
    constexpr bool FLAGS = COUNT || T::sep_flag;
    constexpr int NWORDS = W / 32;
    constexpr int UT = NW * WAVE;
    __shared__ uint32_t allowed[NWORDS];
    __shared__ acc_t vals[COUNT ? 1 : W];
    __shared__ uint8_t flags[FLAGS ? W : 1];
    __shared__ StanzaLds<T> st[NW];
    __shared__ int claim;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)), ut = threadIdx.x;
    const int u = __builtin_amdgcn_readfirstlane(g.units[blockIdx.x]);
    const Operands& o = BATCH ? g.ops[__builtin_amdgcn_readfirstlane(g.unit_prob[u])] : g.op;
    const int64_t i = g.unit_row[u];
    const int t = g.unit_tile[u];
    const int sidx = g.unit_aux[u];
    const int nchunk = g.split_nchunk[sidx];
    const int wt = (int)o.n;  // <= W: split rows have a single column tile
    for (int x = ut; x < NWORDS; x += UT) {
        const int lo = x * 32;
        const uint32_t valid = (lo + 32 <= wt) ? 0xFFFFFFFFu : (lo >= wt ? 0u : ((1u << (wt - lo)) - 1u));
        allowed[x] = o.complement ? valid : 0u;
    }
    if (!COUNT) for (int x = ut; x < wt; x += UT) vals[x] = T::identity();
    if (FLAGS) for (int x = ut; x < wt; x += UT) flags[x] = 0;
    if (lane() < STREAM_U) st[wv].S[lane()] = 0ull;
    if (ut == 0) claim = 0;
    __syncthreads();
    for (int64_t p = o.Mrp[i] + ut; p < o.Mrp[i + 1]; p += UT) {
        const int c = o.Mci[p];
        const uint32_t bit = 1u << (c & 31);
        if (o.complement) atomicAnd(&allowed[c >> 5], ~bit);
        else atomicOr(&allowed[c >> 5], bit);
    }
    __syncthreads();
    const int64_t ra0 = o.Arp[i], alen = o.Arp[i + 1] - ra0;
    const int64_t chunk = (alen + nchunk - 1) / nchunk;
    const int64_t a0 = ra0 + min((int64_t)t * chunk, alen), a1 = ra0 + min((int64_t)(t + 1) * chunk, alen);
    StanzaLds<T>& S = st[wv];
    stream_products<T, CI>(o, a0, a1, false, 0, 0, wv, NW, S,
                       [&](const int32_t* j, const int* s, const uint64_t* cb, const bool* act) {
                           int c[STREAM_U];
                           uint32_t w[STREAM_U];
#pragma unroll
                           for (int u = 0; u < STREAM_U; ++u) {
                               c[u] = act[u] ? j[u] : 0;
                               w[u] = allowed[c[u] >> 5];
                           }
#pragma unroll
                           for (int u = 0; u < STREAM_U; ++u)
                               c[u] = act[u] && __builtin_amdgcn_ubfe(w[u], (uint32_t)c[u], 1) ? c[u] : -1;
                           window_accumulate<T, FLAGS, COUNT, CI>(c, s, cb, o, S, vals, flags);
                       },
                       [] {}, batch_claim<NW>(&claim, a1 - a0));
    __syncthreads();
    unsigned int* gset = g.gset + (int64_t)sidx * (DENSE_B_COLS / 32);
    acc_t* gval = static_cast<acc_t*>(g.gval) + (int64_t)sidx * DENSE_B_COLS;
    for (int c = ut; c < wt; c += UT) {
        const bool set = FLAGS ? (flags[c] != 0) : T::is_set(vals[c]);
        if (set) {
            atomicOr(&gset[c >> 5], 1u << (c & 31));
            if (!COUNT) T::merge(&gval[c], vals[c]);
        }
    }
    if (ut == 0 && MODE != MODE_DIRECT) g.cnt[u] = 0;  // the row's output is emitted by k_split_emit
}

// One block per split row: ordered emission from the global accumulator
// into the output place of the row's first unit.
template <int SR, int MODE, bool BATCH>
__global__ __launch_bounds__(BLOCK_NW * WAVE) void k_split_emit(NumArgs g) {
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    constexpr int W = DENSE_B_COLS;
    constexpr int NW = BLOCK_NW;
    constexpr bool COUNT = MODE == MODE_COUNT;
    __shared__ int64_t tmp[NW];
    const int64_t sidx = g.split_off + blockIdx.x;
    const int u = g.split_first[sidx];
    const Operands& o = BATCH ? g.ops[g.unit_prob[u]] : g.op;
    const int wt = (int)o.n;
    const unsigned int* gset = g.gset + (int64_t)sidx * (W / 32);
    const acc_t* gval = static_cast<const acc_t*>(g.gval) + (int64_t)sidx * W;
    const int64_t ob = COUNT ? 0 : g.out_off[u];
    typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
    const int64_t total = ordered_emit<NW>(
        wt, tmp, (int)threadIdx.x, [&](int c) { return (gset[c >> 5] >> (c & 31)) & 1u; },
        [&](int c, int64_t pos) {
            if (!COUNT) {
                g.out_col[ob + pos] = c;
                ov[ob + pos] = T::finish(gval[c]);
            }
        });
    if (threadIdx.x == 0 && MODE != MODE_DIRECT) g.cnt[u] = total;
}

// ---------------------------------------------- mask-keyed accumulators
// Accumulator slots indexed by the rank of the column within the row's mask
// chunk (at most CAP mask entries, kept sorted in LDS). The rank comes from
// an open-addressing hash table keyed by column (HASHED; load factor <= 1/2,
// linear probing) or from a branch-free binary search over the sorted keys.
// Emission walks the ranks in order, i.e. the mask's column order.
__device__ __forceinline__ int rank_search(const int32_t* keys, int cnt, int top, int32_t j) {
    int pos = 0;
    for (int step = top; step > 0; step >>= 1) {
        const int np = pos + step;
        if (np <= cnt && keys[np - 1] < j) pos = np;
    }
    return (pos < cnt && keys[pos] == j) ? pos : -1;
}

__device__ __forceinline__ uint32_t hash_slot(int32_t j, int tbits) {
    return ((uint32_t)j * 0x9E3779B1u) >> (32 - tbits);
}

// Bucketed open addressing: buckets of 4 keys (16 bytes, -1 = empty) filled
// in slot order, at most two keys per bucket on average; the mask rank of a
// key sits in a parallel table. One 16-byte LDS read settles a lookup unless
// the home bucket is full without holding the key, in which case the next
// buckets are read (linear probing over buckets).
// All four compares are evaluated, so the bucket is one 16-byte LDS read.
__device__ __forceinline__ int bucket_hit(int4 e, int32_t j) {
    int h = (e.w == j) ? 3 : -1;
    h = (e.z == j) ? 2 : h;
    h = (e.y == j) ? 1 : h;
    h = (e.x == j) ? 0 : h;
    return h;
}

// j must not be -1 (the empty marker); a column below zero never matches.
__device__ __forceinline__ int hash_find(const int4* tkey, const uint16_t* trank, uint32_t bmask, int bbits,
                                         int32_t j) {
    uint32_t b = hash_slot(j, bbits);
    int4 e = tkey[b];
    int h = bucket_hit(e, j);
    while (h < 0 && e.w != -1) {  // full home bucket without the key: rare
        b = (b + 1) & bmask;
        e = tkey[b];
        h = bucket_hit(e, j);
    }
    return h < 0 ? -1 : (int)trank[b * 4 + h];
}

// Most products of a row miss its mask, so a lookup is preceded by a
// membership filter: a bitmap of FILTER_WORDS * 32 bits with bit (j mod
// bits) set for every key. A product that passes (a key, or a rare false
// positive) goes to a per-wave ring of candidates; whenever a wave has 64
// candidates it looks them up together, one per lane, so the lookup runs at
// full lane occupancy instead of once per product. The ring is drained at
// the end of every batch of A entries (candidates refer to that batch's A
// values).
// Search kind, exact-bitmap mode: when the tile's keys span at most
// 32 * FILTER_WORDS columns and at most BMP_SPAN_PER_KEY columns per key, the
// filter words instead hold an exact bitmap of the keys over [first key,
// last key], and a per-word prefix count of the set bits (2-byte counts, in
// the otherwise unused candidate rings) gives a key's rank in O(1):
// rank(j) = prefix[w] + popcount(word w below bit b). A product is then
// tested and, on a hit, folded straight away, with no candidate ring and no
// binary search. That pays where hits are frequent: masks dense within
// their column range (the batch's masks of 10% to 80% density, the hub rows
// of k-truss). Where few products hit (triangle counting: 2% in its light
// rows, 18% in its heavy ones), folding slot by slot issues a wave-wide LDS
// atomic per slot for a few lanes, and the candidate ring, which gathers the
// hits into full rounds, is faster: such rows, and the hash kind, keep the
// filter and the lookups (measured: triangle counting's hash_block 0.397
// against 0.431 ms with the bitmap mode). The one-wave search kernel has no
// bitmap mode at all: its code alone cost triangle counting's light rows 3%.
constexpr uint32_t BMP_SPAN_PER_KEY = 16;
// Hash table size: buckets of four slots, at least (keys >> shift) of them.
// Shift 1 fills at most half of the slots, in half the LDS of shift 0: one
// more workgroup of the 512-key block kernel per CU, which outweighs the
// longer probes.
#ifndef MSP_HASH_BUCKET_SHIFT
#define MSP_HASH_BUCKET_SHIFT 1
#endif

template <int CAP, bool QVAL>
struct MaskKeyCfg {
    static constexpr int FILTER_WORDS = CAP < 1024 ? CAP : 1024;  // <= 1 key per 32 bits up to 1024 keys
    // candidates are appended DRAIN slots at a time before full rounds are looked up, so the
    // ring holds up to 63 waiting + 64 * DRAIN new ones (entries with value positions are larger;
    // the one-wave kernels, CAP <= 256, keep the smaller ring for occupancy)
    static constexpr int DRAIN = QVAL || CAP <= 256 ? 1 : 2;
    static constexpr int QCAP = DRAIN == 1 ? 2 * WAVE : (DRAIN == 2 ? 4 * WAVE : 8 * WAVE);
    static_assert(WAVE - 1 + WAVE * DRAIN <= QCAP, "candidate ring too small");
};

template <int SR, int MODE, int NW, int CAP, bool HASHED, int WPB, bool BATCH>
__global__ __launch_bounds__(NW * WPB * WAVE, NW > 1 ? MSP_MINW_BLOCK : MSP_MINW_WAVE) void k_maskkey(NumArgs g) {
    static_assert(NW == 1 || WPB == 1, "a block holds one multi-wave unit or several one-wave units");
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    constexpr bool COUNT = MODE == MODE_COUNT;
    constexpr bool FLAGS = COUNT || T::sep_flag;
    constexpr bool QVAL = !COUNT && T::needs_values;  // candidates carry the positions of their values
    constexpr int HSHIFT = MSP_HASH_BUCKET_SHIFT;      // buckets >= keys >> HSHIFT
    static_assert(HSHIFT >= 0 && HSHIFT <= 1, "at most two keys per bucket of four slots");
    constexpr int NBK = HASHED ? CAP >> HSHIFT : 1;   // buckets (4 slots each)
    constexpr int UT = NW * WAVE;
    constexpr int FW = MaskKeyCfg<CAP, QVAL>::FILTER_WORDS;
    constexpr int FW_BITS = __builtin_ctz(FW);
    static_assert((FW & (FW - 1)) == 0, "filter words: a power of two");
    constexpr int QCAP = MaskKeyCfg<CAP, QVAL>::QCAP;
    constexpr int DRAIN = MaskKeyCfg<CAP, QVAL>::DRAIN;
    static_assert(STREAM_U % DRAIN == 0, "slots per window: a multiple of the drain group");
    __shared__ int32_t keys_[WPB][CAP];
    __shared__ int4 tkey_[WPB][NBK];
    __shared__ uint16_t trank_[WPB][4 * NBK];
    __shared__ acc_t vals_[WPB][COUNT ? 1 : CAP];
    __shared__ uint8_t flags_[WPB][FLAGS ? CAP : 1];
    __shared__ uint32_t filt_[WPB][FW];
    __shared__ int32_t qj_[WPB * NW][QCAP + WAVE];
    __shared__ uint64_t qq_[QVAL ? WPB * NW : 1][QVAL ? QCAP + WAVE : 1];  // column byte addresses
    __shared__ uint8_t qs_[QVAL ? WPB * NW : 1][QVAL ? QCAP + WAVE : 1];
    __shared__ StanzaLds<T> st[WPB * NW];
    __shared__ int64_t tmp[NW];
    __shared__ int claim_[WPB];
    // the wave index is the same on every lane: keep it (and what derives from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int gi = wave / NW, wv = wave % NW, ut = threadIdx.x % UT;
    const int64_t uix = (int64_t)blockIdx.x * WPB + gi;
    if (uix >= g.nunits) return;  // only one-wave units can leave early (WPB > 1 implies NW == 1)
    int32_t* keys = keys_[gi];
    int4* tkey = tkey_[gi];
    uint16_t* trank = trank_[gi];
    acc_t* vals = vals_[gi];
    uint8_t* flags = flags_[gi];
    uint32_t* filt = filt_[gi];
    int32_t* qj = qj_[wave];
    uint64_t* qq = qq_[QVAL ? wave : 0];
    uint8_t* qs = qs_[QVAL ? wave : 0];
    // the unit is the same for every lane of the wave
    const int u = __builtin_amdgcn_readfirstlane(g.units[uix]);
    const Operands& o = BATCH ? g.ops[__builtin_amdgcn_readfirstlane(g.unit_prob[u])] : g.op;
    const int64_t i = g.unit_row[u];
    const int64_t r0 = (int64_t)g.unit_tile[u] * CAP;
    const int64_t mrow = o.Mrp[i];
    const int64_t mnnz = o.Mrp[i + 1] - mrow;
    const int cnt = (int)min((int64_t)CAP, mnnz - r0);
    const bool tiled = mnnz > CAP;
    // the tile's column range; an exact bitmap of it may fit the filter words
    const int32_t lo = __builtin_amdgcn_readfirstlane(o.Mci[mrow + r0]);
    const int32_t hi = __builtin_amdgcn_readfirstlane(o.Mci[mrow + r0 + cnt - 1]);
    const uint32_t span = (uint32_t)(hi - lo) + 1u;
    // (the one-wave kernels have tiles of at most 256 keys, whose rows are light: they keep the ring)
    constexpr bool BMP_OK = !HASHED && CAP > 256;
    const bool bmp = BMP_OK && span <= 32u * (uint32_t)FW && span <= BMP_SPAN_PER_KEY * (uint32_t)cnt;
    static_assert(2 * FW <= 4 * NW * (QCAP + WAVE), "the prefix counts fit the unit's candidate rings");
    uint16_t* pre = reinterpret_cast<uint16_t*>(qj_[gi * NW]);  // the unit's rings, contiguous
    for (int x = ut; x < cnt; x += UT) {
        keys[x] = o.Mci[mrow + r0 + x];
        if (!COUNT) vals[x] = T::identity();
        if (FLAGS) flags[x] = 0;
    }
    int bbits = 1;
    while ((1 << bbits) < cnt) ++bbits;
    // the hash table's buckets: 2^hbits >= cnt >> HSHIFT, so at most half of the slots fill
    const int hbits = max(1, bbits - HSHIFT);
    const uint32_t bmask = (1u << hbits) - 1u;
    // the filter uses about one word (32 bits) per key: at most 1 bit in 32 set
    const int fwb = min(bbits, FW_BITS);
    const int nbw = (int)((span + 31u) >> 5);  // bitmap words (exact-bitmap mode)
    for (int x = ut; x < (bmp ? nbw : (1 << fwb)); x += UT) filt[x] = 0u;
    if (HASHED)
        for (int x = ut; x <= (int)bmask; x += UT) tkey[x] = make_int4(-1, -1, -1, -1);
    if (lane() < STREAM_U) st[wave].S[lane()] = 0ull;
    if (ut == 0) claim_[gi] = 0;
    unit_sync<NW>();
    for (int x = ut; x < cnt; x += UT) {
        const int32_t key = keys[x];
        if (bmp) {
            const uint32_t d = (uint32_t)(key - lo);
            atomicOr(&filt[d >> 5], 1u << (d & 31));
            continue;
        }
        atomicOr(&filt[(key >> 5) & ((1 << fwb) - 1)], 1u << (key & 31));
        if (HASHED) {
            int32_t* slots = reinterpret_cast<int32_t*>(tkey);
            uint32_t b = hash_slot(key, hbits);
            int sl = 0;
            while (atomicCAS(&slots[b * 4 + sl], -1, key) != -1) {
                if (++sl == 4) { sl = 0; b = (b + 1) & bmask; }
            }
            trank[b * 4 + sl] = (uint16_t)x;
        }
    }
    unit_sync<NW>();
    if (bmp) {  // prefix counts of the bitmap words: each thread takes a run of consecutive words
        const int per = (nbw + UT - 1) / UT;
        const int w0 = min(ut * per, nbw), w1 = min(w0 + per, nbw);
        int64_t c = 0;
        for (int w = w0; w < w1; ++w) c += __popc(filt[w]);
        int64_t total;
        int64_t run = block_excl_scan<NW>(c, tmp, total);
        for (int w = w0; w < w1; ++w) {
            pre[w] = (uint16_t)run;
            run += __popc(filt[w]);
        }
        unit_sync<NW>();
    }
    const int top = 1 << (31 - __clz(cnt));
    StanzaLds<T>& S = st[wave];
    const ValAddr<T::vbytes> va(o.Bv, o.Bci);
    // candidate ring of this wave: entries [qh, qn) (mod QCAP) wait for a lookup; qh, qn are wave-uniform
    uint32_t qh = 0, qn = 0;
    // looks up `count` <= 64 candidates starting at ring entry `base`, one per lane
    auto lookup_round = [&](uint32_t base, int count) {
        const int x = lane();
        const int e = (int)((base + (uint32_t)x) & (QCAP - 1));
        const int32_t jv = x < count ? qj[e] : INT32_MIN;  // an idle lane looks up a column no mask holds
        const int r = HASHED ? hash_find(tkey, trank, bmask, hbits, jv) : rank_search(keys, cnt, top, jv);
        if (r >= 0) {
            if (FLAGS) flags[r] = 1;
            if (!COUNT) {
                typename T::in_t av = T::one(), bv = T::one();
                if constexpr (QVAL) {
                    if (o.Bv) bv = T::load_at(va.at(qq[e]));
                    av = S.a[qs[e]];
                }
                T::lds_add(&vals[r], T::term(av, bv));
            }
        }
    };
    stream_products<T>(
        o, o.Arp[i], o.Arp[i + 1], tiled, lo, hi, wv, NW, S,
        [&](const int32_t* j, const int* s, const uint64_t* cb, const bool* act) {
            if (!HASHED && bmp) {  // exact bitmap: rank by prefix count, fold at once
                int r[STREAM_U];
                uint32_t bw[STREAM_U];
#pragma unroll
                for (int u = 0; u < STREAM_U; ++u) {
                    const uint32_t d = (uint32_t)(j[u] - lo);
                    const bool in = act[u] && d < span;
                    bw[u] = in ? filt[d >> 5] : 0u;
                    r[u] = in && ((bw[u] >> (d & 31)) & 1u) ? (int)(d >> 5) : -1;
                }
#pragma unroll
                for (int u = 0; u < STREAM_U; ++u)
                    if (r[u] >= 0) {
                        const uint32_t d = (uint32_t)(j[u] - lo);
                        r[u] = (int)pre[r[u]] + __popc(bw[u] & ((1u << (d & 31)) - 1u));
                    }
                window_accumulate<T, FLAGS, COUNT>(r, s, cb, o, S, vals, flags);
                return;
            }
            uint32_t w[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) w[u] = filt[__builtin_amdgcn_ubfe((uint32_t)j[u], 5, (uint32_t)fwb)];
            // pass[u] is 0 or 1 (an integer, so that it selects the ring entry arithmetically
            // below instead of through a lane mask)
            uint32_t pass[STREAM_U];
            uint64_t m[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                pass[u] = __builtin_amdgcn_ubfe(w[u], (uint32_t)j[u], 1) & (uint32_t)act[u];
                m[u] = __ballot(pass[u] != 0u);
            }
            // append the window's candidates to the ring, DRAIN slots at a time, and look up every
            // full round of 64; the ring indices are wave-uniform
            uint32_t cum = (uint32_t)__builtin_amdgcn_readfirstlane((int)qn);
            uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane((int)qh);
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                // every lane writes (branch-free): a rejected product to its own spare entry past the ring
                const int ea = (int)((cum + (uint32_t)rank_below(m[u])) & (QCAP - 1));
                const int eb = QCAP + lane();
                const int e = eb + (int)pass[u] * (ea - eb);
                qj[e] = j[u];
                if (QVAL) {
                    qq[e] = cb[u];
                    qs[e] = (uint8_t)s[u];
                }
                cum += (uint32_t)__popcll(m[u]);
                if ((u + 1) % DRAIN == 0 && cum - h >= (uint32_t)WAVE) {
                    wave_lds_sync();
                    do {
                        lookup_round(h, WAVE);
                        h += WAVE;
                    } while (cum - h >= (uint32_t)WAVE);
                    wave_lds_sync();  // the round's reads come before later appends reuse its entries
                }
            }
            qn = cum;
            qh = h;
        },
        [&] {
            if (qn != qh) {
                wave_lds_sync();
                lookup_round(qh, (int)(qn - qh));
                qh = qn;
            }
        },
        batch_claim<NW>(&claim_[gi], o.Arp[i + 1] - o.Arp[i]));
    unit_sync<NW>();
    const int64_t ob = COUNT ? 0 : g.out_off[u];
    typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
    auto keep = [&](int r) { return FLAGS ? (flags[r] != 0) : T::is_set(vals[r]); };
    auto put = [&](int r, int64_t pos) {
        if (!COUNT) {
            g.out_col[ob + pos] = keys[r];
            ov[ob + pos] = T::finish(vals[r]);
        }
    };
    int64_t total;
    if constexpr (NW > 1 && CAP / (NW * WAVE) <= 8) {
        // the unit's candidate rings are free again: they hold the per-round counts
        total = ordered_emit_1b<NW, CAP>(cnt, reinterpret_cast<int32_t*>(qj_[gi * NW]), ut, keep, put);
    } else {
        total = ordered_emit<NW>(cnt, tmp, ut, keep, put);
    }
    if (ut == 0 && MODE != MODE_DIRECT) g.cnt[u] = total;
}

// ----------------------------------------------------------- inner product
// Pull formulation: lane x of the wave owns mask entry (i, j) and computes
// the sparse dot product of A(i,:) with column j of B (row j of B^T) by
// looking up every k of that column in A's row (column indices staged in LDS
// up to ACAP entries, else a binary search in global memory); A's value is
// read only for a match.
template <int SR, int MODE, int CAP, int ACAP, int WPB, bool BATCH>
__global__ __launch_bounds__(WPB * WAVE) void k_inner(NumArgs g) {
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    using in_t = typename T::in_t;
    constexpr bool COUNT = MODE == MODE_COUNT;
    __shared__ int32_t akeys_[WPB][ACAP];
    const int ln = lane();
    const int gi = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int64_t uix = (int64_t)blockIdx.x * WPB + gi;
    if (uix >= g.nunits) return;
    int32_t* akeys = akeys_[gi];
    // the unit is the same for every lane of the wave
    const int u = __builtin_amdgcn_readfirstlane(g.units[uix]);
    const Operands& o = BATCH ? g.ops[__builtin_amdgcn_readfirstlane(g.unit_prob[u])] : g.op;
    const int64_t i = g.unit_row[u];
    const int64_t r0 = (int64_t)g.unit_tile[u] * CAP;
    const int64_t mrow = o.Mrp[i];
    const int cnt = (int)min((int64_t)CAP, o.Mrp[i + 1] - mrow - r0);
    const int64_t pa0 = o.Arp[i];
    const int64_t alen = o.Arp[i + 1] - pa0;
    const bool in_lds = alen <= ACAP;
    if (in_lds) {
        for (int x = ln; x < alen; x += WAVE) akeys[x] = o.Aci[pa0 + x];
    }
    wave_lds_sync();
    const int top = in_lds && alen > 0 ? 1 << (31 - __clz((int)alen)) : 0;
    const int64_t ob = COUNT ? 0 : g.out_off[u];
    typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
    int64_t running = 0;
    for (int base = 0; base < cnt; base += WAVE) {
        const int x = base + ln;
        bool set = false;
        acc_t acc = T::identity();
        int32_t j = 0;
        if (x < cnt) {
            j = o.Mci[mrow + r0 + x];
            const int64_t q0 = o.BTrp[j], q1 = o.BTrp[j + 1];
            for (int64_t q = q0; q < q1; ++q) {
                const int32_t k = o.BTci[q];
                int64_t idx;
                if (in_lds) idx = rank_search(akeys, (int)alen, top, k);
                else {
                    const int64_t p = lower_bound_g(o.Aci, pa0, pa0 + alen, k);
                    idx = (p < pa0 + alen && o.Aci[p] == k) ? p - pa0 : -1;
                }
                if (idx >= 0) {
                    set = true;
                    if (!COUNT) {
                        const in_t a = T::needs_values ? T::load(o.Av, pa0 + idx) : T::one();
                        const in_t b = T::needs_values ? T::load(o.BTv, q) : T::one();
                        acc = T::add(acc, T::term(a, b));
                    }
                }
            }
        }
        const uint64_t bm = __ballot(set);
        if (set && !COUNT) {
            const int64_t pos = ob + running + rank_below(bm);
            g.out_col[pos] = j;
            ov[pos] = T::finish(acc);
        }
        running += __popcll(bm);
    }
    if (ln == 0 && MODE != MODE_DIRECT) g.cnt[u] = running;
}

// ---------------------------------------------------------------- heap kind
//
// Masked heap merge (Section "Masked Heap SpGEVM Algorithm"), one lane per
// row. The lane keeps one iterator per entry A(i,k_s) over the row B(k_s,:);
// a binary min-heap of the iterators, stored in LDS, yields the products in
// ascending column order, so products of one column arrive one after another
// and fold into a running value, and the row comes out sorted.
//
// Mask handling: before an iterator enters (or re-enters) the heap it is moved
// past every column the mask does not admit, each column being tested against
// the mask row. Only admitted products are merged, and a product's B value is
// read when it leaves the heap. For a complemented mask the same test is
// negated.
//
// Heap entries are 64-bit keys: column (bits 63..32), slot s of the iterator
// (bits 31..24), remaining entries of its B row (bits 23..0; rows have fewer
// than 2^24 products). Equal columns leave in slot order, which is the order
// of k, so the fold order is the order of the row of A. The end position of
// each iterator's row is kept per slot, so the current position is
// end - remaining.
//
// Latency: a lane walks its row serially, so every dependent memory access
// is paid in full. The columns of the B rows are therefore read HEAP_B at a
// time: windows of HEAP_B positions counted back from the row's end, loaded
// together into an LDS buffer per iterator when the iterator enters the
// window; at the start the first (partial) window of every iterator is
// loaded in one batch. Mask rows of up to HEAP_MREG entries sit in registers
// and are tested by comparisons; longer ones are binary-searched.
//
// LDS per lane: HEAP_CAP x (key 8 B + end 8 B + HEAP_B columns 4 B) = 256 B,
// 16 KiB per one-wave workgroup. Entry e of a lane's arrays sits at
// [e][lane], so lanes at the same depth hit consecutive words. One wave per
// workgroup spreads a small bin over as many CUs as possible: the bin's time
// is bounded below by its slowest lane.
constexpr int HEAP_T = WAVE;
constexpr int HEAP_MREG = 8;
constexpr int HEAP_B = 4;
static_assert((HEAP_B & (HEAP_B - 1)) == 0, "windows are a power of two");

template <int SR, int MODE, bool BATCH>
__global__ __launch_bounds__(HEAP_T) void k_heap(NumArgs g) {
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    using in_t = typename T::in_t;
    constexpr bool COUNT = MODE == MODE_COUNT;
    __shared__ unsigned long long hkey[HEAP_CAP][HEAP_T];
    __shared__ int64_t hend[HEAP_CAP][HEAP_T];
    __shared__ int32_t hcol[HEAP_CAP * HEAP_B][HEAP_T];
    const int t = threadIdx.x;
    const int64_t uix = (int64_t)blockIdx.x * HEAP_T + t;
    if (uix >= g.nunits) return;  // lanes are independent: no wave-wide operation follows
    const int u = g.units[uix];
    const Operands& o = BATCH ? g.ops[g.unit_prob[u]] : g.op;
    const int32_t* __restrict__ Aci = o.Aci;
    const int64_t* __restrict__ Brp = o.Brp;
    const int32_t* __restrict__ Bci = o.Bci;
    const int32_t* __restrict__ Mci = o.Mci;
    const void* Av = o.Av;
    const void* Bv = o.Bv;
    const bool comp = o.complement != 0;
    const int64_t i = g.unit_row[u];
    const int64_t pa0 = o.Arp[i];
    const int alen = (int)(o.Arp[i + 1] - pa0);  // <= HEAP_CAP by classification
    const int64_t m0 = o.Mrp[i], m1 = o.Mrp[i + 1];
    const bool mreg = m1 - m0 <= HEAP_MREG;
    int32_t mk[HEAP_MREG];
#pragma unroll
    for (int x = 0; x < HEAP_MREG; ++x) mk[x] = mreg && m0 + x < m1 ? Mci[m0 + x] : -1;
    auto admitted = [&](int32_t col) -> bool {
        bool f = false;
        if (mreg) {
#pragma unroll
            for (int x = 0; x < HEAP_MREG; ++x) f |= mk[x] == col;
        } else {
            const int64_t q = lower_bound_g(Mci, m0, m1, col);
            f = q < m1 && Mci[q] == col;
        }
        return f != comp;
    };
    // column at position p of slot s's row (ending at e): from the buffer, or, at the first
    // position of a window, by loading the whole window (it lies inside the row)
    auto col_at = [&](int s, int64_t p, int64_t e) -> int32_t {
        const int idx = (int)((e - p - 1) & (HEAP_B - 1));
        if (idx == HEAP_B - 1) {
            int32_t c[HEAP_B];
#pragma unroll
            for (int x = 0; x < HEAP_B; ++x) c[x] = Bci[p + x];
#pragma unroll
            for (int x = 1; x < HEAP_B; ++x) hcol[s * HEAP_B + HEAP_B - 1 - x][t] = c[x];
            return c[0];
        }
        return hcol[s * HEAP_B + idx][t];
    };
    // first position in [p, e) whose column the mask admits (e if none); its column in `col`
    auto next_admitted = [&](int s, int64_t p, int64_t e, int32_t& col) -> int64_t {
        for (; p < e; ++p) {
            col = col_at(s, p, e);
            if (admitted(col)) break;
        }
        return p;
    };
    auto make_key = [](int32_t col, int s, int64_t rem) -> unsigned long long {
        return ((unsigned long long)(uint32_t)col << 32) | ((unsigned long long)s << 24) | (unsigned long long)rem;
    };
    // the iterators' rows and first windows, each level loaded in one batch
    int32_t ks[HEAP_CAP];
#pragma unroll
    for (int s = 0; s < HEAP_CAP; ++s) ks[s] = s < alen ? Aci[pa0 + s] : 0;
    int64_t bs[HEAP_CAP], be[HEAP_CAP];
#pragma unroll
    for (int s = 0; s < HEAP_CAP; ++s) {
        bs[s] = s < alen ? Brp[ks[s]] : 0;
        be[s] = s < alen ? Brp[ks[s] + 1] : 0;
    }
    int32_t cw[HEAP_CAP][HEAP_B];
#pragma unroll
    for (int s = 0; s < HEAP_CAP; ++s) {
        const int n0 = bs[s] < be[s] ? (int)((be[s] - bs[s] - 1) & (HEAP_B - 1)) + 1 : 0;  // rest of the window
#pragma unroll
        for (int x = 0; x < HEAP_B; ++x) cw[s][x] = x < n0 ? Bci[bs[s] + x] : 0;
#pragma unroll
        for (int x = 1; x < HEAP_B; ++x)
            if (x < n0) hcol[s * HEAP_B + n0 - 1 - x][t] = cw[s][x];
    }
    // build the heap: one iterator per entry of A's row that has an admitted product
    int h = 0;
#pragma unroll
    for (int s = 0; s < HEAP_CAP; ++s) {
        if (s < alen && bs[s] < be[s]) {
            const int64_t e = be[s];
            int32_t col = cw[s][0];
            int64_t p = bs[s];
            if (!admitted(col)) p = next_admitted(s, p + 1, e, col);
            if (p < e) {
                hend[s][t] = e;
                const unsigned long long key = make_key(col, s, e - p);
                int x = h++;
                while (x > 0) {  // sift up
                    const int par = (x - 1) >> 1;
                    const unsigned long long pk = hkey[par][t];
                    if (pk <= key) break;
                    hkey[x][t] = pk;
                    x = par;
                }
                hkey[x][t] = key;
            }
        }
    }
    const int64_t ob = COUNT ? 0 : g.out_off[u];
    typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
    int64_t cnt = 0;
    int32_t prev = -1;
    acc_t acc = T::identity();
    while (h > 0) {
        const unsigned long long top = hkey[0][t];
        const int32_t col = (int32_t)(top >> 32);
        const int s = (int)((top >> 24) & 0xffu);
        const int64_t e = hend[s][t];
        const int64_t p = e - (int64_t)(top & 0xffffffull);
        if (col != prev) {  // a new output column: the previous one is complete
            if (prev >= 0) {
                if (!COUNT) {
                    g.out_col[ob + cnt] = prev;
                    ov[ob + cnt] = T::finish(acc);
                }
                ++cnt;
            }
            prev = col;
            acc = T::identity();
        }
        if (!COUNT) {
            const in_t a = T::needs_values ? T::load(Av, pa0 + s) : T::one();
            const in_t b = T::needs_values ? T::load(Bv, p) : T::one();
            acc = T::add(acc, T::term(a, b));
        }
        // advance the popped iterator; a finished one is replaced by the last entry
        int32_t nc = 0;
        const int64_t np = next_admitted(s, p + 1, e, nc);
        unsigned long long key;
        if (np < e) {
            key = make_key(nc, s, e - np);
        } else {
            if (--h == 0) break;
            key = hkey[h][t];
        }
        int x = 0;
        while (true) {  // sift down from the root
            int c = 2 * x + 1;
            if (c >= h) break;
            unsigned long long ck = hkey[c][t];
            if (c + 1 < h) {
                const unsigned long long ck2 = hkey[c + 1][t];
                if (ck2 < ck) { ck = ck2; ++c; }
            }
            if (key <= ck) break;
            hkey[x][t] = ck;
            x = c;
        }
        hkey[x][t] = key;
    }
    if (prev >= 0) {
        if (!COUNT) {
            g.out_col[ob + cnt] = prev;
            ov[ob + cnt] = T::finish(acc);
        }
        ++cnt;
    }
    if (MODE != MODE_DIRECT) g.cnt[u] = cnt;
}

// ------------------------------------------------------ packed light rows
// Rows of the packed bin (a normal mask row of at most PACK_MASK entries, at
// most PACK_FLOPS products, at most PACK_ALEN entries in the row of A) take a
// group of PACK_G lanes each, PACK_RPW rows to a wave. The row's mask keys
// sit sorted in LDS, padded with INT32_MAX to PACK_MASK entries, and a
// product's rank among them comes from a four-step branch-free binary search
// (the mask-indexed kind). The row's products, numbered in the order of A's
// row and then of each B row, go to the group's lanes round-robin (product p
// to lane p mod PACK_G), PACK_UNR of them in flight per lane; the A entry of
// product p is the last one whose first product is at most p, found by
// walking forward a prefix of the B row lengths kept in LDS. A hit folds
// A's and B's values into the key's slot with an LDS atomic; emission walks
// the keys in order (PACK_MASK / PACK_G per lane). Each wave works alone:
// its groups only synchronize through the wave's own LDS accesses.
constexpr int PACK_RPW = WAVE / PACK_G;  // rows per wave
constexpr int PACK_WPB = 2;              // waves per block
#ifndef MSP_PACK_UNR
#define MSP_PACK_UNR 4
#endif
constexpr int PACK_UNR = MSP_PACK_UNR;   // products in flight per lane
static_assert(PACK_MASK == 16, "the search takes four steps over 16 keys");
static_assert(PACK_G >= 2 && PACK_G <= 16 && (PACK_G & (PACK_G - 1)) == 0 && PACK_MASK % PACK_G == 0 &&
                  PACK_ALEN % PACK_G == 0,
              "keys and A entries are dealt to the group's lanes in whole rounds");

// inclusive prefix sum over the PACK_G lanes of a group
__device__ __forceinline__ int group_incl_scan(int v, int q) {
#pragma unroll
    for (int d = 1; d < PACK_G; d <<= 1) {
        const int y = __shfl_up(v, d, PACK_G);
        if (q >= d) v += y;
    }
    return v;
}

template <int SR, int MODE, bool BATCH>
__global__ __launch_bounds__(PACK_WPB * WAVE) void k_pack(NumArgs g) {
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    constexpr bool COUNT = MODE == MODE_COUNT;
    constexpr bool FLAGS = COUNT || T::sep_flag;
    constexpr int R = PACK_WPB * PACK_RPW;  // rows per block
    constexpr int NT = PACK_ALEN / PACK_G;  // A entries per lane
    __shared__ int32_t keys_[R][PACK_MASK];
    __shared__ acc_t vals_[COUNT ? 1 : R][COUNT ? 1 : PACK_MASK];
    __shared__ uint8_t flags_[FLAGS ? R : 1][FLAGS ? PACK_MASK : 1];
    __shared__ int32_t pre_[R][PACK_ALEN + 1];  // first product of each A entry; pre[alen] = products
    __shared__ int64_t shift_[R][PACK_ALEN];    // B position of the row's product p in entry s: shift[s] + p
    const int ln = lane();
    const int q = ln & (PACK_G - 1);
    const int r = (int)threadIdx.x / PACK_G;
    const int64_t uix = (int64_t)blockIdx.x * R + r;
    const bool live = uix < g.nunits;  // no early exit: the emission takes wave-wide ballots
    int u = 0;
    int64_t i = 0;
    if (live) {
        u = g.units[uix];
        i = g.unit_row[u];
    }
    // the row's operands (the groups of one wave may belong to different products of a batch)
    const int64_t* Arp;
    const int32_t* Aci;
    const void* Av;
    const int64_t* Brp;
    const int32_t* Bci;
    const void* Bv;
    const int64_t* Mrp;
    const int32_t* Mci;
    if constexpr (BATCH) {
        const Operands& o = g.ops[live ? g.unit_prob[u] : 0];
        Arp = o.Arp; Aci = o.Aci; Av = o.Av; Brp = o.Brp; Bci = o.Bci; Bv = o.Bv; Mrp = o.Mrp; Mci = o.Mci;
    } else {
        Arp = g.op.Arp; Aci = g.op.Aci; Av = g.op.Av; Brp = g.op.Brp; Bci = g.op.Bci; Bv = g.op.Bv;
        Mrp = g.op.Mrp; Mci = g.op.Mci;
    }
    int64_t pa0 = 0, m0 = 0;
    int alen = 0, mcnt = 0;  // <= PACK_ALEN and <= PACK_MASK by classification
    if (live) {
        pa0 = Arp[i];
        alen = (int)(Arp[i + 1] - pa0);
        m0 = Mrp[i];
        mcnt = (int)(Mrp[i + 1] - m0);
    }
    int32_t* keys = keys_[r];
    acc_t* vals = vals_[COUNT ? 0 : r];
    uint8_t* flags = flags_[FLAGS ? r : 0];
    int32_t* pre = pre_[r];
    int64_t* shift = shift_[r];
#pragma unroll
    for (int t = 0; t < PACK_MASK / PACK_G; ++t) {
        const int x = q + t * PACK_G;
        keys[x] = x < mcnt ? Mci[m0 + x] : INT32_MAX;
        if (!COUNT) vals[x] = T::identity();
        if (FLAGS) flags[x] = 0;
    }
    // entry e = q + PACK_G * t of A's row: its B row [b0, b0 + len)
    int len[NT];
    int64_t b0[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int e = q + t * PACK_G;
        int32_t k = 0;
        if (e < alen) k = Aci[pa0 + e];
        b0[t] = e < alen ? Brp[k] : 0;
        len[t] = e < alen ? (int)(Brp[k + 1] - b0[t]) : 0;
    }
    int total = 0;  // products of the row (<= PACK_FLOPS)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int incl = group_incl_scan(len[t], q);
        const int e = q + t * PACK_G;
        const int start = total + incl - len[t];
        if (e < alen) {
            pre[e] = start;
            shift[e] = b0[t] - start;
        }
        total += __shfl(incl, PACK_G - 1, PACK_G);
    }
    if (q == 0) pre[alen] = total;
    wave_lds_sync();
    int s = 0;  // A entry of this lane's current product (products only move forward)
    for (int p0 = q; p0 < total; p0 += PACK_G * PACK_UNR) {
        int sx[PACK_UNR];
        int64_t bpos[PACK_UNR];
        int32_t j[PACK_UNR];
#pragma unroll
        for (int x = 0; x < PACK_UNR; ++x) {
            const int p = p0 + x * PACK_G;
            if (p < total)
                while (pre[s + 1] <= p) ++s;
            sx[x] = s;
            bpos[x] = p < total ? shift[s] + p : -1;
        }
#pragma unroll
        for (int x = 0; x < PACK_UNR; ++x) j[x] = bpos[x] >= 0 ? Bci[bpos[x]] : -1;  // -1: below every key
        int rk[PACK_UNR];
#pragma unroll
        for (int x = 0; x < PACK_UNR; ++x) {
            // rank of the first key >= j (at most PACK_MASK - 1); a hit if that key is j
            int pos = keys[7] < j[x] ? 8 : 0;
            pos += keys[pos + 3] < j[x] ? 4 : 0;
            pos += keys[pos + 1] < j[x] ? 2 : 0;
            pos += keys[pos] < j[x] ? 1 : 0;
            rk[x] = keys[pos] == j[x] ? pos : -1;
        }
#pragma unroll
        for (int x = 0; x < PACK_UNR; ++x) {
            if (rk[x] >= 0) {
                if (FLAGS) flags[rk[x]] = 1;
                if (!COUNT) T::lds_add(&vals[rk[x]], T::term(T::load(Av, pa0 + sx[x]), T::load(Bv, bpos[x])));
            }
        }
    }
    wave_lds_sync();
    // emission in key order: round t holds keys t * PACK_G .. t * PACK_G + PACK_G - 1, one per lane
    const uint64_t gm = ((1ull << PACK_G) - 1ull) << (ln & ~(PACK_G - 1));  // this group's lanes
    const uint64_t below = (1ull << ln) - 1ull;
    const int64_t ob = (!COUNT && live) ? g.out_off[u] : 0;
    typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
    int emitted = 0;
#pragma unroll
    for (int t = 0; t < PACK_MASK / PACK_G; ++t) {
        const int x = q + t * PACK_G;
        const bool kp = x < mcnt && (FLAGS ? flags[x] != 0 : T::is_set(vals[x]));
        const uint64_t mb = __ballot(kp) & gm;
        if (!COUNT && kp) {  // kp implies live
            const int64_t pos = ob + emitted + __popcll(mb & below);
            g.out_col[pos] = keys[x];
            ov[pos] = T::finish(vals[x]);
        }
        emitted += __popcll(mb);
    }
    if (MODE != MODE_DIRECT && live && q == 0) g.cnt[u] = emitted;
}

// ----------------------------------- expand, sort, fold (complemented rows)
// One workgroup of NT threads per row of the sorting bin (a complemented mask
// over more than DENSE_B_COLS columns, more than heap_flops and at most CAP
// products; also a small heap bin of rows under 256 products, either mask
// mode), product-driven instead of tile by tile:
//  1. expand: every product of the row goes to LDS as the key
//     (column << SB | its index in the row's product order: A's row, then
//     each B row; SB = 12 in 64-bit keys, log2 CAP in 32-bit ones) and,
//     unless counting, its term a * b; the entries of A are
//     taken NT at a time, and a product finds its entry by a binary search
//     over the chunk's prefix of B row lengths;
//  2. sort the keys with a bitonic network over the next power of two: in
//     registers and lane shuffles in a one-wave workgroup (no barriers), in
//     LDS with a block barrier per stage in a larger one;
//  3. fold: the first key of each column is a candidate; it is kept when the
//     mask admits the column (a binary search in the mask row, staged in LDS
//     when it has at most 4 NT entries), and its value is the fold of
//     its column's terms in key order, which is the order of A's row (the
//     Gustavson order);
//  4. emit the kept columns in order (each thread takes a contiguous run of
//     sorted keys; a block scan gives the positions).
// Work per row is O(flops log^2 flops) in LDS, independent of the width n.
// The bin runs as three launches by product count (heaviest units first in
// the unit list), so that light rows take small workgroups with little LDS
// and many of them fit a CU: a wave for rows under 256 products (4 keys per
// lane), a wave for rows under 1024 (16 keys per lane), four waves with room
// for ESC_MAX.
// units of bucket b have fewer than 4^(b+1) products
static_assert((int64_t(4) << (2 * ESC_LIGHT_FROM_BUCKET)) <= 256 && (int64_t(4) << (2 * ESC_MID_FROM_BUCKET)) <= 1024,
              "the light and middle launches hold 256 and 1024 products");
static_assert(ESC_MAX <= 4096, "product index in 12 bits");
constexpr int esc_mcap(int nt) { return 4 * nt; }  // mask entries staged in LDS

constexpr int ESC_EU = 4;  // expansion: products per lane with their loads in flight together

template <int SR, int MODE, bool BATCH, int NT, int CAP, class KT>
__global__ __launch_bounds__(NT) void k_esc(NumArgs g) {
    using T = SRT<SR>;
    using acc_t = typename T::acc_t;
    using in_t = typename T::in_t;
    constexpr bool COUNT = MODE == MODE_COUNT;
    constexpr int NW = NT / WAVE;
    constexpr int PER = CAP / NT;  // sorted keys per thread at most
    constexpr int MCAP = esc_mcap(NT);
    static_assert(CAP <= 4096 && CAP % NT == 0 && PER <= 32 && (CAP & (CAP - 1)) == 0,
                  "product index in 12 bits; whole rounds per thread; one bit per key of a run");
    static_assert(std::is_same<KT, uint32_t>::value || std::is_same<KT, unsigned long long>::value, "key width");
    // key = column << SB | product index: 64-bit keys keep 12 index bits; 32-bit keys (launched
    // only when every column is below 2^(32 - log2 CAP)) keep log2 CAP
    constexpr int SB = sizeof(KT) == 8 ? 12 : __builtin_ctz(CAP);
    constexpr KT SMASK = (KT(1) << SB) - 1;
    __shared__ KT key_[CAP];
    __shared__ acc_t val_[COUNT ? 1 : CAP];
    __shared__ int32_t off_[NT + 1];
    __shared__ int64_t bpos_[NT];
    __shared__ in_t aval_[T::needs_values ? NT : 1];
    __shared__ int32_t mrow_[MCAP];
    __shared__ int64_t tmp[NW];
    const int t = threadIdx.x;
    const int u = __builtin_amdgcn_readfirstlane(g.units[blockIdx.x]);
    const Operands& o = BATCH ? g.ops[__builtin_amdgcn_readfirstlane(g.unit_prob[u])] : g.op;
    const int64_t i = g.unit_row[u];
    const int64_t pa0 = o.Arp[i], pa1 = o.Arp[i + 1];
    const int64_t m0 = o.Mrp[i], m1 = o.Mrp[i + 1];
    const bool mstaged = m1 - m0 <= MCAP;
    if (mstaged)
        for (int64_t q = m0 + t; q < m1; q += NT) mrow_[q - m0] = o.Mci[q];
    // 1. expand
    int total = 0;  // products so far (<= CAP by classification and launch)
    for (int64_t c0 = pa0; c0 < pa1; c0 += NT) {
        const int64_t p = c0 + t;
        int64_t b0 = 0, len = 0;
        in_t a = T::one();
        if (p < pa1) {
            const int32_t k = o.Aci[p];
            b0 = o.Brp[k];
            len = o.Brp[k + 1] - b0;
            if (T::needs_values) a = T::load(o.Av, p);
        }
        int64_t ctot;
        const int64_t ex = block_excl_scan<NW>(len, tmp, ctot);
        off_[t] = (int)ex;
        if (t == 0) off_[NT] = (int)ctot;
        bpos_[t] = b0;
        if (T::needs_values) aval_[t] = a;
        __syncthreads();
        // ESC_EU products per lane a round: their entries found first, then all their loads issued
        for (int q0 = t; q0 < (int)ctot; q0 += NT * ESC_EU) {
            int lo[ESC_EU];
            int64_t bp[ESC_EU];
#pragma unroll
            for (int x = 0; x < ESC_EU; ++x) {
                const int q = q0 + x * NT;
                lo[x] = 0;
                bp[x] = 0;
                if (q < (int)ctot) {
                    int l = 0, h = NT;  // off_[l] <= q < off_[h]: the last entry starting at or before q
                    while (h - l > 1) {
                        const int mid = (l + h) >> 1;
                        if (off_[mid] <= q) l = mid;
                        else h = mid;
                    }
                    lo[x] = l;
                    bp[x] = bpos_[l] + (q - off_[l]);
                }
            }
            int32_t jc[ESC_EU];
            in_t bv[ESC_EU];
#pragma unroll
            for (int x = 0; x < ESC_EU; ++x) {
                const bool ok = q0 + x * NT < (int)ctot;
                jc[x] = ok ? o.Bci[bp[x]] : 0;
                bv[x] = (!COUNT && ok) ? T::load(o.Bv, bp[x]) : T::one();
            }
#pragma unroll
            for (int x = 0; x < ESC_EU; ++x) {
                const int q = q0 + x * NT;
                if (q < (int)ctot) {
                    const int slot = total + q;
                    key_[slot] = ((KT)(uint32_t)jc[x] << SB) | (KT)slot;
                    if (!COUNT) val_[slot] = T::term(T::needs_values ? aval_[lo[x]] : T::one(), bv[x]);
                }
            }
        }
        total += (int)ctot;
        __syncthreads();  // the chunk's tables are rewritten by the next chunk
    }
    // 2. sort
    int nsort = 1;
    while (nsort < total) nsort <<= 1;
    if constexpr (NT == WAVE) {
        // one wave: the keys in registers, element t * PER + r in register r of lane t; partners
        // closer than PER are in the lane's own registers, farther ones a lane shuffle away
        KT kr[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) kr[r] = t * PER + r < total ? key_[t * PER + r] : ~KT(0);
        for (int k = 2; k <= nsort; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                if (jj >= PER) {
                    const bool lower = (t & (jj / PER)) == 0;
#pragma unroll
                    for (int r = 0; r < PER; ++r) {
                        const KT o = __shfl_xor(kr[r], jj / PER, WAVE);
                        const bool asc = ((t * PER + r) & k) == 0;
                        kr[r] = (lower == asc) ? (kr[r] < o ? kr[r] : o) : (kr[r] < o ? o : kr[r]);
                    }
                } else {
                    // partners in the lane's own registers: one unrolled body per distance, so that
                    // every register index is a constant
#pragma unroll
                    for (int lj = 0; (1 << lj) < PER; ++lj) {
                        if (jj == (1 << lj)) {
#pragma unroll
                            for (int r = 0; r < PER; ++r) {
                                if ((r & (1 << lj)) == 0) {
                                    const int y = r | (1 << lj);
                                    const bool asc = ((t * PER + r) & k) == 0;
                                    const KT a = kr[r], b = kr[y];
                                    const bool sw = (a > b) == asc;
                                    kr[r] = sw ? b : a;
                                    kr[y] = sw ? a : b;
                                }
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < PER; ++r)
            if (t * PER + r < nsort) key_[t * PER + r] = kr[r];
        wave_lds_sync();
    } else {
        for (int x = total + t; x < nsort; x += NT) key_[x] = ~KT(0);
        __syncthreads();
        for (int k = 2; k <= nsort; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int x = t; x < nsort; x += NT) {
                    const int y = x ^ jj;
                    if (y > x) {
                        const KT kx = key_[x], ky = key_[y];
                        if ((kx > ky) == ((x & k) == 0)) {
                            key_[x] = ky;
                            key_[y] = kx;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    // 3. candidates and the mask: thread t takes the sorted keys [e0, e1)
    const int per = (total + NT - 1) / NT;  // <= PER
    const int e0 = min(t * per, total), e1 = min(e0 + per, total);
    uint32_t keepbits = 0;
    int kept = 0;
    int64_t ms = 0;  // the search starts past the previous candidate's position (columns ascend)
    const int64_t mlen = m1 - m0;
    for (int e = e0; e < e1; ++e) {
        const uint32_t col = (uint32_t)(key_[e] >> SB);
        if (e > 0 && (uint32_t)(key_[e - 1] >> SB) == col) continue;  // not the first of its column
        int64_t lo = ms, hi = mlen;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            const int32_t mc = mstaged ? mrow_[mid] : o.Mci[m0 + mid];
            if ((uint32_t)mc < col) lo = mid + 1;
            else hi = mid;
        }
        ms = lo;
        const bool in_mask = lo < mlen && (uint32_t)(mstaged ? mrow_[lo] : o.Mci[m0 + lo]) == col;
        if (in_mask != (o.complement != 0)) {
            keepbits |= 1u << (e - e0);
            ++kept;
        }
    }
    int64_t ktot;
    const int64_t pos0 = block_excl_scan<NW>(kept, tmp, ktot);
    // 4. emit
    if (!COUNT) {
        const int64_t ob = g.out_off[u];
        typename T::out_t* ov = static_cast<typename T::out_t*>(g.out_val);
        int64_t pos = ob + pos0;
        for (int e = e0; e < e1; ++e) {
            if (!((keepbits >> (e - e0)) & 1u)) continue;
            const uint32_t col = (uint32_t)(key_[e] >> SB);
            acc_t acc = T::identity();
            for (int f = e; f < total && (uint32_t)(key_[f] >> SB) == col; ++f)
                acc = T::add(acc, val_[(int)(key_[f] & SMASK)]);
            g.out_col[pos] = (int32_t)col;
            ov[pos] = T::finish(acc);
            ++pos;
        }
    }
    if (t == 0 && MODE != MODE_DIRECT) g.cnt[u] = ktot;
}

#ifndef MSP_HASH_LOOKUP
#define MSP_HASH_LOOKUP 1
#endif
#ifndef MSP_WPB
#define MSP_WPB 1
#endif
constexpr int WPB = MSP_WPB;  // independent one-wave units per block

// A dispatch holds fewer than 2^32 work-items, so a bin with more units than
// this (a workgroup of 256 per unit in the block kinds) runs as several
// launches over consecutive slices of its unit list.
constexpr int64_t NUM_CHUNK = int64_t(1) << 22;

template <int SR, int MODE, bool BATCH>
static hipError_t launch_numeric_one(int bin, const NumArgs& a, hipStream_t s) {
    const dim3 gw((unsigned)((a.nunits + WPB - 1) / WPB)), gb((unsigned)a.nunits);
    const dim3 bw(WPB * WAVE), bb(BLOCK_NW * WAVE);
    switch (bin) {
    case BIN_DENSE_W:
        if (!BATCH && a.op.Bci16) MSP_LAUNCH((k_dense<SR, MODE, 1, DENSE_W_COLS, WPB, BATCH, uint16_t>), gw, bw, 0, s, a);
        else MSP_LAUNCH((k_dense<SR, MODE, 1, DENSE_W_COLS, WPB, BATCH>), gw, bw, 0, s, a);
        break;
    case BIN_DENSE_B:
        MSP_LAUNCH((k_dense<SR, MODE, BLOCK_NW, DENSE_B_COLS, 1, BATCH>), gb, bb, 0, s, a);
        break;
    case BIN_HASH_W:
        MSP_LAUNCH((k_maskkey<SR, MODE, 1, HASH_W_CAP, MSP_HASH_LOOKUP != 0, WPB, BATCH>), gw, bw, 0, s, a);
        break;
    case BIN_HASH_B:
        MSP_LAUNCH((k_maskkey<SR, MODE, BLOCK_NW, HASH_B_CAP, MSP_HASH_LOOKUP != 0, 1, BATCH>), gb, bb, 0, s, a);
        break;
    case BIN_MASKIDX_W:
        MSP_LAUNCH((k_maskkey<SR, MODE, 1, MASKIDX_W_CAP, false, WPB, BATCH>), gw, bw, 0, s, a);
        break;
    case BIN_MASKIDX_B:
        MSP_LAUNCH((k_maskkey<SR, MODE, MASKIDX_B_NW, MASKIDX_B_CAP, false, 1, BATCH>), gb,
                   dim3(MASKIDX_B_NW * WAVE), 0, s, a);
        break;
    case LAUNCH_MASKIDX_B_WIDE:
        MSP_LAUNCH((k_maskkey<SR, MODE, MASKIDX_B_WIDE_NW, MASKIDX_B_CAP, false, 1, BATCH>), gb,
                   dim3(MASKIDX_B_WIDE_NW * WAVE), 0, s, a);
        break;
    case BIN_INNER_W:
        MSP_LAUNCH((k_inner<SR, MODE, INNER_CAP, INNER_ACAP, WPB, BATCH>), gw, bw, 0, s, a);
        break;
    case BIN_DENSE_BN:
        if (!BATCH && a.op.Bci16) MSP_LAUNCH((k_dense<SR, MODE, BLOCK_NW, DENSE_W_COLS, 1, BATCH, uint16_t>), gb, bb, 0, s, a);
        else MSP_LAUNCH((k_dense<SR, MODE, BLOCK_NW, DENSE_W_COLS, 1, BATCH>), gb, bb, 0, s, a);
        break;
    case BIN_DENSE_SPLIT:  // a narrow LDS tile (more blocks per CU) when every column fits it
        if (!BATCH && a.op.n <= DENSE_W_COLS && a.op.Bci16)
            MSP_LAUNCH((k_dense_split<SR, MODE, BATCH, DENSE_W_COLS, uint16_t>), gb, bb, 0, s, a);
        else if (!BATCH && a.op.n <= DENSE_W_COLS)
            MSP_LAUNCH((k_dense_split<SR, MODE, BATCH, DENSE_W_COLS>), gb, bb, 0, s, a);
        else
            MSP_LAUNCH((k_dense_split<SR, MODE, BATCH, DENSE_B_COLS>), gb, bb, 0, s, a);
        break;
    case BIN_HEAP_L: case BIN_HEAP_LM:
        MSP_LAUNCH((k_heap<SR, MODE, BATCH>), dim3((unsigned)((a.nunits + HEAP_T - 1) / HEAP_T)), dim3(HEAP_T), 0,
                   s, a);
        break;
    case BIN_ESC:  // the heaviest units of the sorting bin
        MSP_LAUNCH((k_esc<SR, MODE, BATCH, 4 * WAVE, (int)ESC_MAX, unsigned long long>), gb, dim3(4 * WAVE), 0, s,
                   a);
        break;
    case LAUNCH_ESC_MID:  // 32-bit keys when every column is below 2^22
        if (a.max_n > 0 && a.max_n <= (int64_t(1) << 22))
            MSP_LAUNCH((k_esc<SR, MODE, BATCH, WAVE, 1024, uint32_t>), gb, dim3(WAVE), 0, s, a);
        else
            MSP_LAUNCH((k_esc<SR, MODE, BATCH, WAVE, 1024, unsigned long long>), gb, dim3(WAVE), 0, s, a);
        break;
    case LAUNCH_ESC_LIGHT:  // 32-bit keys when every column is below 2^24
        if (a.max_n > 0 && a.max_n <= (int64_t(1) << 24))
            MSP_LAUNCH((k_esc<SR, MODE, BATCH, WAVE, 256, uint32_t>), gb, dim3(WAVE), 0, s, a);
        else
            MSP_LAUNCH((k_esc<SR, MODE, BATCH, WAVE, 256, unsigned long long>), gb, dim3(WAVE), 0, s, a);
        break;
    case BIN_MASKIDX_P: {
        constexpr int64_t rows = PACK_WPB * PACK_RPW;
        MSP_LAUNCH((k_pack<SR, MODE, BATCH>), dim3((unsigned)((a.nunits + rows - 1) / rows)), dim3(PACK_WPB * WAVE),
                   0, s, a);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SR, int MODE, bool BATCH>
static hipError_t launch_numeric_t(int bin, const NumArgs& a, hipStream_t s) {
    for (int64_t off = 0; off < a.nunits; off += NUM_CHUNK) {
        NumArgs c = a;
        c.units = a.units + off;
        c.nunits = std::min(NUM_CHUNK, a.nunits - off);
        const hipError_t e = launch_numeric_one<SR, MODE, BATCH>(bin, c, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int SR, int MODE>
static hipError_t launch_split_emit_t(const NumArgs& a, hipStream_t s) {
    for (int64_t off = 0; off < a.nsplit; off += NUM_CHUNK) {  // a workgroup per split row
        NumArgs c = a;
        c.split_off = off;
        const dim3 g((unsigned)std::min(NUM_CHUNK, a.nsplit - off));
        if (a.ops) MSP_LAUNCH((k_split_emit<SR, MODE, true>), g, dim3(BLOCK_NW * WAVE), 0, s, c);
        else MSP_LAUNCH((k_split_emit<SR, MODE, false>), g, dim3(BLOCK_NW * WAVE), 0, s, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int SR>
static hipError_t launch_split_emit_sr(int mode, const NumArgs& a, hipStream_t s) {
    switch (mode) {
    case MODE_COUNT: return launch_split_emit_t<SR, MODE_COUNT>(a, s);
    case MODE_STAGE: return launch_split_emit_t<SR, MODE_STAGE>(a, s);
    case MODE_DIRECT: return launch_split_emit_t<SR, MODE_DIRECT>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_split_emit(int semiring, int mode, const NumArgs& a, hipStream_t s) {
    if (a.nsplit <= 0) return hipSuccess;
    if (mode == MODE_COUNT) return launch_split_emit_sr<MSP_PLUS_PAIR_I64>(mode, a, s);
    switch (semiring) {
    case MSP_PLUS_TIMES_F64: return launch_split_emit_sr<MSP_PLUS_TIMES_F64>(mode, a, s);
    case MSP_PLUS_PAIR_I64: return launch_split_emit_sr<MSP_PLUS_PAIR_I64>(mode, a, s);
    case MSP_LOR_LAND_BOOL: return launch_split_emit_sr<MSP_LOR_LAND_BOOL>(mode, a, s);
    case MSP_PLUS_TIMES_I32: return launch_split_emit_sr<MSP_PLUS_TIMES_I32>(mode, a, s);
    case MSP_PLUS_TIMES_I64: return launch_split_emit_sr<MSP_PLUS_TIMES_I64>(mode, a, s);
    default: return hipErrorInvalidValue;
    }
}

size_t split_acc_bytes(int) {
    // inserted bits plus DENSE_B_COLS slots of at most 8 bytes
    return (size_t)DENSE_B_COLS / 32 * 4 + (size_t)DENSE_B_COLS * 8;
}

__global__ void k_fill_u32(unsigned int* p, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        p[x] = 0u;
}

// B's column indices narrowed to 16 bits (B has at most 65536 columns), four
// per thread when the input is 16-byte aligned.
__global__ __launch_bounds__(256) void k_narrow_cols(const int32_t* __restrict__ in, uint16_t* __restrict__ out,
                                                     int64_t n, int vec) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (vec) {
        const int64_t n4 = n / 4;
        for (int64_t q = t0; q < n4; q += stride) {
            const int4 v = reinterpret_cast<const int4*>(in)[q];
            const uint2 w = make_uint2(((uint32_t)v.y << 16) | ((uint32_t)v.x & 0xFFFFu),
                                       ((uint32_t)v.w << 16) | ((uint32_t)v.z & 0xFFFFu));
            reinterpret_cast<uint2*>(out)[q] = w;  // out is 256-byte aligned
        }
        for (int64_t q = n4 * 4 + t0; q < n; q += stride) out[q] = (uint16_t)in[q];
    } else {
        for (int64_t q = t0; q < n; q += stride) out[q] = (uint16_t)in[q];
    }
}

hipError_t launch_narrow_cols(const int32_t* in, uint16_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int vec = ((uintptr_t)in % 16) == 0;
    const int64_t work = vec ? (n + 3) / 4 : n;
    const unsigned grid = (unsigned)std::min<int64_t>((work + 255) / 256, 8192);
    MSP_LAUNCH(k_narrow_cols, dim3(grid), dim3(256), 0, s, in, out, n, vec);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    MSP_LAUNCH(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <int SR>
static hipError_t launch_numeric_sr(int bin, int mode, const NumArgs& a, hipStream_t s) {
    // batches (per-unit operands) run one-phase only
    if (a.ops) return mode == MODE_STAGE ? launch_numeric_t<SR, MODE_STAGE, true>(bin, a, s) : hipErrorInvalidValue;
    switch (mode) {
    case MODE_COUNT: return launch_numeric_t<SR, MODE_COUNT, false>(bin, a, s);
    case MODE_STAGE: return launch_numeric_t<SR, MODE_STAGE, false>(bin, a, s);
    case MODE_DIRECT: return launch_numeric_t<SR, MODE_DIRECT, false>(bin, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_numeric(int semiring, int bin, int mode, const NumArgs& a, hipStream_t s) {
    if (a.nunits <= 0) return hipSuccess;
    if (mode == MODE_COUNT) {
        // symbolic counting does not depend on values: one instantiation per value layout suffices
        switch (semiring) {
        case MSP_PLUS_PAIR_I64: return launch_numeric_sr<MSP_PLUS_PAIR_I64>(bin, mode, a, s);
        default: return launch_numeric_sr<MSP_PLUS_PAIR_I64>(bin, mode, a, s);
        }
    }
    switch (semiring) {
    case MSP_PLUS_TIMES_F64: return launch_numeric_sr<MSP_PLUS_TIMES_F64>(bin, mode, a, s);
    case MSP_PLUS_PAIR_I64: return launch_numeric_sr<MSP_PLUS_PAIR_I64>(bin, mode, a, s);
    case MSP_LOR_LAND_BOOL: return launch_numeric_sr<MSP_LOR_LAND_BOOL>(bin, mode, a, s);
    case MSP_PLUS_TIMES_I32: return launch_numeric_sr<MSP_PLUS_TIMES_I32>(bin, mode, a, s);
    case MSP_PLUS_TIMES_I64: return launch_numeric_sr<MSP_PLUS_TIMES_I64>(bin, mode, a, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- compaction

template <typename V>
__global__ __launch_bounds__(256) void k_compact(CompactArgs a) {
    const int64_t first = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t u = first; u < a.U; u += (int64_t)gridDim.x * 4) {
        const OutBind& ob = a.outs ? a.outs[a.unit_prob[u]] : a.one;
        const int64_t src = a.stg_off[u], n = a.out_off[u + 1] - a.out_off[u];
        const int64_t dst = a.out_off[u] - a.out_off[ob.unit_first];
        const V* sv = static_cast<const V*>(a.stg_val);
        V* dv = static_cast<V*>(ob.val);
        for (int64_t x = lane(); x < n; x += WAVE) {
            ob.col[dst + x] = a.stg_col[src + x];
            dv[dst + x] = sv[src + x];
        }
    }
}

// Single-product compaction, CG consecutive units per wave: the group's
// outputs are contiguous (units are numbered in row order), so the wave
// walks them as one run of coalesced writes; each element finds its unit
// among the group's (scalar) offsets and reads from that unit's staging run.
constexpr int CG = 4;

template <typename V>
__device__ __forceinline__ void compact_group(const CompactArgs& a, int64_t grp);

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename V>
__global__ __launch_bounds__(256) void k_compact_group(CompactArgs a) {
    const int64_t first = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t grp = first; grp * CG < a.U; grp += (int64_t)gridDim.x * 4) compact_group<V>(a, grp);
}

template <typename V>
__device__ __forceinline__ void compact_group(const CompactArgs& a, int64_t grp) {
    const int64_t u0 = grp * CG;
    const int nk = (int)min((int64_t)CG, a.U - u0);
    const int l = lane();
    const int64_t oo = l <= nk ? a.out_off[u0 + l] : 0;
    const int64_t so = l < nk ? a.stg_off[u0 + l] : 0;
    int64_t o[CG + 1], st[CG];
#pragma unroll
    for (int k = 0; k <= CG; ++k) o[k] = readlane64(oo, min(k, nk));
#pragma unroll
    for (int k = 0; k < CG; ++k) st[k] = readlane64(so, min(k, nk - 1));
    const int64_t base = o[0];
    const int64_t total = o[nk] - base;
    const int64_t dst0 = base - a.out_off[a.one.unit_first];
    const V* sv = static_cast<const V*>(a.stg_val);
    V* dv = static_cast<V*>(a.one.val);
    for (int64_t x = l; x < total; x += WAVE) {
        int64_t src = st[0] + x;
#pragma unroll
        for (int k = 1; k < CG; ++k)
            if (k < nk && o[k] - base <= x) src = st[k] + (x - (o[k] - base));
        a.one.col[dst0 + x] = a.stg_col[src];
        dv[dst0 + x] = sv[src];
    }
}

hipError_t launch_compact(const CompactArgs& a, hipStream_t s) {
    if (a.U <= 0) return hipSuccess;
    if (!a.outs) {
        const dim3 g(grid_for(a.U, 4 * CG, int64_t(1) << 20));
        switch (a.val_bytes) {
        case 1: MSP_LAUNCH(k_compact_group<uint8_t>, g, dim3(256), 0, s, a); break;
        case 4: MSP_LAUNCH(k_compact_group<uint32_t>, g, dim3(256), 0, s, a); break;
        case 8: MSP_LAUNCH(k_compact_group<unsigned long long>, g, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const dim3 grid(grid_for(a.U, 4, int64_t(1) << 20));
    switch (a.val_bytes) {
    case 1: MSP_LAUNCH(k_compact<uint8_t>, grid, dim3(256), 0, s, a); break;
    case 4: MSP_LAUNCH(k_compact<uint32_t>, grid, dim3(256), 0, s, a); break;
    case 8: MSP_LAUNCH(k_compact<unsigned long long>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One thread per row pointer entry of every product (nrows_p + 1 entries each).
__global__ void k_rowptr(int64_t P, int64_t total, const int64_t* __restrict__ ent_off, const OutBind* outs,
                         OutBind one, const int64_t* __restrict__ unit_base, const int64_t* __restrict__ out_off) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int64_t p = 0;
    if (outs) {  // product of entry t: last p with ent_off[p] <= t
        int64_t lo = 0, hi = P - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (ent_off[mid] <= t) lo = mid; else hi = mid - 1;
        }
        p = lo;
    }
    const OutBind& ob = outs ? outs[p] : one;
    const int64_t i = t - (outs ? ent_off[p] : 0);
    ob.rowptr[i] = out_off[unit_base[ob.row_off + i]] - out_off[ob.unit_first];
}

hipError_t launch_rowptr(int64_t P, int64_t total_entries, const int64_t* ent_off, const OutBind* outs,
                         const OutBind& one, const int64_t* unit_base, const int64_t* out_off, hipStream_t s) {
    if (total_entries <= 0) return hipSuccess;
    MSP_LAUNCH(k_rowptr, dim3(grid_for(total_entries, 256, INT32_MAX)), dim3(256), 0, s, P, total_entries,
                       ent_off, outs, one, unit_base, out_off);
    return hipGetLastError();
}

// ----------------------------------------------------------------- transpose

__global__ void k_colcount(const int32_t* __restrict__ ci, int64_t nnz, int64_t* cnt) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[ci[p]]), 1ull);
}

hipError_t launch_colcount(const int32_t* ci, int64_t nnz, int64_t* cnt, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    MSP_LAUNCH(k_colcount, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, s, ci, nnz, cnt);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_tscatter(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  const uint8_t* __restrict__ v, int vb, int64_t nrows,
                                                  const int64_t* __restrict__ trp, unsigned long long* cursor,
                                                  int32_t* __restrict__ tci, uint8_t* __restrict__ tv) {
    const int64_t first = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    for (int64_t r = first; r < nrows; r += (int64_t)gridDim.x * 4) {
        for (int64_t p = rp[r] + lane(); p < rp[r + 1]; p += WAVE) {
            const int32_t c = ci[p];
            const int64_t pos = trp[c] + (int64_t)atomicAdd(&cursor[c], 1ull);
            tci[pos] = (int32_t)r;
            for (int b = 0; b < vb; ++b) tv[pos * vb + b] = v[p * vb + b];
        }
    }
}

hipError_t launch_transpose_scatter(const int64_t* rp, const int32_t* ci, const void* v, int val_bytes,
                                    int64_t nrows, const int64_t* trp, unsigned long long* cursor, int32_t* tci,
                                    void* tv, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    MSP_LAUNCH(k_tscatter, dim3(grid_for(nrows, 4, int64_t(1) << 20)), dim3(256), 0, s, rp, ci,
                       static_cast<const uint8_t*>(v), v ? val_bytes : 0, nrows, trp, cursor, tci,
                       static_cast<uint8_t*>(tv));
    return hipGetLastError();
}

// ----------------------------------------------------------------- reduction

constexpr int RED_BLOCKS = 1024, RED_T = 256;
int64_t reduce_partial_elems() { return RED_BLOCKS; }

template <int SR> struct Red;
template <> struct Red<MSP_PLUS_TIMES_F64> {
    using V = double; using A = double;
    __device__ static A from(V v) { return v; }
    __device__ static A op(A x, A y) { return x + y; }
    __device__ static V out(A x) { return x; }
};
template <> struct Red<MSP_PLUS_PAIR_I64> {
    using V = int64_t; using A = unsigned long long;
    __device__ static A from(V v) { return (A)v; }
    __device__ static A op(A x, A y) { return x + y; }
    __device__ static V out(A x) { return (V)x; }
};
template <> struct Red<MSP_PLUS_TIMES_I64> : Red<MSP_PLUS_PAIR_I64> {};
template <> struct Red<MSP_PLUS_TIMES_I32> {
    using V = int32_t; using A = unsigned long long;
    __device__ static A from(V v) { return (A)(uint32_t)v; }
    __device__ static A op(A x, A y) { return (A)(uint32_t)(x + y); }
    __device__ static V out(A x) { return (V)(uint32_t)x; }
};
template <> struct Red<MSP_LOR_LAND_BOOL> {
    using V = uint8_t; using A = unsigned long long;
    __device__ static A from(V v) { return v != 0; }
    __device__ static A op(A x, A y) { return (x | y) != 0; }
    __device__ static V out(A x) { return (V)(x != 0); }
};

template <int SR>
__device__ typename Red<SR>::A block_reduce(typename Red<SR>::A v) {
    using R = Red<SR>;
    __shared__ typename R::A t[RED_T / WAVE];
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) v = R::op(v, __shfl_xor(v, d, WAVE));
    if (lane() == 0) t[threadIdx.x / WAVE] = v;
    __syncthreads();
    typename R::A r = t[0];
    for (int w = 1; w < RED_T / WAVE; ++w) r = R::op(r, t[w]);
    return r;
}

// n elements, or min(*n_dev, n) when the count is given on the device
template <int SR>
__global__ __launch_bounds__(RED_T) void k_reduce_partial(const typename Red<SR>::V* __restrict__ v, int64_t n,
                                                          const int64_t* n_dev, typename Red<SR>::A* partial) {
    using R = Red<SR>;
    if (n_dev) n = max((int64_t)0, min(n, *n_dev));
    typename R::A acc = R::from(typename R::V(0));
    for (int64_t x = (int64_t)blockIdx.x * RED_T + threadIdx.x; x < n; x += (int64_t)gridDim.x * RED_T)
        acc = R::op(acc, R::from(v[x]));
    acc = block_reduce<SR>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <int SR>
__global__ __launch_bounds__(RED_T) void k_reduce_final(const typename Red<SR>::A* partial, int nb,
                                                        typename Red<SR>::V* out) {
    using R = Red<SR>;
    typename R::A acc = R::from(typename R::V(0));
    for (int x = threadIdx.x; x < nb; x += RED_T) acc = R::op(acc, partial[x]);
    acc = block_reduce<SR>(acc);
    if (threadIdx.x == 0) *out = R::out(acc);
}

template <int SR>
static hipError_t launch_reduce_t(const void* vals, int64_t n, const int64_t* n_dev, void* partial, void* result,
                                  hipStream_t s) {
    using R = Red<SR>;
    const int nb = (int)grid_for(n, RED_T * 8, RED_BLOCKS);
    MSP_LAUNCH(k_reduce_partial<SR>, dim3(nb), dim3(RED_T), 0, s, static_cast<const typename R::V*>(vals), n, n_dev,
                       static_cast<typename R::A*>(partial));
    MSP_LAUNCH(k_reduce_final<SR>, dim3(1), dim3(RED_T), 0, s, static_cast<const typename R::A*>(partial), nb,
                       static_cast<typename R::V*>(result));
    return hipGetLastError();
}

hipError_t launch_reduce(int semiring, const void* vals, int64_t n, const int64_t* n_dev, void* partial, void* result,
                         hipStream_t s) {
    switch (semiring) {
    case MSP_PLUS_TIMES_F64: return launch_reduce_t<MSP_PLUS_TIMES_F64>(vals, n, n_dev, partial, result, s);
    case MSP_PLUS_PAIR_I64: return launch_reduce_t<MSP_PLUS_PAIR_I64>(vals, n, n_dev, partial, result, s);
    case MSP_LOR_LAND_BOOL: return launch_reduce_t<MSP_LOR_LAND_BOOL>(vals, n, n_dev, partial, result, s);
    case MSP_PLUS_TIMES_I32: return launch_reduce_t<MSP_PLUS_TIMES_I32>(vals, n, n_dev, partial, result, s);
    case MSP_PLUS_TIMES_I64: return launch_reduce_t<MSP_PLUS_TIMES_I64>(vals, n, n_dev, partial, result, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mspk
