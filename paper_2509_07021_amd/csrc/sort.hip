// sort.hip -- fills, exclusive scan, tile|depth key emission, stable LSD radix sort and
// per-tile ranges for the tile/depth key table (gfx950, wave64).
//
// The radix sort is reduce-then-scan with a fixed grid: each workgroup owns a contiguous chunk of
// the input, so the per-pass digit counts form a [256][G] table whose digit-major exclusive scan
// gives every workgroup its scatter base per digit. Ranks inside a workgroup are stable: each
// wave64 owns a contiguous segment of a 4096-item tile, equal digits within a 64-item step are
// found with one 64-bit ballot per digit bit, and per-wave running counts live in LDS. There are no
// inter-workgroup waits, so no pass depends on forward progress of other workgroups. The element
// count is read on device, which lets the same launches run inside a captured graph.
#include "megs_internal.hpp"

namespace megs {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanIpt = 8;
constexpr int kScanTile = kScanThreads * kScanIpt;  // 2048

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / kWave;
constexpr int kRsIpt = 16;
constexpr int kRsTile = kRsThreads * kRsIpt;  // 4096
constexpr int kRsDigits = 256;
constexpr int kRsMaxBlocks = 2048;
static_assert(kRsThreads == kRsDigits, "the downsweep maps one thread to one digit");

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_iota(uint32_t* p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

// ------------------------------------------------------------------- scan ----

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of the 256 threads' values; returns the thread's exclusive prefix and the total.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* lds4, uint32_t& total) {
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(x);
    if (lane == kWave - 1) lds4[w] = inc;
    __syncthreads();
    uint32_t wbase = 0;
    total = 0;
    for (int i = 0; i < 4; ++i) {
        uint32_t s = lds4[i];
        if (i < w) wbase += s;
        total += s;
    }
    __syncthreads();
    return wbase + inc - x;
}

// Sum of the 256 threads' values in 64 bits (every thread receives it). The tile counts are summed in
// 32 bits everywhere else; these wider sums only detect a total that 32 bits cannot hold.
__device__ __forceinline__ uint64_t block_sum64(uint64_t x, uint64_t* lds4) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    __syncthreads();
    if (__lane_id() == 0) lds4[threadIdx.x / kWave] = x;
    __syncthreads();
    const uint64_t t = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    __syncthreads();
    return t;
}

// A 64-bit sum as a 32-bit word, saturated: a total of 2^32 - 1 or more reads as 0xffffffff.
__device__ __forceinline__ uint32_t sat32(uint64_t x) { return x > 0xffffffffull ? 0xffffffffu : (uint32_t)x; }

__device__ __forceinline__ uint32_t scan_load(const uint32_t* x, const uint32_t* idx, int64_t i, int64_t n) {
    if (i >= n) return 0u;
    return x[idx ? idx[i] : i];
}

// Per-workgroup totals. With an index list, the gathered values x[idx[i]] are also stored densely
// to `gathered` (when given), so the second pass reads them without gathering again.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* x, const uint32_t* idx, int64_t n,
                                                              uint32_t* partial, uint32_t* gathered) {
    __shared__ uint64_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (int j = 0; j < kScanIpt; ++j) {
        const int64_t i = base + j * kScanThreads + threadIdx.x;
        const uint32_t v = scan_load(x, idx, i, n);
        if (gathered && i < n) gathered[i] = v;
        s += v;
    }
    const uint64_t total = block_sum64(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = sat32(total);
}

// Single workgroup: exclusive scan of partial[0..m) in place; writes the grand total, saturated at
// 0xffffffff (sat32: a total 32 bits cannot hold, which the pair count check then refuses; the 32-bit
// offsets written here are then meaningless).
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t* partial, int64_t m, uint32_t* total_out) {
    __shared__ uint32_t lds[4];
    __shared__ uint64_t lds64[4];
    uint32_t carry = 0;
    uint64_t carry64 = 0;
    for (int64_t base = 0; base < m; base += kScanTile) {
        uint32_t v[kScanIpt];
        uint32_t s = 0;
        uint64_t s64 = 0;
        for (int j = 0; j < kScanIpt; ++j) {
            int64_t i = base + threadIdx.x * kScanIpt + j;
            v[j] = i < m ? partial[i] : 0u;
            s += v[j];
            s64 += v[j];
        }
        uint32_t total;
        uint32_t ex = block_excl_scan256(s, lds, total) + carry;
        for (int j = 0; j < kScanIpt; ++j) {
            int64_t i = base + threadIdx.x * kScanIpt + j;
            if (i < m) partial[i] = ex;
            ex += v[j];
        }
        carry += total;
        carry64 += block_sum64(s64, lds64);
    }
    if (threadIdx.x == 0 && total_out) *total_out = sat32(carry64);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* x, const uint32_t* idx, int64_t n,
                                                            const uint32_t* partial, uint32_t* out) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanIpt;
    uint32_t v[kScanIpt];
    uint32_t s = 0;
    for (int j = 0; j < kScanIpt; ++j) {
        v[j] = scan_load(x, idx, base + j, n);
        s += v[j];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan256(s, lds, total) + partial[blockIdx.x];
    for (int j = 0; j < kScanIpt; ++j) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
}

// Scan over depth-sorted packed values (record id below bit idb, tile count above it).
__device__ __forceinline__ uint32_t packed_count(uint32_t v, const uint32_t* ntiles, int idb) {
    const uint32_t c = v >> idb, cap = (1u << (32 - idb)) - 1u;
    return c == cap ? ntiles[v & ((1u << idb) - 1u)] : c;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce_packed(const uint32_t* order, const uint32_t* ntiles,
                                                                     int64_t n, int idb, uint32_t* partial) {
    __shared__ uint64_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // every load first (lanes past the end read item 0, n >= 1), so they are in flight together
    uint32_t w[kScanIpt];
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        const int64_t i = base + j * kScanThreads + threadIdx.x;
        w[j] = order[i < n ? i : 0];
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        const int64_t i = base + j * kScanThreads + threadIdx.x;
        if (i < n) s += packed_count(w[j], ntiles, idb);
    }
    const uint64_t total = block_sum64(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = sat32(total);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down_packed(uint32_t* order, const uint32_t* ntiles, int64_t n,
                                                                   int idb, const uint32_t* partial, uint32_t* out) {
    __shared__ uint32_t lds[4];
    static_assert(kScanIpt == 8, "a thread's items are two 16-byte vectors");
    // a thread's 8 consecutive items move as two 16-byte vectors (order and out are 256-byte
    // aligned and base is a multiple of 8), so every access of the wave is contiguous
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanIpt;
    const bool whole = base + kScanIpt <= n;
    const uint32_t idmask = (1u << idb) - 1u;
    uint32_t w[kScanIpt], v[kScanIpt];
    if (whole) {
        const uint4* q = reinterpret_cast<const uint4*>(order + base);
        const uint4 a = q[0], b = q[1];
        w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w; w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < kScanIpt; ++j) w[j] = base + j < n ? order[base + j] : 0u;
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        v[j] = base + j < n ? packed_count(w[j], ntiles, idb) : 0u;
        s += v[j];
        w[j] &= idmask;
    }
    uint32_t total;
    uint32_t ex = block_excl_scan256(s, lds, total) + partial[blockIdx.x];
    uint32_t o[kScanIpt];
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        o[j] = ex;
        ex += v[j];
    }
    if (whole) {
        uint4* q = reinterpret_cast<uint4*>(order + base);
        q[0] = make_uint4(w[0], w[1], w[2], w[3]);
        q[1] = make_uint4(w[4], w[5], w[6], w[7]);
        uint4* r = reinterpret_cast<uint4*>(out + base);
        r[0] = make_uint4(o[0], o[1], o[2], o[3]);
        r[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int j = 0; j < kScanIpt; ++j)
            if (base + j < n) {
                order[base + j] = w[j];
                out[base + j] = o[j];
            }
    }
}

// ------------------------------------------------------------- radix sort ----

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
    return (uint32_t)(key >> shift) & mask;
}

// Lanes of the wave holding the same digit as this lane, restricted to `valid` (mask: the
// pass's digit mask, at most 8 bits).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid, uint32_t mask) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (!((mask >> b) & 1u)) break;
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

struct Chunk {
    int64_t n, t0, t1;
};

__device__ __forceinline__ Chunk chunk_of(const uint32_t* d_count, int64_t max_count) {
    Chunk c;
    int64_t n = (int64_t)*d_count;
    c.n = n < max_count ? n : max_count;
    const int64_t tiles = (c.n + kRsTile - 1) / kRsTile;
    const int64_t per = (tiles + gridDim.x - 1) / gridDim.x;
    c.t0 = (int64_t)blockIdx.x * per;
    c.t1 = c.t0 + per < tiles ? c.t0 + per : tiles;
    return c;
}

template <typename K>
__global__ __launch_bounds__(kRsThreads) void k_radix_upsweep(const K* __restrict__ keys, const uint32_t* d_count,
                                                              int64_t max_count, int shift, uint32_t mask,
                                                              uint32_t* __restrict__ counts) {
    // Digit counts of the workgroup's chunk (order does not matter here): per-wave LDS histograms
    // updated with LDS atomics, or with one add when the whole 64-key step shares its digit. Each
    // wave keeps kCopies histograms, lane l adding to copy l % kCopies: lanes with equal digits
    // then collide on one address a quarter as often (the atomics on one address serialise), and
    // the odd stride puts the copies of a digit in different LDS banks.
    constexpr int U = 8;
    constexpr int kCopies = 4, kStride = kRsDigits + 1;
    __shared__ uint32_t hist[kRsWaves][kCopies * kStride];
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const int cp = (lane & (kCopies - 1)) * kStride;
    for (int i = threadIdx.x; i < kRsWaves * kCopies * kStride; i += kRsThreads) (&hist[0][0])[i] = 0u;
    __syncthreads();
    const Chunk c = chunk_of(d_count, max_count);
    const int64_t i1 = c.t1 * kRsTile < c.n ? c.t1 * kRsTile : c.n;
    for (int64_t base = c.t0 * kRsTile + (int64_t)w * kWave * U; base < i1; base += (int64_t)kRsThreads * U) {
        // every key load first (lanes past the end read the chunk's last key), so the U loads are in
        // flight together; the digits after
        K kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = base + u * kWave + lane;
            kv[u] = keys[idx < i1 ? idx : i1 - 1];
        }
        uint32_t d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = base + u * kWave + lane;
            d[u] = idx < i1 ? digit_of(kv[u], shift, mask) : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t valid = __ballot(d[u] != 0xffffffffu);
            if (!valid) break;  // positions rise with u and lane: nothing valid after this step
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d[u]);  // lane 0 is valid here
            if (__ballot(d[u] == d0) == valid) {
                if (lane == 0) atomicAdd(&hist[w][d0], (uint32_t)__popcll(valid));
            } else if (d[u] != 0xffffffffu) {
                atomicAdd(&hist[w][cp + d[u]], 1u);
            }
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRsDigits; d += kRsThreads) {
        uint32_t s = 0;
        for (int ww = 0; ww < kRsWaves; ++ww)
            for (int cc = 0; cc < kCopies; ++cc) s += hist[ww][cc * kStride + d];
        counts[(int64_t)d * gridDim.x + blockIdx.x] = s;
    }
}

// Exclusive scan of one digit's row of the [256][G] count table (one workgroup per digit, in
// place); the row total goes to totals[digit]. The downsweep adds the digit bases.
__global__ __launch_bounds__(kScanThreads) void k_radix_scan_rows(uint32_t* counts, int G, uint32_t* totals) {
    __shared__ uint32_t lds[4];
    uint32_t* row = counts + (int64_t)blockIdx.x * G;
    uint32_t carry = 0;
    for (int base = 0; base < G; base += kScanThreads * 4) {
        uint32_t v[4];
        uint32_t sum = 0;
        for (int j = 0; j < 4; ++j) {
            const int i = base + threadIdx.x * 4 + j;
            v[j] = i < G ? row[i] : 0u;
            sum += v[j];
        }
        uint32_t total;
        uint32_t ex = block_excl_scan256(sum, lds, total) + carry;
        for (int j = 0; j < 4; ++j) {
            const int i = base + threadIdx.x * 4 + j;
            if (i < G) row[i] = ex;
            ex += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <typename K>
__global__ __launch_bounds__(kRsThreads) void k_radix_downsweep(const K* __restrict__ keys_in,
                                                                const uint32_t* __restrict__ vals_in,
                                                                K* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                                const uint32_t* d_count, int64_t max_count, int shift,
                                                                uint32_t mask, const uint32_t* __restrict__ offsets,
                                                                const uint32_t* __restrict__ totals) {
    // Per tile: stable ranks -> local sorted order staged in LDS -> coalesced writes of each
    // digit's run to its global position.
    __shared__ uint32_t run_off[kRsDigits];
    __shared__ uint32_t whist[kRsWaves][kRsDigits];
    __shared__ uint32_t tile_start[kRsDigits];
    __shared__ uint32_t lds4[4];
    __shared__ K stage_k[kRsTile];
    __shared__ uint32_t stage_v[kRsTile];
    const int w = threadIdx.x / kWave, lane = __lane_id();
    {
        // digit base = exclusive prefix of the digit totals (thread = digit)
        uint32_t all;
        const uint32_t digit_base = block_excl_scan256(totals[threadIdx.x], lds4, all);
        run_off[threadIdx.x] = digit_base + offsets[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    }
    const Chunk c = chunk_of(d_count, max_count);
    // a pass whose digit is the same for every key is the identity permutation: copy the chunk
    if (__syncthreads_or(totals[threadIdx.x] == (uint32_t)c.n && c.n > 0)) {
        const int64_t i1 = c.t1 * kRsTile < c.n ? c.t1 * kRsTile : c.n;
        for (int64_t i = c.t0 * kRsTile + threadIdx.x; i < i1; i += kRsThreads) {
            keys_out[i] = keys_in[i];
            vals_out[i] = vals_in[i];
        }
        return;
    }
    const uint64_t lt = lanemask_lt();
    for (int64_t t = c.t0; t < c.t1; ++t) {
        for (int i = threadIdx.x; i < kRsWaves * kRsDigits; i += kRsThreads) (&whist[0][0])[i] = 0u;
        __syncthreads();
        K key[kRsIpt];
        uint32_t val[kRsIpt], dig[kRsIpt], rank[kRsIpt];
        const int64_t base = t * kRsTile + (int64_t)w * kWave * kRsIpt + lane;
        // all of the tile's loads first (no branch between them), so they are in flight together
#pragma unroll
        for (int j = 0; j < kRsIpt; ++j) {
            const int64_t idx = base + j * kWave;
            const bool ok = idx < c.n;
            key[j] = ok ? keys_in[ok ? idx : 0] : K(0);
            val[j] = ok ? vals_in[ok ? idx : 0] : 0u;
        }
        for (int j = 0; j < kRsIpt; ++j) {
            const int64_t idx = base + j * kWave;
            const bool ok = idx < c.n;
            const uint32_t d = ok ? digit_of(key[j], shift, mask) : 0u;
            dig[j] = ok ? d : 0xffffffffu;
            const uint64_t peers = match_digit(d, __ballot(ok), mask);
            uint32_t before = 0;
            if (ok) before = whist[w][d];
            rank[j] = before + (uint32_t)__popcll(peers & lt);
            if (ok && (__ffsll((unsigned long long)peers) - 1) == lane) whist[w][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per digit (thread = digit): exclusive prefix over waves, tile total, tile-local start
        uint32_t total_d = 0;
        {
            const int d = threadIdx.x;
            for (int ww = 0; ww < kRsWaves; ++ww) {
                const uint32_t cnt = whist[ww][d];
                whist[ww][d] = total_d;
                total_d += cnt;
            }
        }
        uint32_t tile_count;
        const uint32_t start_d = block_excl_scan256(total_d, lds4, tile_count);
        tile_start[threadIdx.x] = start_d;
        __syncthreads();
        for (int j = 0; j < kRsIpt; ++j) {
            if (dig[j] == 0xffffffffu) continue;
            const uint32_t lpos = tile_start[dig[j]] + whist[w][dig[j]] + rank[j];
            stage_k[lpos] = key[j];
            stage_v[lpos] = val[j];
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < tile_count; i += kRsThreads) {
            const K k = stage_k[i];
            const uint32_t d = digit_of(k, shift, mask);
            const uint32_t dst = run_off[d] + (i - tile_start[d]);
            if ((int64_t)dst >= c.n) continue;  // unreachable when the digit counts are consistent
            keys_out[dst] = k;
            vals_out[dst] = stage_v[i];
        }
        __syncthreads();
        run_off[threadIdx.x] += total_d;
        __syncthreads();
    }
}

template <typename K>
hipError_t radix_sort(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, const uint32_t* d_count,
                      int64_t max_count, int begin_bit, int end_bit, void* scratch, hipStream_t stream, bool* in_alt) {
    *in_alt = false;
    if (max_count <= 0 || end_bit <= begin_bit) return hipSuccess;
    int64_t tiles = (max_count + kRsTile - 1) / kRsTile;
    const int G = (int)(tiles < kRsMaxBlocks ? tiles : kRsMaxBlocks);
    uint32_t* counts = static_cast<uint32_t*>(scratch);
    uint32_t* totals = counts + (int64_t)kRsDigits * G;
    K* src_k = keys; uint32_t* src_v = vals;
    K* dst_k = keys_alt; uint32_t* dst_v = vals_alt;
    // the fewest passes of at most 8 bits, with the bits spread evenly over them (14 tile bits sort
    // as 7 + 7: fewer digits per pass give each digit longer runs in the scatter)
    const int passes = radix_passes(begin_bit, end_bit);
    const int width = (end_bit - begin_bit + passes - 1) / passes;
    for (int shift = begin_bit; shift < end_bit; shift += width) {
        const int bits = end_bit - shift < width ? end_bit - shift : width;
        const uint32_t mask = (1u << bits) - 1u;
        hipLaunchKernelGGL(k_radix_upsweep<K>, dim3(G), dim3(kRsThreads), 0, stream, src_k, d_count, max_count, shift,
                           mask, counts);
        hipLaunchKernelGGL(k_radix_scan_rows, dim3(kRsDigits), dim3(kScanThreads), 0, stream, counts, G, totals);
        hipLaunchKernelGGL(k_radix_downsweep<K>, dim3(G), dim3(kRsThreads), 0, stream, src_k, src_v, dst_k, dst_v,
                           d_count, max_count, shift, mask, counts, totals);
        K* tk = src_k; src_k = dst_k; dst_k = tk;
        uint32_t* tv = src_v; src_v = dst_v; dst_v = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- key emission ----

// Key emission. Workgroup b handles the 256 records at positions [256 b, 256 b + 256) of the
// emission order; their pairs occupy one contiguous range of the output (the offsets are an
// exclusive scan in that order). Each thread walks its record's listed tiles row by row and
// drops its pairs into an LDS window of the workgroup's range; the window is then written out
// with coalesced stores, so the scattered per-record runs never reach HBM as scattered writes.
// A window of 2048 pairs (16 KB of LDS) leaves room for five workgroups per CU, and the compiler then
// budgets the kernel's registers for five waves per SIMD (92 instead of 100): emission 0.478 ->
// 0.444 ms on the 8-view 1080p workload against a 4096-pair window, which capped it at four.
constexpr int kEmitThreads = 256;
constexpr int kEmitWindow = 2048;

// With sub-tile masks (sub = 8, tile ids below 2^16), the upper 16 bits of each 32-bit tile key
// flag the 8 x 8 sub-tiles of the tile that the record's cutoff ellipse reaches (bit r S + c for
// sub-row r and sub-column c, S = tile / 8): the row-interval test of the tile selection run at
// 8-pixel granularity, in FP32 and widened by a quarter pixel, so the flags are a superset of the
// exact ones (the blend still tests every flagged record). The pair sort orders on the tile bits
// only, so the flags ride along.
struct BandsF {
    float v, ry, dys, ka, det, b, ia, u;
    bool full;
};

__device__ __forceinline__ BandsF bands_of(const EllipseRows& e) {
    constexpr float kMargin = 0.25f;
    BandsF f;
    f.full = e.full;
    f.u = (float)e.u; f.v = (float)e.v; f.b = (float)e.b; f.det = (float)e.det; f.ia = (float)e.ia;
    f.ka = (float)e.ka; f.dys = (float)e.dys;
    f.ry = (float)e.ry + kMargin;
    return f;
}

// x-extent [xmin, xmax] (widened) of the ellipse within sub-row band y8 (rows y8 * sub ..
// y8 * sub + sub - 1); xmin > xmax when the band misses it.
__device__ __forceinline__ void band_extent(const BandsF& f, int sub, int y8, int height, float& xmin, float& xmax) {
    constexpr float kMargin = 0.25f;
    xmin = 1.0f; xmax = 0.0f;
    if (y8 * sub >= height) return;
    if (f.full) { xmin = -3.0e38f; xmax = 3.0e38f; return; }
    const int ye = (y8 + 1) * sub < height ? (y8 + 1) * sub : height;
    float dl = (y8 * sub + 0.5f) - f.v, dh = (ye - 0.5f) - f.v;
    dl = fmaxf(dl, -f.ry);
    dh = fminf(dh, f.ry);
    if (dl > dh) return;
    const float d1 = fminf(fmaxf(f.dys, dl), dh), d2 = fminf(fmaxf(-f.dys, dl), dh);
    // hardware square root (about 1 ulp): the quarter-pixel margin dwarfs its error
    const float s1 = __builtin_amdgcn_sqrtf(fmaxf(f.ka - f.det * d1 * d1, 0.0f));
    const float s2 = __builtin_amdgcn_sqrtf(fmaxf(f.ka - f.det * d2 * d2, 0.0f));
    xmax = f.u + (s1 - f.b * d1) * f.ia + kMargin;
    xmin = f.u - (s2 + f.b * d2) * f.ia - kMargin;
}

// The image's sub-columns [c0, c1] (8 pixels each) whose pixel-centre range meets [xmin, xmax],
// once per band; c0 > c1 when the band misses the ellipse. Clamped so the per-tile differences
// below cannot overflow.
__device__ __forceinline__ void band_columns(float xmin, float xmax, int sub, int& c0, int& c1) {
    const float isub = 1.0f / (float)sub;  // sub is a power of two
    const float lo = ceilf((xmin + 0.5f) * isub - 1.0f), hi = floorf((xmax - 0.5f) * isub);
    const bool empty = !(xmin <= xmax);
    c0 = empty ? 1 : (int)fminf(fmaxf(lo, -1.0f), 1048576.0f);
    c1 = empty ? 0 : (int)fminf(fmaxf(hi, -2.0f), 1048576.0f);
}

// Bits of the sub-columns of tile column tx (S per tile) within [c0, c1] (branch-free).
__device__ __forceinline__ uint32_t band_bits(int c0, int c1, int tx, int S) {
    const int lo = max(c0 - tx * S, 0), hi = min(c1 - tx * S, S - 1);
    const uint32_t bits = ((2u << max(hi, 0)) - 1u) & ~((1u << min(lo, 31)) - 1u);
    return lo <= hi ? bits : 0u;
}

// Sub-columns [c0, c1] as a bit mask relative to sub-column `first`, over `nbits` <= 64 bits
// (bit p: sub-column first + p); c0 > c1 or no overlap gives 0 (branch-free, shifts kept in range).
__device__ __forceinline__ uint64_t band_mask(int c0, int c1, int first, int nbits) {
    const int lo = max(c0 - first, 0), hi = min(c1 - first, nbits - 1);
    const uint64_t upto = (2ull << min(max(hi, 0), 63)) - 1ull;  // bits 0..hi (all 64 when hi = 63)
    const uint64_t below = (1ull << min(lo, 63)) - 1ull;        // bits 0..lo-1
    return lo <= hi ? upto & ~below : 0ull;
}

// S: sub-tiles per tile edge when the keys carry sub-tile flags (tile = 8 S), 0 without flags.
template <int S>
__global__ __launch_bounds__(kEmitThreads) void k_emit(Records rec, const ViewInfo* __restrict__ views, int64_t n,
                                                       int tile, const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ total, int64_t n_records,
                                                       uint32_t* __restrict__ tile_keys, uint64_t* __restrict__ keys64,
                                                       uint32_t* __restrict__ vals, int64_t capacity, int32_t* status) {
    constexpr int SUB = 8;
    constexpr int kBuckets = 64;  // tile counts >= 63 share the last bucket
    __shared__ uint32_t w_tile[kEmitWindow];
    __shared__ uint32_t w_val[kEmitWindow];
    __shared__ uint32_t range[2];
    __shared__ uint32_t bucket[kBuckets];
    __shared__ uint16_t perm[kEmitThreads];
    // per record of the workgroup (slot = its position in emission order): what the emission reads of
    // it, gathered by the slot's own thread and taken by the thread that emits the record
    __shared__ float4 s_q0[kEmitThreads], s_q1[kEmitThreads];
    __shared__ uint4 s_meta[kEmitThreads];  // opacity bits, record id, tile count, offset
    const int64_t kb = (int64_t)blockIdx.x * kEmitThreads;
    const int64_t k_last = min(kb + kEmitThreads, n_records) - 1;
    {
        // A lane's time is set by the record with the most work in its wave, so the workgroup's
        // records are dealt to lanes grouped by an estimate of their work (a counting sort in LDS):
        // the tile rows the footprint's vertical extent spans (each costs a row test and, where the
        // row lists tiles, four sub-row bands) and the tiles. Which lane handles a record does not
        // change what is written where. A record's tile count is the step of the exclusive scan to the
        // next record (modulo 2^32, exact while the counts fit), read in emission order.
        const int64_t k0 = kb + threadIdx.x;
        uint32_t nt0 = 0, off0 = 0, g0 = 0, key = 0;
        float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
        float ao = 0.f;
        if (k0 < n_records) {
            off0 = offsets[k0];
            nt0 = (k0 + 1 < n_records ? offsets[k0 + 1] : *total) - off0;
            if (k0 == k_last) {
                range[0] = offsets[kb];
                range[1] = (uint32_t)((int64_t)off0 + nt0);
            }
            if (nt0) {  // the record: mean | factor ratio, diagonal factors | opacity; without tiles not read
                g0 = order ? order[k0] : (uint32_t)k0;
                const float4* q = reinterpret_cast<const float4*>(rec.packed + g0);
                a0 = q[0]; a1 = q[1];
                ao = reinterpret_cast<const float*>(q + 2)[0];
                const float my = (float)__hiloint2double(__float_as_int(a0.w), __float_as_int(a0.z));
                const double rr = __hiloint2double(__float_as_int(a1.y), __float_as_int(a1.x));
                const float rho = ceilf(footprint_rho(a1.z, rr, a1.w, ao)), it = 1.0f / (float)tile;
                const int rows = (int)(floorf((my + rho) * it) - floorf((my - rho) * it)) + 1;
                const uint32_t ur = (uint32_t)min(max(rows, 1), 64), ut = min(nt0, 64u);
                key = min((60u * ur + 150u * min(ur, ut) + 12u * ut) / 24u, (uint32_t)kBuckets - 1u);
            }
        }
        s_q0[threadIdx.x] = a0;
        s_q1[threadIdx.x] = a1;
        s_meta[threadIdx.x] = make_uint4(__float_as_uint(ao), g0, nt0, off0);
        if (threadIdx.x < kBuckets) bucket[threadIdx.x] = 0u;
        __syncthreads();
        const uint32_t rank = atomicAdd(&bucket[key], 1u);
        __syncthreads();
        if (threadIdx.x < kBuckets) {  // one wave: exclusive scan of the bucket sizes
            const uint32_t c = bucket[threadIdx.x];
            bucket[threadIdx.x] = wave_incl_scan(c) - c;
        }
        __syncthreads();
        perm[bucket[key] + rank] = (uint16_t)threadIdx.x;
        __syncthreads();
    }
    const int slot = perm[threadIdx.x];
    const int64_t k = kb + slot;
    const bool has = k < n_records;
    const uint4 meta = s_meta[slot];
    const uint32_t g = meta.y, nt = has ? meta.z : 0u;
    const float4 q0 = s_q0[slot], q1 = s_q1[slot];
    const float o = __uint_as_float(meta.x);
    const int64_t off = has ? (int64_t)meta.w : 0;
    // windows past the table's capacity hold nothing that is written (an overflowed table)
    const int64_t lo = range[0], hi = min((int64_t)range[1], capacity);
    if (has && nt && off + (int64_t)nt > capacity) status[1] = 1;
    // record geometry and the view fields the loops need, in registers (only threads with pairs)
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    int vh = 0, vw_w = 0, tiles_x = 0;
    int64_t tile_off = 0;
    EllipseRows er;
    if (nt) {
        const ViewInfo& vw = views[g / n];
        vh = vw.height;
        vw_w = vw.width;
        tiles_x = vw.tiles_x;
        tile_off = vw.tile_off;
        const double mx = __hiloint2double(__float_as_int(q0.y), __float_as_int(q0.x));
        const double my = __hiloint2double(__float_as_int(q0.w), __float_as_int(q0.z));
        const double rr = __hiloint2double(__float_as_int(q1.y), __float_as_int(q1.x));
        // the radius the projection stored for this record (a record with tiles has a finite one)
        const int32_t rad = (int32_t)ceilf(footprint_rho(q1.z, rr, q1.w, o));
        tile_rect(mx, my, rad, vw, tile, x0, x1, y0, y1);
        ellipse_rows(mx, my, shape_of(q1.z, rr, q1.w), cutoff_of(o), er);
    }
    for (int64_t w0 = lo; w0 < hi; w0 += kEmitWindow) {
        const int64_t w1 = w0 + kEmitWindow < hi ? w0 + kEmitWindow : hi;
        if (nt && off < w1 && off + (int64_t)nt > w0) {
            int64_t pos = off;
            const BandsF bf = bands_of(er);
            for (int ty = y0; ty <= y1 && pos < w1; ++ty) {
                int cl, ch;
                if (!row_span(er, vw_w, vh, tile, ty, x0, x1, cl, ch)) continue;
                if (pos + (ch - cl + 1) <= w0) {  // the whole row lies before this window
                    pos += ch - cl + 1;
                    continue;
                }
                int bc0[S > 0 ? S : 1], bc1[S > 0 ? S : 1];
#pragma unroll
                for (int r = 0; r < S; ++r) {
                    float xmin, xmax;
                    band_extent(bf, SUB, ty * S + r, vh, xmin, xmax);
                    band_columns(xmin, xmax, SUB, bc0[r], bc1[r]);
                }
                const uint32_t row_key = (uint32_t)(tile_off + (int64_t)ty * tiles_x) + (uint32_t)cl;
                // the row's tiles k = 0 .. nrow - 1 at positions pos + k; those inside this window (the
                // row reaches into it: w0 - nrow < pos < w1, so base lies in (-nrow, kEmitWindow))
                const int nrow = ch - cl + 1;
                const int base = (int)(pos - w0);
                const int k0 = max(0, -base), k1 = min(nrow, (int)(w1 - w0) - base);
                uint32_t* wt = w_tile + base;
                uint32_t* wv = w_val + base;
                pos += nrow;
                if (!S) {
                    for (int k = k0; k < k1; ++k) {
                        wt[k] = row_key + (uint32_t)k;
                        wv[k] = g;
                    }
                } else if (nrow * S <= 32) {
                    // each sub-row's flags over the row's sub-columns in one 32-bit mask; a tile's S
                    // bits are a bit-field extract from each
                    uint32_t rm[S > 0 ? S : 1];
#pragma unroll
                    for (int r = 0; r < S; ++r) rm[r] = (uint32_t)band_mask(bc0[r], bc1[r], cl * S, nrow * S);
                    for (int k = k0; k < k1; ++k) {
                        uint32_t m = __builtin_amdgcn_ubfe(rm[0], (uint32_t)(k * S), (uint32_t)S);
#pragma unroll
                        for (int r = 1; r < S; ++r)
                            m |= __builtin_amdgcn_ubfe(rm[r], (uint32_t)(k * S), (uint32_t)S) << (r * S);
                        wt[k] = (row_key + (uint32_t)k) | (m << 16);
                        wv[k] = g;
                    }
                } else if (nrow * S <= 64) {
                    uint64_t rm[S > 0 ? S : 1];
#pragma unroll
                    for (int r = 0; r < S; ++r) rm[r] = band_mask(bc0[r], bc1[r], cl * S, nrow * S);
                    for (int k = k0; k < k1; ++k) {
                        uint32_t m = 0;
#pragma unroll
                        for (int r = 0; r < S; ++r)
                            m |= ((uint32_t)(rm[r] >> (k * S)) & ((1u << S) - 1u)) << (r * S);
                        wt[k] = (row_key + (uint32_t)k) | (m << 16);
                        wv[k] = g;
                    }
                } else {  // wider rows form each tile's flags from the sub-rows' column ranges
                    for (int k = k0; k < k1; ++k) {
                        uint32_t m = 0;
#pragma unroll
                        for (int r = 0; r < S; ++r) m |= band_bits(bc0[r], bc1[r], cl + k, S) << (r * S);
                        wt[k] = (row_key + (uint32_t)k) | (m << 16);
                        wv[k] = g;
                    }
                }
            }
        }
        __syncthreads();
        const int cnt = (int)(w1 - w0);
        for (int i = threadIdx.x; i < cnt; i += kEmitThreads) {
            const int64_t pos = w0 + i;
            if (pos >= capacity) break;
            const uint32_t gt = w_tile[i], gv = w_val[i];
            if (tile_keys) tile_keys[pos] = gt;
            if (keys64) keys64[pos] = ((uint64_t)gt << 32) | rec.dkey[gv];  // depth bits (gv has tiles)
            vals[pos] = gv;
        }
        __syncthreads();
    }
}

// ------------------------------------------------- deterministic backward support ----

__global__ void k_copy_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_perm_gather(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ rec_emit,
                              const uint32_t* d_count, int64_t max_count, uint32_t* __restrict__ rec_sorted,
                              uint32_t* __restrict__ inv) {
    const int64_t count = min((int64_t)*d_count, max_count);
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = perm[s];
        rec_sorted[s] = rec_emit[e];
        inv[e] = (uint32_t)s;
    }
}

__global__ void k_pair_reduce(const uint32_t* __restrict__ order, const uint32_t* __restrict__ offsets,
                              const uint32_t* __restrict__ ntiles, int64_t n_records, const uint32_t* __restrict__ inv,
                              const uint32_t* d_count, const float* __restrict__ grad_pair, float* __restrict__ grad2d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_records) return;
    const uint32_t r = order ? order[i] : (uint32_t)i;
    const int64_t count = *d_count;
    const int64_t e0 = offsets[i];
    int64_t e1 = e0 + ntiles[r];
    if (e1 > count) e1 = count;
    float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t e = e0; e < e1; ++e) {
        const float* g = grad_pair + 9 * (int64_t)inv[e];
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[c] += g[c];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) grad2d[grad2d_index(r, c)] = acc[c];
}

// The pair count the sort and ranges read, clamped to the table's capacity; the counted total goes to
// status[0] (saturated at 2^31 - 1), and status[1] flags a total beyond the capacity or beyond 2^31 - 1
// pairs (kMaxPairs: the tables' 32-bit positions and the status word hold no more).
__global__ void k_clamp_count(const uint32_t* total, int64_t capacity, uint32_t* count, int32_t* status) {
    const uint32_t t = *total;
    const bool over = (int64_t)t > capacity || t > kMaxPairs;
    *count = over ? (uint32_t)(capacity < (int64_t)kMaxPairs ? capacity : (int64_t)kMaxPairs) : t;
    status[0] = (int32_t)(t > kMaxPairs ? kMaxPairs : t);
    if (over) status[1] = 1;
}

template <typename K>
__global__ void k_ranges(const K* __restrict__ keys, int shift, uint32_t tmask, const uint32_t* d_count,
                         int64_t max_count, uint2* __restrict__ ranges) {
    int64_t n = (int64_t)*d_count;
    if (n > max_count) n = max_count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(keys[i] >> shift) & tmask;
        if (i == 0 || ((uint32_t)(keys[i - 1] >> shift) & tmask) != t) ranges[t].x = (uint32_t)i;
        if (i == n - 1 || ((uint32_t)(keys[i + 1] >> shift) & tmask) != t) ranges[t].y = (uint32_t)(i + 1);
    }
}

// The same for 32-bit keys, 4 V consecutive keys per thread through V 16-byte loads (the key arrays
// are 256-byte aligned), all issued before any key is compared, plus the keys just before and after
// them: those are the neighbouring lanes' last and first keys, taken by shuffles, and loaded only at
// the wave's ends.
template <int V>
__global__ void k_ranges_u32x4(const uint32_t* __restrict__ keys, uint32_t tmask, const uint32_t* d_count,
                               int64_t max_count, uint2* __restrict__ ranges) {
    constexpr int KPT = 4 * V;  // keys per thread
    int64_t n = (int64_t)*d_count;
    if (n > max_count) n = max_count;
    const int64_t nq = (n + KPT - 1) / KPT;
    const int lane = __lane_id();
    // whole waves take part in every iteration (the shuffles read the neighbouring lanes), lanes
    // past the end with no keys
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q - lane < nq; q += stride) {
        const int64_t i0 = KPT * q;
        uint32_t t[KPT];
        if (i0 + KPT <= n) {
            uint4 v[V];
#pragma unroll
            for (int u = 0; u < V; ++u) v[u] = reinterpret_cast<const uint4*>(keys + i0)[u];
#pragma unroll
            for (int u = 0; u < V; ++u) {
                t[4 * u] = v[u].x & tmask; t[4 * u + 1] = v[u].y & tmask;
                t[4 * u + 2] = v[u].z & tmask; t[4 * u + 3] = v[u].w & tmask;
            }
        } else {
#pragma unroll
            for (int j = 0; j < KPT; ++j) t[j] = i0 + j < n ? keys[i0 + j] & tmask : 0u;
        }
        uint32_t before = (uint32_t)__shfl_up((int)t[KPT - 1], 1);
        uint32_t after = (uint32_t)__shfl_down((int)t[0], 1);
        if (lane == 0) before = i0 > 0 && i0 - 1 < n ? keys[i0 - 1] & tmask : 0u;
        if (lane == kWave - 1) after = i0 + KPT < n ? keys[i0 + KPT] & tmask : 0u;
        if (q >= nq) continue;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int64_t i = i0 + j;
            if (i >= n) break;
            const bool first = i == 0 || (j == 0 ? before : t[j - 1]) != t[j];
            const bool last = i == n - 1 || (j == KPT - 1 ? after : t[j + 1]) != t[j];
            if (first) ranges[t[j]].x = (uint32_t)i;
            if (last) ranges[t[j]].y = (uint32_t)(i + 1);
        }
    }
}

constexpr int kRangeVecs = 4;  // 16-byte vectors of tile keys per thread

inline unsigned grid_for(int64_t count, int threads, int64_t cap = 65536) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256, 8192)), dim3(256), 0, stream, p, value, count);
    return hipGetLastError();
}

hipError_t launch_iota(uint32_t* p, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(count, 256, 8192)), dim3(256), 0, stream, p, count);
    return hipGetLastError();
}

size_t scan_scratch_bytes(int64_t n) {
    const int64_t blocks = (n + kScanTile - 1) / kScanTile;
    return (size_t)((blocks > 0 ? blocks : 1) * sizeof(uint32_t));
}

hipError_t launch_scan(const uint32_t* x, const uint32_t* idx, int64_t n, uint32_t* out, uint32_t* total,
                       void* scratch, hipStream_t stream, uint32_t* gathered) {
    if (n <= 0) {
        return launch_fill_u32(total, 0u, 1, stream);
    }
    const int64_t blocks = (n + kScanTile - 1) / kScanTile;
    uint32_t* partial = static_cast<uint32_t*>(scratch);
    uint32_t* g = idx ? gathered : nullptr;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)blocks), dim3(kScanThreads), 0, stream, x, idx, n, partial, g);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, stream, partial, blocks, total);
    if (g)
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)blocks), dim3(kScanThreads), 0, stream,
                           static_cast<const uint32_t*>(g), static_cast<const uint32_t*>(nullptr), n, partial, out);
    else
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)blocks), dim3(kScanThreads), 0, stream, x, idx, n, partial,
                           out);
    return hipGetLastError();
}

hipError_t launch_scan_packed(uint32_t* order, const uint32_t* ntiles, int64_t n, int idb, uint32_t* out,
                              uint32_t* total, void* scratch, hipStream_t stream) {
    if (n <= 0) return launch_fill_u32(total, 0u, 1, stream);
    if (idb < 1 || idb > 28) return hipErrorInvalidValue;
    const int64_t blocks = (n + kScanTile - 1) / kScanTile;
    uint32_t* partial = static_cast<uint32_t*>(scratch);
    hipLaunchKernelGGL(k_scan_reduce_packed, dim3((unsigned)blocks), dim3(kScanThreads), 0, stream, order, ntiles, n,
                       idb, partial);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, stream, partial, blocks, total);
    hipLaunchKernelGGL(k_scan_down_packed, dim3((unsigned)blocks), dim3(kScanThreads), 0, stream, order, ntiles, n,
                       idb, partial, out);
    return hipGetLastError();
}

// The fewest passes of at most 8 bits over [begin_bit, end_bit); the sorted data ends in the
// alternate buffers exactly when this is odd.
int radix_passes(int begin_bit, int end_bit) { return end_bit > begin_bit ? (end_bit - begin_bit + 7) / 8 : 0; }

size_t radix_scratch_bytes(int64_t max_count) {
    const int64_t tiles = (max_count + kRsTile - 1) / kRsTile;
    const int64_t G = tiles < kRsMaxBlocks ? (tiles > 0 ? tiles : 1) : kRsMaxBlocks;
    return (size_t)((kRsDigits * G + kRsDigits) * sizeof(uint32_t));
}

hipError_t launch_radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                 const uint32_t* d_count, int64_t max_count, int begin_bit, int end_bit,
                                 void* scratch, hipStream_t stream, bool* in_alt) {
    return radix_sort<uint32_t>(keys, vals, keys_alt, vals_alt, d_count, max_count, begin_bit, end_bit, scratch,
                                stream, in_alt);
}

hipError_t launch_radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                                 const uint32_t* d_count, int64_t max_count, int begin_bit, int end_bit,
                                 void* scratch, hipStream_t stream, bool* in_alt) {
    return radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, d_count, max_count, begin_bit, end_bit, scratch,
                                stream, in_alt);
}

hipError_t launch_emit(const Records& rec, const ViewInfo* views, int nv, int64_t n, int tile,
                       const uint32_t* order, const uint32_t* offsets, const uint32_t* total, int64_t n_records,
                       uint32_t* tile_keys, uint64_t* keys64, uint32_t* vals, int64_t capacity,
                       int32_t* status, hipStream_t stream, int sub) {
    (void)nv;
    if (n_records <= 0) return hipSuccess;
    if (sub && (sub != 8 || !tile_keys || (tile != 16 && tile != 32))) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_records + kEmitThreads - 1) / kEmitThreads));
    if (!sub)
        hipLaunchKernelGGL(k_emit<0>, grid, dim3(kEmitThreads), 0, stream, rec, views, n, tile, order, offsets,
                           total, n_records, tile_keys, keys64, vals, capacity, status);
    else if (tile == 16)
        hipLaunchKernelGGL(k_emit<2>, grid, dim3(kEmitThreads), 0, stream, rec, views, n, tile, order, offsets,
                           total, n_records, tile_keys, keys64, vals, capacity, status);
    else
        hipLaunchKernelGGL(k_emit<4>, grid, dim3(kEmitThreads), 0, stream, rec, views, n, tile, order, offsets,
                           total, n_records, tile_keys, keys64, vals, capacity, status);
    return hipGetLastError();
}

hipError_t launch_ranges_u32(const uint32_t* tile_keys, const uint32_t* d_count, int64_t max_count, uint2* ranges,
                             hipStream_t stream, uint32_t tmask) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ranges_u32x4<kRangeVecs>, dim3(grid_for((max_count + 4 * kRangeVecs - 1) / (4 * kRangeVecs), 256)),
                       dim3(256), 0, stream, tile_keys, tmask, d_count, max_count, ranges);
    return hipGetLastError();
}

hipError_t launch_ranges_u64(const uint64_t* keys, const uint32_t* d_count, int64_t max_count, uint2* ranges,
                             hipStream_t stream) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ranges<uint64_t>, dim3(grid_for(max_count, 256)), dim3(256), 0, stream, keys, 32, ~0u,
                       d_count, max_count, ranges);
    return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_u32, dim3(grid_for(count, 256)), dim3(256), 0, stream, dst, src, count);
    return hipGetLastError();
}

hipError_t launch_perm_gather(const uint32_t* perm, const uint32_t* rec_emit, const uint32_t* d_count,
                              int64_t max_count, uint32_t* rec_sorted, uint32_t* inv, hipStream_t stream) {
    if (max_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_perm_gather, dim3(grid_for(max_count, 256)), dim3(256), 0, stream, perm, rec_emit, d_count,
                       max_count, rec_sorted, inv);
    return hipGetLastError();
}

hipError_t launch_pair_reduce(const uint32_t* order, const uint32_t* offsets, const uint32_t* ntiles,
                              int64_t n_records, const uint32_t* inv, const uint32_t* d_count,
                              const float* grad_pair, float* grad2d, hipStream_t stream) {
    if (n_records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_reduce, dim3((unsigned)((n_records + 255) / 256)), dim3(256), 0, stream, order, offsets,
                       ntiles, n_records, inv, d_count, grad_pair, grad2d);
    return hipGetLastError();
}

hipError_t launch_clamp_count(const uint32_t* total, int64_t capacity, uint32_t* count, int32_t* status,
                              hipStream_t stream) {
    hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(1), 0, stream, total, capacity, count, status);
    return hipGetLastError();
}

}  // namespace megs
