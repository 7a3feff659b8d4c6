// Device-wide primitives for wave64 / gfx950: exclusive prefix sums
// (reduce-then-scan, recursive over tile partials) and a stable LSD radix
// sort of 64-bit keys with optional 64-bit payloads (8-bit digits, per-block
// histograms, in-block stable ranking by wave ballots and wave-private
// digit counters).
#include "lv.h"

namespace lv {

template <typename T> __global__ void k_fill(T *p, T v, int64_t n);

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;
constexpr int RADIX_ITEMS = 16;
constexpr int RADIX_TILE = BLOCK * RADIX_ITEMS;

// ---- wave / block helpers --------------------------------------------------
__device__ __forceinline__ int64_t shfl_up_i64(int64_t v, int d)
{
    int lo = __shfl_up((int)(uint32_t)v, d, 64);
    int hi = __shfl_up((int)(v >> 32), d, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// exclusive scan of one value per thread over a 256-thread block; wsum must
// hold 4 entries; returns the exclusive prefix and sets *total
__device__ __forceinline__ int64_t block_exscan(int64_t v, int64_t *wsum, int64_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = shfl_up_i64(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        int64_t t = wsum[w];
        before += (w < wid) ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *wsum)
{
    int64_t t;
    block_exscan(v, wsum, &t);
    return t;
}

// ---- scan -------------------------------------------------------------------
struct LoadI32 {
    const int32_t *p;
    __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct LoadI64 {
    const int64_t *p;
    __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct NonNeg { // 1 where a[i] >= 0
    const int32_t *a;
    __device__ int64_t operator()(int64_t i) const { return a[i] >= 0 ? 1 : 0; }
};
template <int WK> struct TaggedWeight { // the weight of entry i where a[i] == tag, else 0
    const int32_t *a;
    const void *w;
    int32_t tag;
    __device__ int64_t operator()(int64_t i) const { return a[i] == tag ? WLoad<WK>::at(w, i) : 0; }
};
struct Heads {
    const uint64_t *k;
    __device__ int64_t operator()(int64_t i) const { return (i == 0 || k[i] != k[i - 1]) ? 1 : 0; }
};

template <class F>
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(F f, int64_t n, int64_t *part)
{
    __shared__ int64_t wsum[BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        int64_t i = base + r * BLOCK + threadIdx.x;
        if (i < n) s += f(i);
    }
    s = block_sum(s, wsum);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLOCK) void k_scan_single(int64_t *part, int64_t nb, int64_t *total)
{
    __shared__ int64_t wsum[BLOCK / 64];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += BLOCK) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nb ? part[i] : 0;
        int64_t bt;
        int64_t ex = block_exscan(v, wsum, &bt);
        if (i < nb) part[i] = carry + ex;
        carry += bt;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class F, typename T>
__global__ __launch_bounds__(BLOCK) void k_scan_down(F f, int64_t n, const int64_t *part, T *out)
{
    __shared__ int64_t wsum[BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t carry = part[blockIdx.x];
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        int64_t i = base + r * BLOCK + threadIdx.x;
        int64_t v = i < n ? f(i) : 0;
        int64_t bt;
        int64_t ex = block_exscan(v, wsum, &bt);
        if (i < n) out[i] = (T)(carry + ex);
        carry += bt;
    }
}

int64_t scan_partials_needed(int64_t n)
{
    int64_t tot = 0;
    int64_t m = n;
    do {
        m = (m + SCAN_TILE - 1) / SCAN_TILE;
        tot += m + 1;
    } while (m > SCAN_TILE);
    return tot + 16;
}

template <class F, typename T>
static void scan_impl(F f, T *out, int64_t n, int64_t *total, int64_t *part, hipStream_t st)
{
    if (n <= 0) {
        if (total) fill<int64_t>(total, 0, 1, st);
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_reduce<F><<<(unsigned)nb, BLOCK, 0, st>>>(f, n, part);
    if (nb <= SCAN_TILE)
        k_scan_single<<<1, BLOCK, 0, st>>>(part, nb, total);
    else
        scan_impl(LoadI64{part}, part, nb, total, part + nb + 1, st);
    k_scan_down<F, T><<<(unsigned)nb, BLOCK, 0, st>>>(f, n, part, out);
}

void scan_i32_to_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st)
{
    scan_impl(LoadI32{in}, out, n, total, s.part, st);
}

void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st)
{
    scan_impl(LoadI64{in}, out, n, total, s.part, st);
}

void scan_heads(const uint64_t *keys, int64_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st)
{
    scan_impl(Heads{keys}, out, n, total, s.part, st);
}

void scan_nonneg(const int32_t *a, int64_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st)
{
    scan_impl(NonNeg{a}, out, n, total, s.part, st);
}

void scan_tagged_weights(const int32_t *a, int32_t tag, const void *w, int wk, int64_t *out, int64_t n,
                         int64_t *total, Scratch &s, hipStream_t st)
{
    switch (wk) {
    case W_UNIT: scan_impl(TaggedWeight<W_UNIT>{a, w, tag}, out, n, total, s.part, st); break;
    case W_I32: scan_impl(TaggedWeight<W_I32>{a, w, tag}, out, n, total, s.part, st); break;
    default: scan_impl(TaggedWeight<W_I64>{a, w, tag}, out, n, total, s.part, st); break;
    }
}

// ---- radix sort -------------------------------------------------------------
// Digit counts of one tile.  The tile's keys are loaded before any is
// counted; the lanes of a wave that share a digit are found with ballots and
// only the first of them adds their number, so the LDS counters see one
// update per distinct digit of a round (the high digits of the rebuild's
// keys, C(u), are shared by whole runs of keys, which serialized per-key
// atomics on one counter).
__global__ __launch_bounds__(BLOCK) void k_radix_hist(const uint64_t *keys, int64_t n, int shift, int64_t *hist,
                                                      int64_t nb)
{
    __shared__ int32_t h[256];
    const int lane = threadIdx.x & 63;
    h[threadIdx.x] = 0;
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    uint64_t kr[RADIX_ITEMS];
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r) {
        const int64_t i = base + r * BLOCK + threadIdx.x;
        kr[r] = i < n ? keys[i] : 0;
    }
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r) {
        const bool valid = base + r * BLOCK + threadIdx.x < n;
        const int d = (int)((kr[r] >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        if (valid && (peers & lt_mask) == 0) atomicAdd(&h[d], __popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable rank of a tile's keys by the digit at `shift`.  Wave w holds the
// tile's keys [w * 64 * RADIX_ITEMS, (w + 1) * 64 * RADIX_ITEMS) in rounds of 64
// consecutive keys, so tile order is (wave, round, lane): each wave ranks its
// own keys with private digit counters (ballots find the lanes of a round
// that share a digit; the first of them updates the counter), then the
// counters are turned into per-wave offsets and digit starts with two block
// barriers in all.  Returns each key's tile position in pr (-1 past n) and
// the tile start of every digit in loc[0..256).
__device__ __forceinline__ void rank_tile(const uint64_t (&kr)[RADIX_ITEMS], int shift, int64_t base, int64_t n,
                                          int32_t (&pr)[RADIX_ITEMS], int32_t *loc, int32_t (*wcnt)[256],
                                          int32_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int32_t wr[RADIX_ITEMS];
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r) {
        const bool valid = base + (int64_t)wid * 64 * RADIX_ITEMS + r * 64 + lane < n;
        const int d = (int)((kr[r] >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt_mask);
        int32_t before = 0;
        if (valid && rank == 0) {
            before = wcnt[wid][d];
            wcnt[wid][d] = before + __popcll(peers);
        }
        const int leader = valid ? __ffsll((unsigned long long)peers) - 1 : lane;
        before = __shfl(before, leader, 64);
        wr[r] = valid ? before + rank : -1;
    }
    __syncthreads();
    {
        // digit tid: exclusive prefix over the waves, then over the digits
        int32_t tot = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            const int32_t c = wcnt[w][tid];
            wcnt[w][tid] = tot;
            tot += c;
        }
        int32_t inc = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        int32_t pre = inc - tot;
        for (int w = 0; w < wid; ++w) pre += wsum[w];
        loc[tid] = pre;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r) {
        const int d = (int)((kr[r] >> shift) & 255);
        pr[r] = wr[r] >= 0 ? loc[d] + wcnt[wid][d] + wr[r] : -1;
    }
}

// Key-only passes, one tile per block: the tile's keys are ranked (rank_tile),
// placed in LDS in digit order, and written out so that consecutive threads
// write consecutive positions of a digit's run instead of scattering every key.
__global__ __launch_bounds__(BLOCK) void k_radix_scatter_keys(const uint64_t *keys, int64_t n, int shift,
                                                             const int64_t *offs, int64_t nb, uint64_t *okeys)
{
    __shared__ uint64_t s_key[RADIX_TILE];
    __shared__ int64_t base_off[256]; // global start of digit d for this block
    __shared__ int32_t loc[256];      // local start of digit d in the tile
    __shared__ int32_t wcnt[BLOCK / 64][256];
    __shared__ int32_t wsum[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    base_off[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    const int64_t cnt = min((int64_t)RADIX_TILE, n - base);
    // the wave's keys, all loads issued before any is used
    uint64_t kr[RADIX_ITEMS];
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r) {
        const int64_t i = base + (int64_t)wid * 64 * RADIX_ITEMS + r * 64 + lane;
        kr[r] = i < n ? keys[i] : ~0ull;
    }
    int32_t pr[RADIX_ITEMS];
    rank_tile(kr, shift, base, n, pr, loc, wcnt, wsum);
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r)
        if (pr[r] >= 0) s_key[pr[r]] = kr[r];
    __syncthreads();
    // write out: position j of the tile holds digit d = its key's digit
    for (int32_t j = tid; j < cnt; j += BLOCK) {
        const uint64_t key = s_key[j];
        const int d = (int)((key >> shift) & 255);
        okeys[base_off[d] + (j - loc[d])] = key;
    }
}

// Key-value passes: the same ranking; keys, then values, go through one LDS
// staging buffer in digit order (tile positions kept in registers) so both
// are written out in runs.
__global__ __launch_bounds__(BLOCK) void k_radix_scatter_kv(const uint64_t *keys, const int64_t *vals, int64_t n,
                                                          int shift, const int64_t *offs, int64_t nb,
                                                          uint64_t *okeys, int64_t *ovals)
{
    __shared__ uint64_t s_buf[RADIX_TILE];
    __shared__ uint8_t s_dig[RADIX_TILE];
    __shared__ int64_t base_off[256];
    __shared__ int32_t loc[256];
    __shared__ int32_t wcnt[BLOCK / 64][256];
    __shared__ int32_t wsum[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    base_off[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    const int64_t cnt = min((int64_t)RADIX_TILE, n - base);
    uint64_t kr[RADIX_ITEMS];
    int64_t vr[RADIX_ITEMS];
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r) {
        const int64_t i = base + (int64_t)wid * 64 * RADIX_ITEMS + r * 64 + lane;
        kr[r] = i < n ? keys[i] : ~0ull;
        vr[r] = i < n ? vals[i] : 0;
    }
    int32_t pr[RADIX_ITEMS];
    rank_tile(kr, shift, base, n, pr, loc, wcnt, wsum);
    // keys
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r)
        if (pr[r] >= 0) {
            s_buf[pr[r]] = kr[r];
            s_dig[pr[r]] = (uint8_t)((kr[r] >> shift) & 255);
        }
    __syncthreads();
    for (int32_t j = tid; j < cnt; j += BLOCK) {
        const int d = s_dig[j];
        okeys[base_off[d] + (j - loc[d])] = s_buf[j];
    }
    __syncthreads();
    // values
#pragma unroll
    for (int r = 0; r < RADIX_ITEMS; ++r)
        if (pr[r] >= 0) s_buf[pr[r]] = (uint64_t)vr[r];
    __syncthreads();
    for (int32_t j = tid; j < cnt; j += BLOCK) {
        const int d = s_dig[j];
        ovals[base_off[d] + (j - loc[d])] = (int64_t)s_buf[j];
    }
}

int64_t radix_partials_needed(int64_t n)
{
    int64_t nb = (n + RADIX_TILE - 1) / RADIX_TILE;
    return 256 * nb + 16;
}

// hist region after the scan partials in s.part: s.part[hist_base ...]
__global__ __launch_bounds__(BLOCK) void k_copy_back(const uint64_t *src_k, uint64_t *keys, const int64_t *src_v,
                                                     int64_t *vals, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        keys[i] = src_k[i];
        if (src_v) vals[i] = src_v[i];
    }
}

void radix_sort(uint64_t *keys, uint64_t *keys_alt, int64_t *vals, int64_t *vals_alt, int64_t n, int bits,
                Scratch &s, hipStream_t st)
{
    if (n <= 1 || bits <= 0) return;
    const int64_t nb = (n + RADIX_TILE - 1) / RADIX_TILE;
    int64_t *hist = s.part;
    int64_t *part = s.part + 256 * nb + 8;
    uint64_t *src_k = keys, *dst_k = keys_alt;
    int64_t *src_v = vals, *dst_v = vals_alt;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_radix_hist<<<(unsigned)nb, BLOCK, 0, st>>>(src_k, n, shift, hist, nb);
        scan_impl(LoadI64{hist}, hist, 256 * nb, (int64_t *)nullptr, part, st);
        if (vals)
            k_radix_scatter_kv<<<(unsigned)nb, BLOCK, 0, st>>>(src_k, src_v, n, shift, hist, nb, dst_k, dst_v);
        else
            k_radix_scatter_keys<<<(unsigned)nb, BLOCK, 0, st>>>(src_k, n, shift, hist, nb, dst_k);
        uint64_t *tk = src_k; src_k = dst_k; dst_k = tk;
        int64_t *tv = src_v; src_v = dst_v; dst_v = tv;
    }
    if (src_k != keys) {
        // an odd number of passes ends in the alternate buffers: copied back
        // by a kernel, so that a failure shows in the caller's launch check
        unsigned gc = grid_for(n, BLOCK * 8);
        if (gc > 65536) gc = 65536;
        k_copy_back<<<gc, BLOCK, 0, st>>>(src_k, keys, vals ? src_v : nullptr, vals, n);
    }
}

// ---- fills --------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(T *p, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) p[i] = v;
}

template <typename T> void fill(T *p, T v, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    unsigned g = grid_for(n, BLOCK * 8);
    if (g > 65536) g = 65536;
    k_fill<T><<<g, BLOCK, 0, st>>>(p, v, n);
}
template void fill<int32_t>(int32_t *, int32_t, int64_t, hipStream_t);
template void fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);
template void fill<uint64_t>(uint64_t *, uint64_t, int64_t, hipStream_t);

__global__ __launch_bounds__(BLOCK) void k_iota(int32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        p[i] = (int32_t)i;
}

void iota_i32(int32_t *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    unsigned g = grid_for(n, BLOCK * 8);
    if (g > 65536) g = 65536;
    k_iota<<<g, BLOCK, 0, st>>>(p, n);
}

} // namespace lv
