// pic_bin.hip -- binning of particles into cells (Coulombic collision steps
// CCS1-CCS3): order check, cell starts, and a stable LSD counting sort by
// cell id that moves the particle data itself.
//
// The paper builds an index list with one atomic increment per particle and
// notes that those atomics cost up to 40% of its Coulomb kernel.  Here the
// storage is kept in cell order between steps, so the steady state is a
// single streaming check of cell_of (4 B per particle); only unsorted input
// runs the sort passes, which rank elements inside a wave with ballots
// instead of atomics, so the result is stable and deterministic.
#include <string.h>

#include "pic_internal.hpp"

#define HIP_OK(x) do { if ((x) != hipSuccess) return PIC_ERR_HIP; } while (0)

namespace {

constexpr int RS_THREADS = 256;   // radix kernels: 4 waves
constexpr int RS_ITEMS = 16;      // rounds per tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

__global__ void k_reset_flags(DevFlags *f)
{
    if (threadIdx.x == 0) {
        f->unsorted = 0;
        f->range_err = 0;
        f->huge_total = 0;
        f->seg_fallback = 0;
    }
    if (threadIdx.x < 8) {
        f->head[threadIdx.x] = 0;
        f->count[threadIdx.x] = 0;
    }
}

// Any non-finite component of v latches PIC_ERR_NONFINITE (a debug check:
// one streaming read of the velocities).
template <typename R>
__global__ void k_check_finite(const R *__restrict__ v, int64_t m, DevFlags *f)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(v[i]);
    if (__ballot(bad) && (threadIdx.x & (PIC_WAVE - 1)) == 0) atomicOr(&f->sticky_nonfinite, 1);
}

// Latches PIC_ERR_STATE when work list `list` holds any cell.
__global__ void k_reject_list(DevFlags *f, int list)
{
    if (threadIdx.x == 0 && f->count[list] != 0u) f->sticky_state = 1;
}

__global__ void k_set_step(uint64_t *s, uint64_t v)
{
    if (threadIdx.x == 0) *s = v;
}

__global__ void k_step_inc(uint64_t *s)
{
    if (threadIdx.x == 0) *s += 1;
}

// Position i in [0, n] is the boundary between element i-1 and i: every cell
// id j in (cell_of[i-1], cell_of[i]] starts at i, so with sorted input each
// entry of cell_start is written exactly once (empty cells included).  Each
// thread takes four consecutive positions (one 16-byte load when aligned).
__global__ void k_bin_check(const int32_t *__restrict__ cell_of, int64_t n, int32_t n_cells,
                            int32_t *__restrict__ cell_start, DevFlags *f, int set_unsorted,
                            const int *gate)
{
    if (gate && *gate == 0) return;
    int bad = 0, uns = 0;
    const int64_t nq = n / 4 + 1;
    const bool vec = ((uintptr_t)cell_of & 15u) == 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i0 = q * 4;
        int32_t c[5];
        c[0] = i0 > 0 ? cell_of[i0 - 1] : -1;
        if (vec && i0 + 4 <= n) {
            const int4 x = *(const int4 *)(cell_of + i0);
            c[1] = x.x;
            c[2] = x.y;
            c[3] = x.z;
            c[4] = x.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) c[1 + j] = i0 + j < n ? cell_of[i0 + j] : n_cells;
        }
        bool out[4], desc = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j;
            out[j] = i < n && (c[1 + j] < 0 || c[1 + j] >= n_cells);
            desc |= i > 0 && i < n && c[1 + j] < c[j];
            bad |= out[j];
        }
        uns |= desc;
        // A wave whose elements are out of order writes no starts: the input
        // is unsorted, gets sorted, and the starts are written by the check
        // that follows the sort.  Without this, shuffled input would cost a
        // write per cell for every ascending neighbour pair.
        if (set_unsorted && __ballot(desc) != 0) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j;
            if (i > n || out[j]) continue;
            const int32_t cur = c[1 + j];
            const int32_t lo = c[j] + 1 < 0 ? 0 : c[j] + 1;
            for (int32_t k = lo; k <= cur && k <= n_cells; ++k) cell_start[k] = (int32_t)i;
        }
    }
    const uint64_t wb = __ballot(bad), wu = __ballot(uns);
    if ((threadIdx.x & (PIC_WAVE - 1)) == 0) {
        if (wb) {
            atomicOr(&f->range_err, 1);
            atomicOr(&f->sticky_range, 1);
        }
        if (wu && set_unsorted) {
            atomicOr(&f->unsorted, 1);
            if (set_unsorted == 2) atomicOr(&f->sticky_state, 1);
        }
    }
}

__global__ void k_copy32(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src, int64_t n,
                         const int *gate)
{
    if (gate && *gate == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__device__ __forceinline__ uint32_t digit_of(int32_t key, int shift, int bits)
{
    return ((uint32_t)key >> shift) & ((1u << bits) - 1u);
}

// Per-tile digit counts: hist[d * nblocks + tile].
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(RadixPass p, uint32_t *__restrict__ hist)
{
    if (p.gate && *p.gate == 0) return;
    __shared__ uint32_t h[256];
    const int R = 1 << p.bits;
    for (int d = threadIdx.x; d < R; d += RS_THREADS) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t e = base + r * RS_THREADS + threadIdx.x;
        if (e < p.n) atomicAdd(&h[digit_of(p.key_in[e], p.shift, p.bits)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += RS_THREADS) hist[(int64_t)d * gridDim.x + blockIdx.x] = h[d];
}

// Exclusive scan of SCAN_ITEMS consecutive values per thread over the block;
// returns the thread's exclusive prefix and (in *total) the block total.
__device__ uint32_t block_excl_scan(uint32_t x, uint32_t *total)
{
    __shared__ uint32_t wtot[SCAN_THREADS / PIC_WAVE];
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == PIC_WAVE - 1) wtot[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int w = 0; w < SCAN_THREADS / PIC_WAVE; ++w) {
        if (w < wid) off += wtot[w];
        tot += wtot[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t *__restrict__ a, int64_t L,
                                                             uint32_t *__restrict__ bsum,
                                                             const int *gate)
{
    if (gate && *gate == 0) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < L) s += a[base + k];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(uint32_t *__restrict__ bsum, int64_t nb,
                                                          const int *gate)
{
    if (gate && *gate == 0) return;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_CHUNK) {
        const int64_t b0 = base + threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS], s = 0;
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            v[k] = b0 + k < nb ? bsum[b0 + k] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t off = block_excl_scan(s, &tot) + carry;
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (b0 + k < nb) bsum[b0 + k] = off;
            off += v[k];
        }
        carry += tot;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(uint32_t *__restrict__ a, int64_t L,
                                                           const uint32_t *__restrict__ bsum,
                                                           const int *gate)
{
    if (gate && *gate == 0) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS], s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < L ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < L) a[base + k] = off;
        off += v[k];
    }
}

// Stable scatter.  The tile is visited in element order, RS_THREADS elements
// per round; within a round an element's rank among equal digits is
// (count in earlier rounds) + (count in earlier waves) + (earlier lanes of
// its own wave), the last found from ballots over the digit bits.
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(RadixPass p,
                                                              const uint32_t *__restrict__ offs)
{
    if (p.gate && *p.gate == 0) return;
    constexpr int NW = RS_THREADS / PIC_WAVE;
    __shared__ uint32_t base[256];
    __shared__ uint32_t wc[NW * 256];
    __shared__ uint32_t goff[256];
    const int R = 1 << p.bits;
    for (int d = threadIdx.x; d < R; d += RS_THREADS) {
        base[d] = 0;
        goff[d] = offs[(int64_t)d * gridDim.x + blockIdx.x];
        for (int w = 0; w < NW; ++w) wc[w * 256 + d] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (PIC_WAVE - lane));
    const int64_t tile = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t e = tile + r * RS_THREADS + threadIdx.x;
        const bool valid = e < p.n;
        const int32_t key = valid ? p.key_in[e] : 0;
        const uint32_t d = digit_of(key, p.shift, p.bits);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < p.bits; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[wid * 256 + d] = __popcll(peers);
        __syncthreads();
        uint32_t pos = 0;
        if (valid) {
            pos = base[d] + rank;
            for (int w = 0; w < wid; ++w) pos += wc[w * 256 + d];
        }
        __syncthreads();
        for (int dd = threadIdx.x; dd < R; dd += RS_THREADS) {
            uint32_t s = 0;
            for (int w = 0; w < NW; ++w) {
                s += wc[w * 256 + dd];
                wc[w * 256 + dd] = 0;
            }
            base[dd] += s;
        }
        if (valid) {
            const int64_t o = (int64_t)goff[d] + pos;
            p.key_out[o] = key;
            for (int s = 0; s < p.n32; ++s)
                p.p32_out[s][o] = (s == p.iota_slot) ? (uint32_t)e : p.p32_in[s][e];
            for (int s = 0; s < p.n64; ++s) p.p64_out[s][o] = p.p64_in[s][e];
        }
        __syncthreads();
    }
}

// Stable scatter with the tile staged in LDS (tiles of RS_TILE elements, so
// the per-tile digit counts of k_radix_hist apply).  Wave w takes elements
// [w * 256, w * 256 + 256) of the tile in four rounds of 64; an element's rank
// among equal digits of its wave comes from ballots over the digit bits and a
// per-wave running count in LDS (no block barrier while ranking).  The waves'
// counts then give each (wave, digit) its start inside the tile, every element
// goes to its place in a digit-sorted copy of the tile in LDS, and the copy is
// written out in slot order: consecutive slots of one digit go to consecutive
// addresses, so the stores are coalesced runs instead of one scattered word
// per element and array.
constexpr int RS2_THREADS = 1024;
constexpr int RS2_WAVES = RS2_THREADS / PIC_WAVE;
constexpr int RS2_PER_WAVE = RS_TILE / RS2_WAVES;          // 256 elements
constexpr int RS2_ROUNDS = RS2_PER_WAVE / PIC_WAVE;         // 4
static_assert(RS2_ROUNDS * PIC_WAVE * RS2_WAVES == RS_TILE, "tile split");

// Dynamic LDS of the staged scatter (its static part is about 21 KB).
constexpr size_t RS2_LDS_MAX = 136 * 1024;

size_t rs2_stage_bytes(int n32, int n64)
{
    return (size_t)RS_TILE * (4 + 4 * (size_t)n32 + 8 * (size_t)n64);
}

__global__ __launch_bounds__(RS2_THREADS) void k_radix_scatter_lds(RadixPass p,
                                                                   const uint32_t *__restrict__ offs)
{
    if (p.gate && *p.gate == 0) return;
    extern __shared__ __align__(16) unsigned char stage[];
    __shared__ uint32_t run[RS2_WAVES * 256];   // per-wave running digit counts, then wave starts
    __shared__ uint32_t tstart[257];            // digit starts inside the tile
    __shared__ uint32_t goff[256];              // global start of this tile's run of each digit
    const int R = 1 << p.bits;
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (PIC_WAVE - lane));
    const int64_t tile = (int64_t)blockIdx.x * RS_TILE;
    const int64_t tn = p.n - tile < RS_TILE ? p.n - tile : RS_TILE;   // elements in this tile
    uint32_t *skey = (uint32_t *)stage;
    uint32_t *s32 = skey + RS_TILE;
    uint64_t *s64 = (uint64_t *)(s32 + (size_t)p.n32 * RS_TILE);
    for (int q = threadIdx.x; q < RS2_WAVES * 256; q += RS2_THREADS) run[q] = 0;
    if (threadIdx.x < R) goff[threadIdx.x] = offs[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    // digit starts inside the tile from this tile's counts (one wave scans):
    // the offsets are an exclusive scan over (digit, tile), so a tile's count
    // of a digit is the next offset minus its own (the total after the last)
    if (wid == 0) {
        const int64_t L = (int64_t)R * gridDim.x;
        uint32_t carry = 0;
        for (int d0 = 0; d0 < R; d0 += PIC_WAVE) {
            const int d = d0 + lane;
            uint32_t c = 0;
            if (d < R) {
                const int64_t idx = (int64_t)d * gridDim.x + blockIdx.x;
                c = (idx + 1 < L ? offs[idx + 1] : (uint32_t)p.n) - offs[idx];
            }
            const uint32_t inc = wave_incl_scan(c);
            if (d < R) tstart[d] = carry + inc - c;
            carry += __shfl(inc, PIC_WAVE - 1, PIC_WAVE);
        }
        if (lane == 0) tstart[R] = carry;
    }
    // this thread's elements: round r is element wid * 256 + r * 64 + lane
    int32_t key[RS2_ROUNDS];
    uint32_t rank[RS2_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS2_ROUNDS; ++r) {
        const int64_t le = (int64_t)wid * RS2_PER_WAVE + r * PIC_WAVE + lane;
        key[r] = le < tn ? p.key_in[tile + le] : 0;
    }
    __syncthreads();
    uint32_t *wrun = run + wid * 256;
#pragma unroll
    for (int r = 0; r < RS2_ROUNDS; ++r) {
        const int64_t le = (int64_t)wid * RS2_PER_WAVE + r * PIC_WAVE + lane;
        const bool valid = le < tn;
        const uint32_t d = digit_of(key[r], p.shift, p.bits);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < p.bits; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t before = valid ? wrun[d] : 0u;
        rank[r] = before + __popcll(peers & lt);
        // the group's first lane advances the wave's count (same wave: LDS
        // operations stay in order)
        if (valid && (peers & lt) == 0ull) wrun[d] = before + __popcll(peers);
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the count is in LDS
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // wave starts per digit: tile start + the earlier waves' counts
    for (int d = threadIdx.x; d < R; d += RS2_THREADS) {
        uint32_t acc = tstart[d];
        for (int w = 0; w < RS2_WAVES; ++w) {
            const uint32_t c = run[w * 256 + d];
            run[w * 256 + d] = acc;
            acc += c;
        }
    }
    __syncthreads();
    // stage every element at its place in the digit-sorted tile
#pragma unroll
    for (int r = 0; r < RS2_ROUNDS; ++r) {
        const int64_t le = (int64_t)wid * RS2_PER_WAVE + r * PIC_WAVE + lane;
        if (le < tn) {
            const int64_t e = tile + le;
            const uint32_t d = digit_of(key[r], p.shift, p.bits);
            const uint32_t q = wrun[d] + rank[r];
            skey[q] = (uint32_t)key[r];
            for (int s = 0; s < p.n32; ++s)
                s32[(size_t)s * RS_TILE + q] = (s == p.iota_slot) ? (uint32_t)e : p.p32_in[s][e];
            for (int s = 0; s < p.n64; ++s) s64[(size_t)s * RS_TILE + q] = p.p64_in[s][e];
        }
    }
    __syncthreads();
    // write out in slot order
    for (int q = threadIdx.x; q < tn; q += RS2_THREADS) {
        const uint32_t k = skey[q];
        const uint32_t d = digit_of((int32_t)k, p.shift, p.bits);
        const int64_t o = (int64_t)goff[d] + (q - (int64_t)tstart[d]);
        p.key_out[o] = (int32_t)k;
        for (int s = 0; s < p.n32; ++s) p.p32_out[s][o] = s32[(size_t)s * RS_TILE + q];
        for (int s = 0; s < p.n64; ++s) p.p64_out[s][o] = s64[(size_t)s * RS_TILE + q];
    }
}

// Cells by size class.  lists[c * n_cells + k] = k-th cell of class c; the
// class lengths go to flags->count[c]; flags->huge_total sums the members of
// cells beyond the largest LDS class.  Within a class the order is
// arbitrary: cells are independent and their random numbers depend only on
// (seed, step, pid), so processing order never changes results.  Cells the
// gate defers go to the deferred list when they still need a visit.
// Segment plan of cell h of the multi-workgroup list with cnt members:
// S = ceil(cnt / target) segments (equal key ranges), their table entries,
// and the counting work items.  Segment and item ranges are reserved with atomics:
// where a cell's entries sit never changes results.
__device__ void plan_segments(const SegScratch &ss, DevFlags *f, int h, int32_t cnt, int target)
{
    const int64_t want = ((int64_t)cnt + target - 1) / target;
    if (want > SEG_MAX) {
        ss.hc_fb[h] = 1;
        ss.hc_S[h] = 0;
        f->seg_fallback = 1;
        return;
    }
    const uint32_t S = want > 0 ? (uint32_t)want : 1u;
    const uint32_t nch = (uint32_t)(((int64_t)cnt + SEG_CHUNK - 1) / SEG_CHUNK);
    const uint32_t sb = atomicAdd(&f->count[SEG_SLOT], S);
    const uint32_t cb = atomicAdd(&f->count[CHUNK_SLOT], nch);
    ss.hc_fb[h] = 0;
    ss.hc_S[h] = S;
    ss.hc_seg[h] = (int32_t)sb;
    ss.hc_chunk[h] = (int32_t)cb;
    for (uint32_t q = 0; q < S; ++q) {
        ss.sg_cell[sb + q] = h;
        ss.sg_cnt[sb + q] = 0;
        ss.bnd_head[sb + q] = -1;
        ss.bnd_tail[sb + q] = -1;
    }
    for (uint32_t q = 0; q < nch; ++q) ss.ch_owner[cb + q] = h;
}

__global__ void k_build_queue(const int32_t *__restrict__ cell_start, int32_t n_cells, ClassCaps caps,
                              int32_t *__restrict__ lists, DevFlags *f,
                              const uint8_t *__restrict__ skip, int visit, SegScratch ss,
                              int plan, int seg_target)
{
    const int lane = threadIdx.x & (PIC_WAVE - 1);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (PIC_WAVE - lane));
    for (int64_t j0 = blockIdx.x * (int64_t)blockDim.x; j0 < n_cells;
         j0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        const bool valid = j < n_cells;
        int cls = -1;
        int32_t cnt = 0;
        if (valid) {
            // every cell is visited: cells with fewer than two members still
            // need the null-collision step and their moment sums
            cnt = cell_start[j + 1] - cell_start[j];
            cls = caps.ncls;
            for (int c = caps.ncls - 1; c >= 0; --c)
                if (cnt <= caps.cap[c]) cls = c;
            if (skip && skip[j]) cls = visit ? LIST_DEFERRED : -1;
        }
        for (int c = 0; c < QUEUE_LISTS; ++c) {
            const uint64_t m = __ballot(cls == c);
            if (!m) continue;
            const int leader = __ffsll((unsigned long long)m) - 1;
            uint32_t b = 0;
            if (lane == leader) b = atomicAdd(&f->count[c], (uint32_t)__popcll(m));
            b = __shfl(b, leader, PIC_WAVE);
            if (cls == c) {
                const int h = (int)b + __popcll(m & lt);
                lists[(int64_t)c * n_cells + h] = (int32_t)j;
                if (plan && c == caps.ncls) plan_segments(ss, f, h, cnt, seg_target);
            }
        }
        if (cls == caps.ncls) atomicAdd(&f->huge_total, (uint32_t)cnt);
    }
}

int grid_for(int64_t n, int threads, int cap)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

int launch_reset_flags(DevFlags *flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_flags, dim3(1), dim3(64), 0, st, flags);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_check_finite(int dtype, const void *v, int64_t n, DevFlags *flags, hipStream_t st)
{
    if (n <= 0) return PIC_OK;
    const int g = grid_for(3 * n, 256, 4096);
    if (dtype == PIC_F32)
        hipLaunchKernelGGL(k_check_finite<float>, dim3(g), dim3(256), 0, st, (const float *)v, 3 * n, flags);
    else
        hipLaunchKernelGGL(k_check_finite<double>, dim3(g), dim3(256), 0, st, (const double *)v, 3 * n, flags);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_reject_list(DevFlags *flags, int list, hipStream_t st)
{
    hipLaunchKernelGGL(k_reject_list, dim3(1), dim3(64), 0, st, flags, list);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_set_step(uint64_t *step_dev, uint64_t value, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, st, step_dev, value);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_step_inc(uint64_t *step_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, st, step_dev);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_bin_check(const int32_t *cell_of, int64_t n, int32_t n_cells, int32_t *cell_start,
                     DevFlags *flags, int set_unsorted, const int *gate, hipStream_t st)
{
    hipLaunchKernelGGL(k_bin_check, dim3(grid_for(n / 4 + 1, 256, 8192)), dim3(256), 0, st, cell_of, n,
                       n_cells, cell_start, flags, set_unsorted, gate);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_copy32(uint32_t *dst, const uint32_t *src, int64_t n, const int *gate, hipStream_t st)
{
    if (n <= 0) return PIC_OK;
    hipLaunchKernelGGL(k_copy32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, dst, src, n, gate);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

size_t radix_scratch_bytes(int64_t n)
{
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE + 1;
    const int64_t L = 256 * nb;
    const int64_t ns = (L + SCAN_CHUNK - 1) / SCAN_CHUNK + 1;
    return (size_t)(L + ns) * sizeof(uint32_t) + 512;
}

int radix_pass(const RadixPass &p, const BinScratch &s, hipStream_t st)
{
    if (p.n <= 0) return PIC_OK;
    const int64_t nb = (p.n + RS_TILE - 1) / RS_TILE;
    const int64_t L = (int64_t)(1 << p.bits) * nb;
    const int64_t ns = (L + SCAN_CHUNK - 1) / SCAN_CHUNK;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(RS_THREADS), 0, st, p, s.hist);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ns), dim3(SCAN_THREADS), 0, st, s.hist, L, s.bsum,
                       p.gate);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, st, s.bsum, ns, p.gate);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)ns), dim3(SCAN_THREADS), 0, st, s.hist, L, s.bsum,
                       p.gate);
    const size_t lds = rs2_stage_bytes(p.n32, p.n64);
    if (lds <= RS2_LDS_MAX) {
        static size_t attr_set = 0;
        if (lds > attr_set) {
            HIP_OK(hipFuncSetAttribute((const void *)k_radix_scatter_lds,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            attr_set = lds;
        }
        hipLaunchKernelGGL(k_radix_scatter_lds, dim3((unsigned)nb), dim3(RS2_THREADS), lds, st, p,
                           (const uint32_t *)s.hist);
    } else {
        // a tile of this many payload words does not fit: one word per element and array
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(RS_THREADS), 0, st, p,
                           (const uint32_t *)s.hist);
    }
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_build_queue(const int32_t *cell_start, int32_t n_cells, const ClassCaps &caps,
                       int32_t *lists, DevFlags *flags, const uint8_t *skip, int visit,
                       const SegScratch *seg, int seg_target, hipStream_t st)
{
    SegScratch ss;
    memset(&ss, 0, sizeof(ss));
    if (seg) ss = *seg;
    hipLaunchKernelGGL(k_build_queue, dim3(grid_for(n_cells, 256, 1024)), dim3(256), 0, st,
                       cell_start, n_cells, caps, lists, flags, skip, visit, ss, seg ? 1 : 0,
                       seg_target);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}
