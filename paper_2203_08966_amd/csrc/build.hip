// Octree construction on gfx950 (Barnes-Hut loop body, Sec. 3, build step).
//
//  1. bbox + root cube     per-block FP64 min/max, then one block snaps the
//                          root cube (power-of-two side, corner on L/2 grid)
//  2. keys + histograms    21-bit quantisation per axis in FP64, bit-spread
//                          interleave x > y > z (Sec. 4.4); the same pass
//                          counts all eight 8-bit digits of every key
//  3. LDS radix sort       eight stable passes; each pass ranks a 4096-key
//                          tile in LDS (wave-level match via ballots),
//                          finds its global offsets by decoupled look-back,
//                          reorders the tile in LDS and writes runs
//  4. gather               bodies into key order
//  5. topology             bottom-up from adjacent-key common prefixes: each
//                          sorted rank s starts the chain of cells whose
//                          first body it is; a scan of the chain lengths
//                          places every cell in pre-order (Sec. 4.2)
//  6. upward pass (FP64)   leaves from their bodies (with the child table
//                          and the leaf-relative body records), internal
//                          cells level by level, deepest first, from their
//                          children's moments about the cell centre; each
//                          node's FP32/FP64 walk record is written as soon
//                          as its moments are final
#include <float.h>
#include <limits.h>
#include <math.h>
#include <string.h>

#include "bh_internal.h"

namespace bh {
namespace {

constexpr int kSortThreads = 1024;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys
constexpr int kWaveTile = 64 * kSortItems;            // 1024 keys per wave
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;      // 2048

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// popcount(mask & lanes-below-me)
__device__ __forceinline__ unsigned rank_in(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// ------------------------------------------------------------------ zero fill
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------ 1. bbox
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bbox(const T *__restrict__ pos, int n,
                                                   double *__restrict__ part) {
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = (double)pos[3 * (int64_t)i + d];
            bad |= !isfinite(v);
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    }
    __shared__ double sh[6][kThreads / 64];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        for (int o = 32; o > 0; o >>= 1) {
            mn[d] = fmin(mn[d], __shfl_xor(mn[d], o));
            mx[d] = fmax(mx[d], __shfl_xor(mx[d], o));
        }
    }
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) {
        for (int d = 0; d < 3; ++d) {
            sh[d][w] = mn[d];
            sh[3 + d][w] = mx[d];
        }
    }
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    if (ballot(bad) != 0 && lane_id() == 0) bad_s = 1;
    __syncthreads();
    if (threadIdx.x < 6) {
        const int d = threadIdx.x;
        double v = sh[d][0];
        for (int k = 1; k < kThreads / 64; ++k) v = d < 3 ? fmin(v, sh[d][k]) : fmax(v, sh[d][k]);
        part[7 * blockIdx.x + d] = v;
    }
    if (threadIdx.x == 6) part[7 * blockIdx.x + 6] = bad_s ? 1.0 : 0.0;
}

// One block: reduce the partials and snap the root cube; also starts the
// build's flags word (bit 0: a non-finite position).  Same rule as the
// method's definition: smallest power-of-two side L such that, with the
// corner at floor(min / (L/2)) * (L/2), max < corner + L in every axis.
__global__ __launch_bounds__(kThreads) void k_cube(const double *__restrict__ part, int np,
                                                   Cube *__restrict__ cube,
                                                   Cube *__restrict__ mirror,
                                                   uint32_t *__restrict__ flags) {
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool bad = false;
    for (int b = threadIdx.x; b < np; b += blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            mn[d] = fmin(mn[d], part[7 * b + d]);
            mx[d] = fmax(mx[d], part[7 * b + 3 + d]);
        }
        bad |= part[7 * b + 6] != 0.0;
    }
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    if (ballot(bad) != 0 && lane_id() == 0) bad_s = 1;
    for (int d = 0; d < 3; ++d)
        for (int o = 32; o > 0; o >>= 1) {
            mn[d] = fmin(mn[d], __shfl_xor(mn[d], o));
            mx[d] = fmax(mx[d], __shfl_xor(mx[d], o));
        }
    __shared__ double sh[6][kThreads / 64];
    const int w = threadIdx.x / 64;
    if (lane_id() == 0)
        for (int d = 0; d < 3; ++d) {
            sh[d][w] = mn[d];
            sh[3 + d][w] = mx[d];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        *flags = bad_s ? 1u : 0u;
        for (int d = 0; d < 3; ++d) {
            for (int k = 1; k < kThreads / 64; ++k) {
                sh[d][0] = fmin(sh[d][0], sh[d][k]);
                sh[3 + d][0] = fmax(sh[3 + d][0], sh[3 + d][k]);
            }
            mn[d] = sh[d][0];
            mx[d] = sh[3 + d][0];
        }
        double ext = 0.0;
        for (int d = 0; d < 3; ++d) ext = fmax(ext, mx[d] - mn[d]);
        double L = 1.0;
        if (ext > 0.0) {
            int e;
            frexp(ext, &e);
            L = ldexp(1.0, e - 1);
        }
        double lo[3];
        for (;;) {
            const double half = 0.5 * L;
            bool ok = true;
            for (int d = 0; d < 3; ++d) {
                lo[d] = floor(mn[d] / half) * half;
                ok = ok && (mx[d] < lo[d] + L);
            }
            if (ok) break;
            L *= 2.0;
        }
        for (int d = 0; d < 3; ++d) cube->lo[d] = mirror->lo[d] = lo[d];
        cube->L = mirror->L = L;
    }
}

// ------------------------------------------------------------------ 2. keys
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x001f00000000ffffull;
    x = (x | x << 16) & 0x001f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}
__device__ __forceinline__ uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x001f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x001f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x00000000001fffffull;
    return (uint32_t)x;
}
// Peano-Hilbert index of the integer point (qx, qy, qz), 21 bits per axis
// (Sec. 4.4 names the curve as the remedy for the Morton order's jumps).
// Butz's construction, level by level from the top: the point's three bits
// at the level (x in bit 0) are reflected through the current cube's entry
// corner e and rotated right by d + 1 places, which carries the cube's curve
// onto the standard one; the sub-cube's rank w is then their inverse Gray
// code and the next octal digit of the index; the sub-cube's curve enters
// at corner E(w) (rotated left by d + 1 into the cube's frame, then added to
// e) and d grows by D(w) + 1 modulo 3.  E(w) is the Gray code of the largest
// even number below w (0 for w = 0): 0 0 0 3 3 6 6 5; D(w) counts the
// trailing ones of w - 1 (w even) or of w (w odd), modulo 3: 0 1 1 2 2 1 1 0.
// Both are packed in one word each, 3 and 2 bits per entry.
constexpr uint32_t kHbEntry = (0u << 0) | (0u << 3) | (0u << 6) | (3u << 9) | (3u << 12) |
                              (6u << 15) | (6u << 18) | (5u << 21);
constexpr uint32_t kHbAxis = (0u << 0) | (1u << 2) | (1u << 4) | (2u << 6) | (2u << 8) |
                             (1u << 10) | (1u << 12) | (0u << 14);
__device__ __forceinline__ uint32_t rot3r(uint32_t x, uint32_t r) {  // r in 0..2
    return ((x >> r) | (x << (3u - r))) & 7u;
}
__device__ __forceinline__ uint32_t rot3l(uint32_t x, uint32_t r) {
    return ((x << r) | (x >> (3u - r))) & 7u;
}
// One level: state s = 3 e + d, the level's three bits l; returns the next
// state and the digit w.
__device__ __forceinline__ uint32_t hb_step(uint32_t s, uint32_t l, uint32_t &w) {
    uint32_t e = s / 3u, d = s - 3u * (s / 3u);
    const uint32_t t = rot3r(l ^ e, d == 2 ? 0u : d + 1u);
    w = t ^ (t >> 1) ^ (t >> 2);
    e ^= rot3l((kHbEntry >> (3u * w)) & 7u, d == 2 ? 0u : d + 1u);
    d += ((kHbAxis >> (2u * w)) & 3u) + 1u;
    d = d >= 3u ? d - 3u : d;
    d = d >= 3u ? d - 3u : d;
    return 3u * e + d;
}
// Two levels per lookup: entry 64 s + (l_hi << 3 | l_lo) of this table
// holds the two digits (6 bits) and the state after them (bits 6..10), for
// the 24 states; filled by the threads of a workgroup from hb_step.
constexpr int kHbTable = 24 * 64;
__device__ __forceinline__ void hb_table_fill(uint16_t *tab, int t, int nt) {
    for (int idx = t; idx < kHbTable; idx += nt) {
        uint32_t w1, w2;
        const uint32_t s1 = hb_step((uint32_t)idx >> 6, ((uint32_t)idx >> 3) & 7u, w1);
        const uint32_t s2 = hb_step(s1, (uint32_t)idx & 7u, w2);
        tab[idx] = (uint16_t)((w1 << 3) | w2 | (s2 << 6));
    }
}
__device__ __forceinline__ uint64_t hilbert3_tab(uint32_t qx, uint32_t qy, uint32_t qz,
                                                 const uint16_t *tab) {
    // the point's three bits of every level i in bits 3i .. 3i + 2 (x in the
    // lowest), so that two levels' bits are one 6-bit field
    const uint64_t b = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
    uint32_t w;
    uint32_t s = hb_step(0u, (uint32_t)(b >> (3 * (kLevels - 1))) & 7u, w);  // the top level alone
    uint64_t h = w;
#pragma unroll
    for (int i = kLevels - 2; i > 0; i -= 2) {  // levels i and i - 1
        const uint32_t v = tab[64u * s + ((uint32_t)(b >> (3 * (i - 1))) & 63u)];
        h = (h << 6) | (v & 63u);
        s = v >> 6;
    }
    return h;
}
__device__ __forceinline__ uint32_t quantise(double x, double lo, double scale) {
    double t = __dmul_rn(__dsub_rn(x, lo), scale);
    double f = floor(t);
    f = f < 0.0 ? 0.0 : f;
    f = f > 2097151.0 ? 2097151.0 : f;
    return (uint32_t)f;
}

// Keys (pos not NULL: computed and stored; NULL: read), and (hist not
// NULL) the counts of every 8-bit digit of every key (8 x 256 bins) that
// the full radix sort takes: a block histogram in LDS, added to the global
// one bin by bin.  Few large blocks keep the global adds few.
constexpr int kKeyThreads = 1024;
constexpr int kKeyBlocks = 256;
template <typename T>
__global__ __launch_bounds__(kKeyThreads) void k_keys(const T *__restrict__ pos, int n,
                                                      const Cube *__restrict__ cube,
                                                      uint64_t *__restrict__ keys,
                                                      uint32_t *__restrict__ hist, int curve) {
    __shared__ uint32_t h[8][256];
    __shared__ uint16_t hb_tab[kHbTable];
    if (hist)
        for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) (&h[0][0])[i] = 0;
    if (pos && curve == BH_CURVE_HILBERT) hb_table_fill(hb_tab, threadIdx.x, blockDim.x);
    __syncthreads();
    const double lx = cube->lo[0], ly = cube->lo[1], lz = cube->lo[2];
    const double scale = ldexp(1.0, kLevels) / cube->L;
    const unsigned lane = lane_id();
    const int stride = gridDim.x * blockDim.x;
    const int iters = (n + stride - 1) / stride;
    for (int it = 0; it < iters; ++it) {
        const int i = it * stride + blockIdx.x * blockDim.x + threadIdx.x;
        const bool valid = i < n;
        uint64_t k = 0;
        if (valid && !pos) {
            k = keys[i];
        } else if (valid) {
            const int64_t b = 3 * (int64_t)i;
            const uint32_t qx = quantise((double)pos[b + 0], lx, scale),
                           qy = quantise((double)pos[b + 1], ly, scale),
                           qz = quantise((double)pos[b + 2], lz, scale);
            k = curve == BH_CURVE_HILBERT ? hilbert3_tab(qx, qy, qz, hb_tab)
                                          : (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
            keys[i] = k;
        }
        if (!hist) continue;
        const uint64_t live = ballot(valid);
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t d = (uint32_t)(k >> (8 * p)) & 255u;
            // neighbouring bodies (input in curve order) share most digits:
            // up to two distinct digit values are counted with one add each
            uint64_t rem = live;
            for (int r = 0; r < 2 && rem; ++r) {
                const int l0 = __builtin_ctzll(rem);
                const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, l0);
                const uint64_t same = ballot(d == d0) & rem;
                if ((int)lane == l0) atomicAdd(&h[p][d0], (uint32_t)__popcll(same));
                rem &= ~same;
            }
            if ((rem >> lane) & 1ull) atomicAdd(&h[p][d], 1u);
        }
    }
    if (!hist) return;
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) {
        const uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

// Exclusive scan of each pass's 256-bin histogram (8 blocks x 256 threads);
// also clears the per-pass tile counters, and the histogram for the next
// build.
__global__ __launch_bounds__(256) void k_hist_scan(uint32_t *__restrict__ hist,
                                                   uint32_t *__restrict__ off,
                                                   uint32_t *__restrict__ tile_ctr) {
    __shared__ uint32_t s[256];
    const int p = blockIdx.x, t = threadIdx.x;
    const uint32_t own = hist[256 * p + t];
    hist[256 * p + t] = 0u;
    s[t] = own;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t v = t >= o ? s[t - o] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    off[256 * p + t] = s[t] - own;
    if (t == 0) tile_ctr[p] = 0;
}

// ------------------------------------------------------------------ 3. one radix pass
// Status word per (tile, digit): epoch << 34 | flag << 32 | count,
// flag 1 = tile aggregate only, 2 = inclusive prefix through this tile.
__device__ __forceinline__ void st_status(unsigned long long *p, uint32_t epoch, uint32_t flag,
                                          uint32_t cnt) {
    unsigned long long v = ((unsigned long long)epoch << 34) |
                           ((unsigned long long)flag << 32) | cnt;
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kSortThreads) void k_sort_pass(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int n, int shift,
    const uint32_t *__restrict__ digit_off, unsigned long long *__restrict__ status,
    uint32_t *__restrict__ tile_ctr, uint32_t epoch) {
    __shared__ uint32_t hist[kSortThreads / 64][256];
    __shared__ uint32_t tstart[256];
    __shared__ int32_t gbase[256];
    __shared__ uint32_t wsum[kSortThreads / 64];
    __shared__ uint64_t sk[kSortTile];
    __shared__ uint32_t sv[kSortTile];
    __shared__ uint32_t tile_s;

    const int t = threadIdx.x;
    if (t == 0) tile_s = atomicAdd(tile_ctr, 1u);
    for (int i = t; i < (kSortThreads / 64) * 256; i += kSortThreads) (&hist[0][0])[i] = 0;
    __syncthreads();
    const int tile = (int)tile_s;
    const int wave = t / 64;
    const unsigned lane = lane_id();
    const int64_t base = (int64_t)tile * kSortTile + wave * kWaveTile;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rnk[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + k * 64 + lane;
        const bool valid = i < n;
        key[k] = valid ? kin[i] : 0ull;
        val[k] = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + k * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
        uint64_t m = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = ballot(valid && bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t r = rank_in(m);
        uint32_t c = 0;
        if (valid) c = hist[wave][d];
        rnk[k] = c + r;
        if (valid && r == 0) hist[wave][d] = c + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // digit phase: thread t < 256 (the first four waves) owns digit t
    const bool dig = t < 256;
    uint32_t tot = 0, incl = 0, excl = 0;
    if (dig) {
        // per digit: prefix over waves, tile total
        for (int w = 0; w < kSortThreads / 64; ++w) {
            const uint32_t c = hist[w][t];
            hist[w][t] = tot;
            tot += c;
        }
        // exclusive scan of tile totals over digits
        incl = tot;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o);
            if ((int)lane >= o) incl += v;
        }
        if (lane == 63) wsum[wave] = incl;
    }
    // look-back for digit t
    unsigned long long *my = status + (size_t)tile * 256 + (dig ? t : 0);
    if (dig) st_status(my, epoch, tile == 0 ? 2u : 1u, tot);
    if (dig && tile > 0) {
        int j = tile - 1;
        for (;;) {
            const unsigned long long v = __hip_atomic_load(status + (size_t)j * 256 + t,
                                                           __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ep = (uint32_t)(v >> 34), fl = (uint32_t)(v >> 32) & 3u;
            if (ep != epoch || fl == 0) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += (uint32_t)v;
            if (fl == 2) break;
            --j;
        }
        st_status(my, epoch, 2u, excl + tot);
    }
    __syncthreads();
    if (dig) {
        uint32_t wpre = 0;
        for (int w = 0; w < wave; ++w) wpre += wsum[w];
        const uint32_t ts = wpre + incl - tot;
        tstart[t] = ts;
        gbase[t] = (int32_t)(digit_off[t] + excl) - (int32_t)ts;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + k * 64 + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
            const uint32_t p = tstart[d] + hist[wave][d] + rnk[k];
            sk[p] = key[k];
            sv[p] = val[k];
        }
    }
    __syncthreads();
    const int64_t t0 = (int64_t)tile * kSortTile;
    const int tn = (int)(n - t0 < kSortTile ? n - t0 : kSortTile);
    for (int p = t; p < tn; p += kSortThreads) {
        const uint64_t kk = sk[p];
        const uint32_t d = (uint32_t)(kk >> shift) & 255u;
        const int o = gbase[d] + p;
        kout[o] = kk;
        vout[o] = sv[p];
    }
}

// ------------------------------------------------------------------ 3b. nearly sorted input
// A simulation rebuilds its tree from the bodies in the order of its previous
// build, and after a short step that order is still nearly sorted (Sec. 4.4
// makes the same observation and re-sorts by insertion).  Here a body whose
// new key keeps the key prefix of the leaf it sat in "stays": the leaves of
// the previous tree are disjoint key ranges in rank order, so staying bodies
// of different leaves are already in order; a leaf whose staying bodies are
// out of key order among themselves has all its bodies moved.  The movers
// (about 1 % of the bodies per step of the 2^22-body Plummer sphere) are
// radix-sorted, then merged with the stayers by rank.  Keys are compared
// with the input position as tie-break, so the result is exactly the stable
// sort of the new keys whatever the previous tree was (its leaves only
// decide how much moves).

// Per leaf of the previous tree (thread per node): each body's byte in
// mover[] is kNsMover for a mover, else kNsStay + (its rank among the leaf's
// stayers sorted by (key, position)) - (its rank among them in input
// order), the offset that puts the leaf's stayers in order.  A leaf whose
// stayers are out of order gets oflag 1 (k_ns_reorder then sets those
// offsets); one with more than 64 bodies moves whole instead.  Every node
// writes its oflag.
constexpr uint8_t kNsMover = 255, kNsStay = 64;
__global__ __launch_bounds__(kThreads) void k_ns_mark(int m_old, const int32_t *__restrict__ next,
                                                      const int32_t *__restrict__ level,
                                                      const int32_t *__restrict__ begin,
                                                      const int32_t *__restrict__ count,
                                                      const uint64_t *__restrict__ old_keys,
                                                      const uint64_t *__restrict__ new_keys,
                                                      int n, uint8_t *__restrict__ mover,
                                                      uint8_t *__restrict__ oflag) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m_old) return;
    oflag[c] = 0;
    if (next[c] != c + 1) return;
    const int b = begin[c];
    const int e = min(b + count[c], n);  // guard
    if (b < 0 || b >= e) return;
    const int sh = 3 * (kLevels - level[c]);  // 63 for a root leaf: every key stays
    const uint64_t pre = old_keys[b] >> sh;
    bool in_order = true, have = false;
    uint64_t prev = 0;
    for (int i = b; i < e; ++i) {
        const uint64_t k = new_keys[i];
        const bool stay = (k >> sh) == pre;
        mover[i] = stay ? kNsStay : kNsMover;
        if (stay) {
            if (have && k < prev) in_order = false;  // equal keys: input order is the tie-break
            prev = k;
            have = true;
        }
    }
    if (in_order) return;
    if (e - b > 64) {
        for (int i = b; i < e; ++i) mover[i] = kNsMover;
        return;
    }
    oflag[c] = 1;
}

// The flagged leaves: a wavefront takes 64 consecutive nodes and reorders
// its flagged leaves one after the other (lane j: body begin + j): a
// stayer's rank by (key, position) among the stayers against its rank by
// position.
__global__ __launch_bounds__(kThreads) void k_ns_reorder(int m_old,
                                                         const int32_t *__restrict__ begin,
                                                         const int32_t *__restrict__ count,
                                                         const uint64_t *__restrict__ new_keys,
                                                         int n, uint8_t *__restrict__ mover,
                                                         const uint8_t *__restrict__ oflag) {
    const int lane = (int)lane_id();
    const int c0 = (blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6)) * 64;
    if (c0 >= m_old) return;  // whole wavefront
    uint64_t fl = ballot(c0 + lane < m_old && oflag[c0 + lane]);
    while (fl) {
        const int c = c0 + __builtin_ctzll(fl);
        fl &= fl - 1;
        const int b = begin[c];
        const int cnt = min(count[c], n - b);  // at most 64 (k_ns_mark)
        const bool live = lane < cnt;
        const uint64_t k = live ? new_keys[b + lane] : 0ull;
        const bool stay = live && mover[b + lane] != kNsMover;
        const uint64_t smask = ballot(stay);
        int rs = 0;
        for (int t = 0; t < cnt; ++t) {
            const uint64_t kt = __shfl(k, t);
            if ((smask >> t) & 1ull) rs += kt < k || (kt == k && t < lane) ? 1 : 0;
        }
        const int rin = (int)rank_in(smask);
        if (stay) mover[b + lane] = (uint8_t)(kNsStay + rs - rin);
    }
}

// Movers per chunk of kThreads bodies, and the 8 digit histograms of the
// movers' keys (for their radix sort).  Few large blocks stride over the
// chunks, so that the histogram reaches global memory in few adds.
constexpr int kNsCountBlocks = 256;
__global__ __launch_bounds__(1024) void k_ns_count(int n, const uint8_t *__restrict__ mover,
                                                   const uint64_t *__restrict__ keys,
                                                   uint32_t *__restrict__ bcnt,
                                                   uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[8][256];
    __shared__ uint32_t ws[16];
    for (int j = threadIdx.x; j < 8 * 256; j += 1024) (&h[0][0])[j] = 0u;
    __syncthreads();
    const int nchunk = (n + kThreads - 1) / kThreads;
    // four chunks of kThreads bodies per iteration of the block
    for (int c0 = 4 * blockIdx.x; c0 < nchunk; c0 += 4 * gridDim.x) {
        const int i = c0 * kThreads + threadIdx.x;
        const bool mv = i < n && mover[i] == kNsMover;
        if (mv) {
            const uint64_t k = keys[i];
#pragma unroll
            for (int p = 0; p < 8; ++p) atomicAdd(&h[p][(uint32_t)(k >> (8 * p)) & 255u], 1u);
        }
        const uint64_t bal = ballot(mv);
        if (lane_id() == 0) ws[threadIdx.x / 64] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (threadIdx.x < 4 && c0 + (int)threadIdx.x < nchunk) {
            const int q = threadIdx.x;
            bcnt[c0 + q] = ws[4 * q] + ws[4 * q + 1] + ws[4 * q + 2] + ws[4 * q + 3];
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < 8 * 256; j += 1024) {
        const uint32_t v = (&h[0][0])[j];
        if (v) atomicAdd(&hist[j], v);
    }
}

// Stayers to (skeys, sidx) in input order, movers to (mkeys, midx) in input
// order; boff: the exclusive scan of the block counts.  Every kNsSample-th
// stayer is also copied to (tkeys, tidx), a sample small enough to stay in
// cache for the movers' searches.
constexpr int kNsSample = 64;
__global__ __launch_bounds__(kThreads) void k_ns_split(int n, const uint8_t *__restrict__ mover,
                                                       const uint64_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ boff,
                                                       uint64_t *__restrict__ skeys,
                                                       uint32_t *__restrict__ sidx,
                                                       uint64_t *__restrict__ mkeys,
                                                       uint32_t *__restrict__ midx,
                                                       uint64_t *__restrict__ tkeys,
                                                       uint32_t *__restrict__ tidx) {
    __shared__ uint32_t ws[kThreads / 64];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const uint8_t code = i < n ? mover[i] : kNsMover;
    const bool mv = i < n && code == kNsMover;
    const uint64_t bal = ballot(mv);
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) ws[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = boff[blockIdx.x] + rank_in(bal);
    for (int q = 0; q < w; ++q) before += ws[q];
    if (i < n) {
        const uint64_t k = keys[i];
        if (mv) {
            mkeys[before] = k;
            midx[before] = (uint32_t)i;
        } else {  // the stayer's place, reordered within its leaf
            const int si = i - (int)before + ((int)code - (int)kNsStay);
            skeys[si] = k;
            sidx[si] = (uint32_t)i;
            if (si % kNsSample == 0) {
                tkeys[si / kNsSample] = k;
                tidx[si / kNsSample] = (uint32_t)i;
            }
        }
    }
}

// (key, position) order: the stable order of keys
__device__ __forceinline__ bool ns_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}
// how many of the sorted pairs (k, v)[lo, hi) come before (key, id), plus lo
__device__ __forceinline__ int ns_rank_in(const uint64_t *__restrict__ k,
                                          const uint32_t *__restrict__ v, int lo, int hi,
                                          uint64_t key, uint32_t id) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ns_less(k[mid], v[mid], key, id)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge by rank: stayer j goes to j + (movers before it), mover q to q +
// (stayers before it).  A wavefront takes kNsPerLane * 64 consecutive
// stayers (sorted): one full search each for its first and last stayer
// bounds the movers' range that the others search (usually a few movers
// wide), so the chains of dependent loads are few.
// stayers per lane of k_ns_merge_stay: more for a large sort (fewer chains
// of dependent loads), fewer for a small one (more wavefronts to hide them)
constexpr int kNsPerLaneSmall = 4, kNsPerLaneLarge = 16, kNsLargeStayers = 1 << 24;
// the movers' rank of (key, id): first among every kNsSample-th mover
// (tkeys, tidx: cached), then within one block of kNsSample movers
__device__ __forceinline__ int ns_rank_sampled(const uint64_t *__restrict__ k,
                                               const uint32_t *__restrict__ v, int len,
                                               const uint64_t *__restrict__ tk,
                                               const uint32_t *__restrict__ tv, uint64_t key,
                                               uint32_t id) {
    const int c = ns_rank_in(tk, tv, 0, (len + kNsSample - 1) / kNsSample, key, id);
    const int lo = c > 0 ? kNsSample * (c - 1) + 1 : 0;
    return ns_rank_in(k, v, lo, min(kNsSample * c, len), key, id);
}

// every kNsSample-th mover (sorted), for ns_rank_sampled
__global__ __launch_bounds__(kThreads) void k_ns_sample(int nm, const uint64_t *__restrict__ mkeys,
                                                        const uint32_t *__restrict__ midx,
                                                        uint64_t *__restrict__ tkeys,
                                                        uint32_t *__restrict__ tidx) {
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q * kNsSample < nm) {
        tkeys[q] = mkeys[q * kNsSample];
        tidx[q] = midx[q * kNsSample];
    }
}

template <int kNsPerLane>
__global__ __launch_bounds__(kThreads) void k_ns_merge_stay(int ns, int nm,
                                                            const uint64_t *__restrict__ skeys,
                                                            const uint32_t *__restrict__ sidx,
                                                            const uint64_t *__restrict__ mkeys,
                                                            const uint32_t *__restrict__ midx,
                                                            const uint64_t *__restrict__ mtk,
                                                            const uint32_t *__restrict__ mti,
                                                            uint64_t *__restrict__ okeys,
                                                            uint32_t *__restrict__ oidx) {
    constexpr int kSpan = 64 * kNsPerLane;
    const int lane = (int)lane_id();
    const int w0 = (blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6)) * kSpan;
    if (w0 >= ns) return;  // whole wavefront
    const int last = min(w0 + kSpan - 1, ns - 1);
    int r = 0;
    if (lane == 0) r = ns_rank_sampled(mkeys, midx, nm, mtk, mti, skeys[w0], sidx[w0]);
    if (lane == 63) r = ns_rank_sampled(mkeys, midx, nm, mtk, mti, skeys[last], sidx[last]);
    const int lo = __builtin_amdgcn_readfirstlane(r);
    const int hi = __builtin_amdgcn_readlane(r, 63);
#pragma unroll
    for (int e = 0; e < kNsPerLane; ++e) {
        const int j = w0 + 64 * e + lane;
        if (j < ns) {
            const uint64_t k = skeys[j];
            const uint32_t v = sidx[j];
            const int o = j + ns_rank_in(mkeys, midx, lo, hi, k, v);
            okeys[o] = k;
            oidx[o] = v;
        }
    }
}

// The movers' side: c samples (every kNsSample-th stayer) come before the
// mover, so do the stayers up to kNsSample (c - 1), and none from
// kNsSample c on.
__global__ __launch_bounds__(kThreads) void k_ns_merge_move(int ns, int nm,
                                                            const uint64_t *__restrict__ skeys,
                                                            const uint32_t *__restrict__ sidx,
                                                            const uint64_t *__restrict__ mkeys,
                                                            const uint32_t *__restrict__ midx,
                                                            const uint64_t *__restrict__ tkeys,
                                                            const uint32_t *__restrict__ tidx,
                                                            uint64_t *__restrict__ okeys,
                                                            uint32_t *__restrict__ oidx) {
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= nm) return;
    const uint64_t k = mkeys[q];
    const uint32_t v = midx[q];
    const int c = ns_rank_in(tkeys, tidx, 0, (ns + kNsSample - 1) / kNsSample, k, v);
    const int lo = c > 0 ? kNsSample * (c - 1) + 1 : 0;
    const int hi = min(kNsSample * c, ns);
    const int o = q + ns_rank_in(skeys, sidx, lo, hi, k, v);
    okeys[o] = k;
    oidx[o] = v;
}

// ------------------------------------------------------------------ 4. gather
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(int n, uint32_t *__restrict__ flags,
                                                     const uint32_t *__restrict__ perm,
                                                     const T *__restrict__ pos,
                                                     const T *__restrict__ mass,
                                                     const T *__restrict__ vel,
                                                     const uint32_t *__restrict__ id,
                                                     T *__restrict__ spos, T *__restrict__ smass,
                                                     T *__restrict__ svel,
                                                     uint32_t *__restrict__ sid) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t j = perm[r];
    if (j >= n) {  // guard: a broken permutation is reported, not followed
        atomicOr(flags, 2u);
        j = 0;
    }
    spos[3 * (int64_t)r + 0] = pos[3 * j + 0];
    spos[3 * (int64_t)r + 1] = pos[3 * j + 1];
    spos[3 * (int64_t)r + 2] = pos[3 * j + 2];
    smass[r] = mass[j];
    if (svel) {
        svel[3 * (int64_t)r + 0] = vel[3 * j + 0];
        svel[3 * (int64_t)r + 1] = vel[3 * j + 1];
        svel[3 * (int64_t)r + 2] = vel[3 * j + 2];
    }
    if (sid) sid[r] = id ? id[j] : (uint32_t)j;
}

// ------------------------------------------------------------------ 5. topology
// Number of leading octal digits shared by the keys of ranks i-1 and i
// (21 when equal); -1 at i = 0 and i = n.
__device__ __forceinline__ int key_delta(const uint64_t *__restrict__ keys, int n, int i) {
    if (i <= 0 || i >= n) return -1;
    const uint64_t x = keys[i - 1] ^ keys[i];
    return x ? (__clzll(x) - 1) / 3 : kLevels;
}

// Chain length of every sorted rank s: the cells whose first body is s.
// They are the levels delta[s]+1 .. k_leaf(s), present only if the
// level-delta[s] cell around s holds more than B bodies (its parent is
// split); k_leaf is the first level at which the cell starting at s holds
// at most B bodies (or 21).  Also, per block, the sum of chain lengths and
// the number of cells at every level: bsum[b] and bsum[(1 + k) * nb + b].
// delta (n + 1 entries) is computed here from the sorted keys and stored
// for the later steps.
__global__ __launch_bounds__(kThreads) void k_chain(const uint64_t *__restrict__ keys, int n,
                                                    int B, int8_t *__restrict__ delta,
                                                    uint8_t *__restrict__ ns,
                                                    uint32_t *__restrict__ bsum) {
    constexpr int kSd = kThreads + 2 * (kMaxLeaf + 1) + 1;
    __shared__ int8_t sd[kSd], ta[kSd], tb[kSd];
    __shared__ uint32_t ws[kThreads / 64];
    __shared__ uint32_t lh[kLevels + 1];
    const int H = B + 1;
    const int NS = kThreads + 2 * H + 1;  // sd entries in use
    if (threadIdx.x <= kLevels) lh[threadIdx.x] = 0;
    const int b0 = blockIdx.x * kThreads;
    // sd[k] = delta[b0 - H + k] (-1 outside [1, n))
    for (int k = threadIdx.x; k < NS; k += kThreads)
        sd[k] = (int8_t)key_delta(keys, n, b0 - H + k);
    __syncthreads();
    // The level-ds cell around s (ds = delta[s]) holds more than B bodies iff
    // some B + 1 consecutive ranks around s all lie in it, i.e. iff the
    // largest over p in [s - B, s] of W(p) = min(delta[p+1 .. p+B]) is at
    // least ds; and the chain of s ends at level max(ds, W(s)) + 1.  Both
    // windows by doubling tables in LDS (ta, tb alternate; sd is kept).
    const int8_t *src = sd;
    int8_t *dst = ta;
    int w = 1;
    for (; 2 * w <= B; w *= 2) {  // src[i] = min(sd[i .. i + 2w - 1])
        for (int i = threadIdx.x; i + 2 * w <= NS; i += kThreads) {
            const int8_t x = src[i], y = src[i + w];
            dst[i] = x < y ? x : y;
        }
        __syncthreads();
        src = dst;
        dst = dst == ta ? tb : ta;
    }
    for (int q = threadIdx.x; q + B < NS; q += kThreads) {  // dst[q] = W at local q
        const int8_t x = src[q + 1], y = src[q + 1 + B - w];
        dst[q] = x < y ? x : y;
    }
    __syncthreads();
    const int s = b0 + threadIdx.x;
    const int L = threadIdx.x + H;  // local index of s
    const int ds = sd[L];
    const int mu = dst[L];  // min(delta[s+1 .. s+B]), -1 past the last rank
    src = dst;
    dst = dst == ta ? tb : ta;
    for (w = 1; 2 * w <= B + 1; w *= 2) {  // src[i] = max(W over [i, i + 2w - 1])
        for (int i = threadIdx.x; i + 2 * w <= NS; i += kThreads) {
            const int8_t x = src[i], y = src[i + w];
            dst[i] = x > y ? x : y;
        }
        __syncthreads();
        src = dst;
        dst = dst == ta ? tb : ta;
    }
    if (s < n) delta[s] = (int8_t)ds;
    if (s == n - 1) delta[n] = -1;
    uint32_t cnt_s = 0;
    if (s < n) {
        if (ds < kLevels) {
            const int e0 = src[L - B], e1 = src[L + 1 - w];
            const bool exists = s == 0 || (e0 > e1 ? e0 : e1) >= ds;
            if (exists) {
                int kl = ds + 1 > mu + 1 ? ds + 1 : mu + 1;
                kl = kl > kLevels ? kLevels : kl;
                cnt_s = (uint32_t)(kl - ds);
                for (int k = ds + 1; k <= kl; ++k) atomicAdd(&lh[k], 1u);
            }
        }
        ns[s] = (uint8_t)cnt_s;
    }
    uint32_t v = cnt_s;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) ws[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tsum = 0;
        for (int w = 0; w < kThreads / 64; ++w) tsum += ws[w];
        bsum[blockIdx.x] = tsum;
    }
    if (threadIdx.x <= kLevels) bsum[(size_t)(1 + threadIdx.x) * gridDim.x + blockIdx.x] = lh[threadIdx.x];
}

// Exclusive scan, in place, of each of gridDim.x segments of nb per-block
// sums (one block of 1024 threads per segment); the segment total goes to
// tot[segment].  Chunks of 8192 sums: loaded coalesced into LDS, eight
// consecutive sums scanned per thread, the thread totals across the block,
// then stored coalesced (one chunk covers 2^21 bodies' block sums, so the
// block's chain of dependent steps stays short).
constexpr int kScanPer = 8;
constexpr int kScanChunk = 1024 * kScanPer;
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *__restrict__ sums, int nb,
                                                    uint32_t *__restrict__ tot) {
    __shared__ uint32_t buf[kScanChunk];
    __shared__ uint32_t ws[16];
    uint32_t *s = sums + (size_t)blockIdx.x * nb;
    const int t = threadIdx.x;
    const unsigned lane = lane_id();
    const int w = t / 64;
    uint32_t carry = 0;  // the same in every thread: the previous chunks' total
    for (int c0 = 0; c0 < nb; c0 += kScanChunk) {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int i = c0 + k * 1024 + t;
            buf[k * 1024 + t] = i < nb ? s[i] : 0u;
        }
        __syncthreads();
        uint32_t v[kScanPer];
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = run;
            run += buf[t * kScanPer + k];
        }
        uint32_t incl = run;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t x = __shfl_up(incl, o);
            if ((int)lane >= o) incl += x;
        }
        if (lane == 63) ws[w] = incl;
        __syncthreads();
        uint32_t pre = carry + incl - run, ctot = 0;
        for (int k = 0; k < 16; ++k) {
            pre += k < w ? ws[k] : 0u;
            ctot += ws[k];
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) buf[t * kScanPer + k] = pre + v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int i = c0 + k * 1024 + t;
            if (i < nb) s[i] = buf[k * 1024 + t];
        }
        carry += ctot;
        __syncthreads();  // buf and ws are refilled by the next chunk
    }
    if (t == 0) tot[blockIdx.x] = carry;
}

// offs[s] = exclusive prefix of ns over ranks; offs[n] = node count.  Four
// ranks per thread (one 4-byte load, one 16-byte store), 1024 per block:
// the block's prefix is the scanned sum of its first 256-rank block of
// k_chain.
constexpr int kDownPer = 4;
constexpr int kDownRanks = kThreads * kDownPer;
__global__ __launch_bounds__(kThreads) void k_scan_down(const uint8_t *__restrict__ ns, int n,
                                                        const uint32_t *__restrict__ bpre,
                                                        int32_t *__restrict__ offs,
                                                        uint32_t *__restrict__ total) {
    static_assert(kDownRanks % kThreads == 0, "a block covers whole k_chain blocks");
    __shared__ uint32_t ws[kThreads / 64];
    const int s0 = (int)(blockIdx.x * kThreads + threadIdx.x) * kDownPer;
    uint32_t x[kDownPer];
    if (s0 + kDownPer <= n) {
        const uchar4 v = *(const uchar4 *)(ns + s0);
        x[0] = v.x, x[1] = v.y, x[2] = v.z, x[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < kDownPer; ++k) x[k] = s0 + k < n ? ns[s0 + k] : 0u;
    }
    const uint32_t run = x[0] + x[1] + x[2] + x[3];
    uint32_t incl = run;
    const unsigned lane = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if ((int)lane >= o) incl += v;
    }
    const int w = threadIdx.x / 64;
    if (lane == 63) ws[w] = incl;
    __syncthreads();
    uint32_t pre = bpre[blockIdx.x * (kDownRanks / kThreads)] + incl - run;
    for (int k = 0; k < w; ++k) pre += ws[k];
    const int4 o4 = make_int4((int)pre, (int)(pre + x[0]), (int)(pre + x[0] + x[1]),
                              (int)(pre + x[0] + x[1] + x[2]));
    if (s0 + kDownPer <= n) {
        *(int4 *)(offs + s0) = o4;
    } else if (s0 < n) {
        offs[s0] = o4.x;
        if (s0 + 1 < n) offs[s0 + 1] = o4.y;
        if (s0 + 2 < n) offs[s0 + 2] = o4.z;
    }
    if (s0 < n && n <= s0 + kDownPer) {  // the thread holding rank n - 1
        offs[n] = (int32_t)(pre + run);
        *total = pre + run;
    }
}

// First rank in (s, hi) whose key prefix (key >> shift) differs from pre;
// hi if none.  Galloping, then bisection.
__device__ int seg_end(const uint64_t *__restrict__ keys, int s, int hi, int shift, uint64_t pre) {
    int lo = s, step = 1, probe = s + 1;
    while (probe < hi && (keys[probe] >> shift) == pre) {
        lo = probe;
        step <<= 1;
        probe = s + step;
    }
    int r = probe < hi ? probe : hi;
    while (r - lo > 1) {
        const int mid = lo + ((r - lo) >> 1);
        if ((keys[mid] >> shift) == pre) lo = mid;
        else r = mid;
    }
    return r;
}
// First rank a <= s whose key prefix equals that of s.
__device__ int seg_begin(const uint64_t *__restrict__ keys, int s, int shift, uint64_t pre) {
    int hi = s, step = 1, probe = s - 1;
    while (probe >= 0 && (keys[probe] >> shift) == pre) {
        hi = probe;
        step <<= 1;
        probe = s - step;
    }
    int l = probe >= 0 ? probe : -1;  // keys[l] differs (or l = -1)
    while (hi - l > 1) {
        const int mid = l + ((hi - l) >> 1);
        if ((keys[mid] >> shift) == pre) hi = mid;
        else l = mid;
    }
    return hi;
}

// Per-level placement of the cells: base[k] is the first slot of level k in
// the level list (an exclusive scan of the level totals, host computed).
struct LevelBase {
    int32_t base[kLevels + 1];
};

// Writes every cell in pre-order: hashed key, level, body range, skip
// pointer, parent and integer centre, and lists it under its level.
// Block b covers ranks [256 b, 256 b + 256) and the cells of their chains,
// one thread per cell (a chain's cells are independent: each finds its own
// segment end), so a long chain of shallow cells is spread over threads.
// Block b places its level-k cells after those of blocks < b (scanned
// per-block level counts in lvl_pre[(1 + k) * nb + b]).  A block is one
// wavefront: 256 ranks hold about 60 cells (one per 4 to 5 bodies at
// leaf capacity 16), which then keep its lanes busy.  A cell's integer
// centre comes from the integer point of its first body: under the Morton
// curve the key's bits, under the Peano-Hilbert curve the body's sorted
// position quantised as its key was (the same bits as inverting the key,
// at a fraction of the cost).
constexpr int kEmitThreads = 64;
template <typename T>
__global__ __launch_bounds__(kEmitThreads) void k_emit(
    const uint64_t *__restrict__ keys, const T *__restrict__ spos,
    const Cube *__restrict__ cube, const int8_t *__restrict__ delta,
    const int32_t *__restrict__ offs, int n, int m,
    const uint32_t *__restrict__ lvl_pre, LevelBase lb, uint64_t *__restrict__ hkey,
    int32_t *__restrict__ level, int32_t *__restrict__ begin, int32_t *__restrict__ count,
    int32_t *__restrict__ next, int32_t *__restrict__ parent, int32_t *__restrict__ cx,
    int32_t *__restrict__ cy, int32_t *__restrict__ cz, int32_t *__restrict__ lvl_list,
    uint32_t *__restrict__ ucnt, int32_t *__restrict__ kids, int curve) {
    __shared__ uint32_t lcnt[kLevels + 1];
    // the upward pass's list counters start at zero
    if (blockIdx.x == 0 && threadIdx.x < 3) ucnt[threadIdx.x] = 0u;
    __shared__ int32_t lbase[kLevels + 1];
    __shared__ int32_t so[kThreads + 1];  // first cell of each rank's chain
    if (threadIdx.x <= kLevels) {
        lcnt[threadIdx.x] = 0;
        lbase[threadIdx.x] = lb.base[threadIdx.x] +
                             (int32_t)lvl_pre[(size_t)(1 + threadIdx.x) * gridDim.x + blockIdx.x];
    }
    const int b0 = blockIdx.x * kThreads;
    for (int j = threadIdx.x; j <= kThreads; j += kEmitThreads) {
        const int r = b0 + j;
        so[j] = offs[r < n ? r : n];
    }
    __syncthreads();
    const int c1 = so[kThreads] < m ? so[kThreads] : m;
    const double lx = cube->lo[0], ly = cube->lo[1], lz = cube->lo[2];
    const double scale = ldexp(1.0, kLevels) / cube->L;
    for (int node = so[0] + threadIdx.x; node < c1; node += kEmitThreads) {
        // the rank whose chain holds node: the last local r with so[r] <= node
        int lo = 0, hi = kThreads;  // so[lo] <= node < so[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (so[mid] <= node) lo = mid;
            else hi = mid;
        }
        const int s = b0 + lo;
        const int t = node - so[lo];
        const int ds = delta[s];
        const uint64_t key = keys[s];
        const int k = ds + 1 + t;
        const int sh = 3 * (kLevels - k);
        const uint64_t pre = k > 0 ? key >> sh : 0ull;
        const int e = k > 0 ? seg_end(keys, s, n, sh, pre) : n;
        int par = -1;
        if (t > 0) {
            par = node - 1;
        } else if (s > 0) {
            const int shp = 3 * (kLevels - ds);
            const uint64_t prep = ds > 0 ? key >> shp : 0ull;
            const int a = ds > 0 ? seg_begin(keys, s, shp, prep) : 0;
            par = offs[a] + (ds - (delta[a] + 1));
        }
        // the cell is named by its Morton hashed key whatever the curve the
        // bodies follow (a curve prefix and a Morton prefix of k digits name
        // the same cube); its centre from the integer point of body s
        uint32_t qx, qy, qz;
        if (curve == BH_CURVE_HILBERT) {
            const int64_t b = 3 * (int64_t)s;
            qx = quantise((double)spos[b + 0], lx, scale);
            qy = quantise((double)spos[b + 1], ly, scale);
            qz = quantise((double)spos[b + 2], lz, scale);
        } else {
            qx = compact3(key >> 2);
            qy = compact3(key >> 1);
            qz = compact3(key);
        }
        const uint64_t mkey =
            curve == BH_CURVE_HILBERT ? (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz) : key;
        hkey[node] = (1ull << (3 * k)) | (k > 0 ? mkey >> sh : 0ull);
        level[node] = k;
        begin[node] = s;
        count[node] = e - s;
        next[node] = offs[e];
        parent[node] = par < m ? par : -1;
        // the parent's child table, one slot per digit of the sort key (all
        // -1 before this launch): the slots follow the pre-order; the upward
        // pass compacts them
        if (par >= 0 && par < m) kids[8 * (int64_t)par + (int)(pre & 7u)] = node;
        const int cs = kLevels - k;
        cx[node] = (int32_t)(((qx >> cs) * 2u + 1u) << cs);
        cy[node] = (int32_t)(((qy >> cs) * 2u + 1u) << cs);
        cz[node] = (int32_t)(((qz >> cs) * 2u + 1u) << cs);
        const int slot = lbase[k] + (int)atomicAdd(&lcnt[k], 1u);
        if (slot < m) lvl_list[slot] = node;
    }
}

// ------------------------------------------------------------------ 6. upward pass
// The node arrays that the upward pass reads and writes.
struct UpArgs {
    int m;
    const int4 *kids;
    int32_t *kids_out;  // the same table, compacted by the upward pass
    const uint64_t *hkey;
    const int32_t *level, *begin, *count, *next, *parent, *cx, *cy, *cz;
    const Cube *cube;
    Moments *mom;
    uint32_t *cmask;
    void *recs;  // NodeRecT<R>::type[m]
    float *kc;   // M l^3 per node (the error budget's per-cell term)
};

__device__ __forceinline__ void set_level(NodeRec32 &, int) {}
__device__ __forceinline__ void set_level(NodeRec64 &r, int k) { r.level = k; }

// A node's own index data, loaded before its moments are combined (the
// stores of the moments would otherwise order these loads after them).
struct NodeGeo {
    int cx, cy, cz, begin, count, next, level;
};
__device__ __forceinline__ NodeGeo node_geo(const UpArgs &a, int i) {
    return NodeGeo{a.cx[i], a.cy[i], a.cz[i], a.begin[i], a.count[i], a.next[i], a.level[i]};
}

// Stores node i's final moments and its walk record (centre, COM offset,
// mass, traceless quadrupole 3T - tr(T) I, body range, skip pointer, side^2).
// h = L 2^-(kLevels+1): centres and sides are exact multiples of it.
template <typename R>
__device__ __forceinline__ void finish_node(const UpArgs &a, int i, const NodeGeo &gn,
                                            const Moments &q, uint32_t mask, double h) {
    a.mom[i] = q;
    a.cmask[i] = mask;
    {
        const double side = ldexp(h, kLevels + 1 - gn.level);
        a.kc[i] = (float)(q.m * side * side * side);
    }
    const double tr = q.t[0] + q.t[3] + q.t[5];
    typename NodeRecT<R>::type r{};
    r.cx = (R)(gn.cx * h);  // exact
    r.cy = (R)(gn.cy * h);
    r.cz = (R)(gn.cz * h);
    r.mx = (R)q.c[0];
    r.my = (R)q.c[1];
    r.mz = (R)q.c[2];
    r.m = (R)q.m;
    r.qxx = (R)(3.0 * q.t[0] - tr);
    r.qxy = (R)(3.0 * q.t[1]);
    r.qxz = (R)(3.0 * q.t[2]);
    r.qyy = (R)(3.0 * q.t[3] - tr);
    r.qyz = (R)(3.0 * q.t[4]);
    r.begin = gn.begin;
    r.count = gn.count;
    r.next = gn.next;
    const double side = ldexp(h, kLevels + 1 - gn.level);
    r.l2 = (R)(side * side);
    set_level(r, gn.level);
    ((typename NodeRecT<R>::type *)a.recs)[i] = r;
}

// One thread per node.  Leaves: FP64 moments straight from their bodies,
// about the leaf centre, the node record, and the walk's body records
// (offset from the leaf centre, computed in FP64, and mass) with the leaf
// centre as each body's anchor.  Internal cells are listed for the upward
// pass.  (The child table kids[8 c + q], the children in pre-order = key
// digit order for q < #children, then -1, which the upward pass and the
// group walk read in one load, is written by k_emit one slot per digit and
// compacted by the upward pass.)
// The internal cells are combined by the upward pass in two parts: the
// maximal subtrees of at most kSubNodes nodes (a subtree is the contiguous
// pre-order range [r, next[r])), one workgroup each, and the cells above
// them ("upper" cells, whose subtree is larger), in one workgroup.  k_leaves
// lists both: ulist[0 .. ucnt[0]) the subtree roots (internal cells of at
// most kSubNodes nodes whose parent's subtree is larger, or the root),
// ulist[m .. m + ucnt[1]) the upper cells (ucnt[2] is spare).
// One wavefront per subtree (a subtree has few cells per level), so that
// the ~N/1400 subtrees of a Plummer sphere are all resident at once.
constexpr int kSubThreads = 64;
constexpr int kSubSlots = 16;                         // nodes per thread
constexpr int kSubNodes = kSubThreads * kSubSlots;    // 1024

template <typename T, typename R>
__global__ __launch_bounds__(kThreads) void k_leaves(UpArgs ua, const T *__restrict__ spos,
                                                     const T *__restrict__ smass,
                                                     BodyRec<R> *__restrict__ bodies,
                                                     Anchor<R> *__restrict__ anchors,
                                                     int32_t *__restrict__ ulist,
                                                     uint32_t *__restrict__ ucnt) {
    // a wavefront's 64 consecutive nodes in pre-order own one contiguous
    // range of bodies: it is staged through LDS with coalesced loads (when it
    // fits), and each leaf's lane then reads its bodies from there
    constexpr int kStage = 2048 / (int)sizeof(T);  // bodies per wavefront
    __shared__ T stg[kThreads / 64][4][kStage];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = ua.m;
    const int32_t *__restrict__ next = ua.next;
    const Cube *__restrict__ cube = ua.cube;
    const bool valid = i < m;
    const int end = valid ? next[i] : 0;
    if (valid) {
        if (end != i + 1) {  // internal: a subtree root, an upper cell, or neither
            if (end - i > kSubNodes) {
                ulist[m + (int)atomicAdd(&ucnt[1], 1u)] = i;
            } else {
                const int p = ua.parent[i];
                if (p < 0 || ua.next[p] - p > kSubNodes) ulist[atomicAdd(&ucnt[0], 1u)] = i;
            }
        }
    }
    const bool leaf = valid && end == i + 1;
    NodeGeo gn{};
    if (leaf) gn = node_geo(ua, i);
    const int b = leaf ? gn.begin : 0, e = leaf ? gn.begin + gn.count : 0;
    // the wavefront's body range
    int lo = leaf ? b : INT_MAX, hi = leaf ? e : INT_MIN;
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    const int w = (int)threadIdx.x >> 6;
    const bool staged = hi > lo && hi - lo <= kStage;
    if (staged) {
        for (int j = lo + (int)lane_id(); j < hi; j += 64) {
            stg[w][0][j - lo] = spos[3 * (int64_t)j + 0];
            stg[w][1][j - lo] = spos[3 * (int64_t)j + 1];
            stg[w][2][j - lo] = spos[3 * (int64_t)j + 2];
            stg[w][3][j - lo] = smass[j];
        }
    }
    __syncthreads();
    const double h = ldexp(cube->L, -(kLevels + 1));
    if (leaf) {
        // body j's position component d and mass, from LDS or memory
        auto P = [&](int j, int d) -> double {
            return (double)(staged ? stg[w][d][j - lo] : spos[3 * (int64_t)j + d]);
        };
        auto Mj = [&](int j) -> T { return staged ? stg[w][3][j - lo] : smass[j]; };
        const double c0 = cube->lo[0] + gn.cx * h, c1 = cube->lo[1] + gn.cy * h,
                     c2 = cube->lo[2] + gn.cz * h;
        Anchor<R> an;
        an.x = (R)(gn.cx * h);  // exact
        an.y = (R)(gn.cy * h);
        an.z = (R)(gn.cz * h);
        an.leaf = i;
        double mt = 0, s0 = 0, s1 = 0, s2 = 0;
        for (int j = b; j < e; ++j) {
            const T mm = Mj(j);
            const double mj = (double)mm;
            const double y0 = P(j, 0) - c0;
            const double y1 = P(j, 1) - c1;
            const double y2 = P(j, 2) - c2;
            mt += mj;
            s0 += mj * y0;
            s1 += mj * y1;
            s2 += mj * y2;
            if (!staged) {  // (a staged wavefront writes its records below)
                BodyRec<R> br;
                br.x = (R)y0;
                br.y = (R)y1;
                br.z = (R)y2;
                br.m = (R)mm;
                bodies[j] = br;
                anchors[j] = an;
            }
        }
        Moments r;
        r.m = mt;
        r.c[0] = mt > 0 ? s0 / mt : 0.0;
        r.c[1] = mt > 0 ? s1 / mt : 0.0;
        r.c[2] = mt > 0 ? s2 / mt : 0.0;
        for (int a = 0; a < 6; ++a) r.t[a] = 0.0;
        for (int j = b; j < e; ++j) {
            const double mj = (double)Mj(j);
            const double y0 = P(j, 0) - c0 - r.c[0];
            const double y1 = P(j, 1) - c1 - r.c[1];
            const double y2 = P(j, 2) - c2 - r.c[2];
            r.t[0] += mj * y0 * y0;
            r.t[1] += mj * y0 * y1;
            r.t[2] += mj * y0 * y2;
            r.t[3] += mj * y1 * y1;
            r.t[4] += mj * y1 * y2;
            r.t[5] += mj * y2 * y2;
        }
        finish_node<R>(ua, i, gn, r, 0u, h);
    }
    // A staged wavefront writes the body and anchor records of its whole
    // body range with coalesced stores: its leaves, in body order (pre-order
    // leaves hold consecutive ranges), are listed in LDS, and each body finds
    // its leaf by a binary search of their first bodies.
    __shared__ int32_t lb[kThreads / 64][64], lnode[kThreads / 64][64];
    __shared__ int32_t lcx[kThreads / 64][64], lcy[kThreads / 64][64], lcz[kThreads / 64][64];
    const uint64_t lm = ballot(leaf);
    if (staged && leaf) {
        const int slot = (int)rank_in(lm);
        lb[w][slot] = b;
        lnode[w][slot] = i;
        lcx[w][slot] = gn.cx;
        lcy[w][slot] = gn.cy;
        lcz[w][slot] = gn.cz;
    }
    __syncthreads();
    if (staged) {
        const int nl = __popcll(lm);
        for (int j = lo + (int)lane_id(); j < hi; j += 64) {
            int s0 = 0, s1 = nl;  // lb[w][s0] <= j < lb[w][s1]
            while (s1 - s0 > 1) {
                const int mid = (s0 + s1) >> 1;
                if (lb[w][mid] <= j) s0 = mid;
                else s1 = mid;
            }
            const int cx = lcx[w][s0], cy = lcy[w][s0], cz = lcz[w][s0];
            const T mm = stg[w][3][j - lo];
            BodyRec<R> br;
            br.x = (R)((double)stg[w][0][j - lo] - (cube->lo[0] + cx * h));
            br.y = (R)((double)stg[w][1][j - lo] - (cube->lo[1] + cy * h));
            br.z = (R)((double)stg[w][2][j - lo] - (cube->lo[2] + cz * h));
            br.m = (R)mm;
            bodies[j] = br;
            Anchor<R> an;
            an.x = (R)(cx * h);  // exact
            an.y = (R)(cy * h);
            an.z = (R)(cz * h);
            an.leaf = lnode[w][s0];
            anchors[j] = an;
        }
    }
}

// One internal cell: combine its children (already done, one level deeper)
// in octant order, in one pass over them: mass, first and second moments
// about this cell's centre (the centre offsets are exact), then the shift
// to the COM, T = S2 - M com com^T.  Also the 8-bit child mask and the
// node record.
// The part that does not depend on the children's moments: node data and
// child table.
struct UpPre {
    int p;  // -1: nothing to combine (a leaf, or no node)
    NodeGeo gn;
    int4 k0, k1;
};
__device__ __forceinline__ UpPre up_pre(const UpArgs &a, int p) {
    UpPre u;
    u.p = -1;
    if (p < 0 || p >= a.m) return u;
    u.gn = node_geo(a, p);
    u.k0 = a.kids[2 * (int64_t)p];
    u.k1 = a.kids[2 * (int64_t)p + 1];
    if (u.gn.next != p + 1) u.p = p;  // leaves are done
    return u;
}

template <typename R>
__device__ __forceinline__ void up_combine(const UpArgs &a, const UpPre &u, double h) {
    const int p = u.p;
    if (p < 0) return;
    const NodeGeo &gn = u.gn;
    const int ch[8] = {u.k0.x, u.k0.y, u.k0.z, u.k0.w, u.k1.x, u.k1.y, u.k1.z, u.k1.w};
    const int pcx = gn.cx, pcy = gn.cy, pcz = gn.cz;
    double mt = 0, s0 = 0, s1 = 0, s2 = 0;
    double q[6] = {0, 0, 0, 0, 0, 0};
    uint32_t mask = 0;
    // the children in two batches of four, each batch's loads issued
    // together: an absent child loads the cell's own (unused) slot instead,
    // so no load waits behind a branch
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        Moments qm[4];
        int gx[4], gy[4], gz[4];
        uint32_t oct[4];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = ch[4 * half + j];
            ok[j] = c > p && c < a.m;
            const int cc = ok[j] ? c : p;
            qm[j] = a.mom[cc];
            gx[j] = a.cx[cc];
            gy[j] = a.cy[cc];
            gz[j] = a.cz[cc];
            oct[j] = (uint32_t)(a.hkey[cc] & 7u);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!ok[j]) continue;
            const double g0 = qm[j].c[0] + (double)(gx[j] - pcx) * h;
            const double g1 = qm[j].c[1] + (double)(gy[j] - pcy) * h;
            const double g2 = qm[j].c[2] + (double)(gz[j] - pcz) * h;
            const double w0 = qm[j].m * g0, w1 = qm[j].m * g1, w2 = qm[j].m * g2;
            mt += qm[j].m;
            s0 += w0;
            s1 += w1;
            s2 += w2;
            q[0] += qm[j].t[0] + w0 * g0;
            q[1] += qm[j].t[1] + w0 * g1;
            q[2] += qm[j].t[2] + w0 * g2;
            q[3] += qm[j].t[3] + w1 * g1;
            q[4] += qm[j].t[4] + w1 * g2;
            q[5] += qm[j].t[5] + w2 * g2;
            mask |= 1u << oct[j];
        }
    }
    // the child table compacted in place: children first, in digit order
    {
        // (selects only: no dynamically indexed register array)
        int kc[8], rank[8], nk = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            rank[j] = ch[j] > p && ch[j] < a.m ? nk : -1;
            nk += rank[j] >= 0 ? 1 : 0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            kc[q] = -1;
#pragma unroll
            for (int j = 0; j < 8; ++j) kc[q] = rank[j] == q ? ch[j] : kc[q];
        }
        int4 *o = (int4 *)a.kids_out + 2 * (int64_t)p;
        o[0] = make_int4(kc[0], kc[1], kc[2], kc[3]);
        o[1] = make_int4(kc[4], kc[5], kc[6], kc[7]);
    }
    Moments r;
    r.m = mt;
    r.c[0] = mt > 0 ? s0 / mt : 0.0;
    r.c[1] = mt > 0 ? s1 / mt : 0.0;
    r.c[2] = mt > 0 ? s2 / mt : 0.0;
    r.t[0] = q[0] - s0 * r.c[0];
    r.t[1] = q[1] - s0 * r.c[1];
    r.t[2] = q[2] - s0 * r.c[2];
    r.t[3] = q[3] - s1 * r.c[1];
    r.t[4] = q[4] - s1 * r.c[2];
    r.t[5] = q[5] - s2 * r.c[2];
    finish_node<R>(a, p, gn, r, mask, h);
}

template <typename R>
__device__ __forceinline__ void up_node(const UpArgs &a, int p, double h) {
    up_combine<R>(a, up_pre(a, p), h);
}

// Level buckets of a workgroup's cells in LDS: cells are placed by a
// counting sort over their levels (order within a level is free: the cells
// of one level are independent), so that each level is then one contiguous
// run that the workgroup's threads take in turn, from one call site.
struct LevelBuckets {
    int cnt[kLevels + 2];
    int off[kLevels + 2];
};
__device__ __forceinline__ void buckets_clear(LevelBuckets &b, int t) {
    if (t <= kLevels + 1) b.cnt[t] = 0;
}
__device__ __forceinline__ void buckets_scan(LevelBuckets &b, int t) {
    if (t == 0) {
        int acc = 0;
        for (int k = 0; k <= kLevels + 1; ++k) {
            b.off[k] = acc;
            acc += b.cnt[k];
            b.cnt[k] = b.off[k];  // becomes the placement cursor
        }
    }
}

// The subtrees: workgroup b takes roots b, b + gridDim.x, ... of the list,
// buckets each subtree's internal cells by level, and combines them level
// by level, deepest first, with a workgroup barrier between levels (all
// waves share one CU, so the barrier's fence makes a level's moments visible
// to the next).  The leaves were done by k_leaves, the launch before.  Any
// grid size is correct.  (A shared atomic hand-out counter cost more than
// the uneven sizes of the subtrees: 166 against 88 us at 2^22 bodies.)
template <typename R>
__global__ __launch_bounds__(kSubThreads) void k_up_sub(UpArgs a,
                                                        const int32_t *__restrict__ roots,
                                                        const uint32_t *__restrict__ ucnt) {
    __shared__ LevelBuckets bk;
    __shared__ int32_t cell[kSubNodes];
    const double h = ldexp(a.cube->L, -(kLevels + 1));
    const int t = (int)threadIdx.x;
    const int total = (int)ucnt[0];
    for (int w = (int)blockIdx.x; w < total; w += (int)gridDim.x) {
        buckets_clear(bk, t);
        __syncthreads();
        const int r = roots[w];
        const int e = a.next[r];
        // every slot's loads at once (indices clamped into the subtree)
        int nx[kSubSlots], lv[kSubSlots];
#pragma unroll
        for (int q = 0; q < kSubSlots; ++q) {
            const int i = min(r + t + q * kSubThreads, e - 1);
            nx[q] = a.next[i];
            lv[q] = a.level[i];
        }
#pragma unroll
        for (int q = 0; q < kSubSlots; ++q) {
            const int i = r + t + q * kSubThreads;
            if (i >= e || nx[q] == i + 1) lv[q] = -1;  // outside, or a leaf
            if (lv[q] >= 0) atomicAdd(&bk.cnt[lv[q]], 1);
        }
        __syncthreads();
        buckets_scan(bk, t);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSubSlots; ++q)
            if (lv[q] >= 0) cell[atomicAdd(&bk.cnt[lv[q]], 1)] = r + t + q * kSubThreads;
        __syncthreads();
        const int kr = a.level[r];
        for (int k = kLevels; k >= kr; --k) {
            const int b0 = bk.off[k], b1 = bk.off[k + 1];
            if (b0 == b1) continue;  // uniform
            for (int j = b0 + t; j < b1; j += kSubThreads) up_node<R>(a, cell[j], h);
            __syncthreads();
        }
        __syncthreads();
    }
}

// The upper cells, in one workgroup, level by level, deepest first: their
// children are upper cells (done at a deeper level by this workgroup) or
// subtree roots and leaves (done by the launches before).  Up to kUpLds of
// them are bucketed by level in LDS; a longer list (only for trees far from
// balanced) is scanned again at every level.
constexpr int kUpThreads = 512;
constexpr int kUpLds = 8192;
template <typename R>
__global__ __launch_bounds__(kUpThreads) void k_up_upper(UpArgs a,
                                                         const int32_t *__restrict__ list,
                                                         const uint32_t *__restrict__ ucnt) {
    __shared__ LevelBuckets bk;
    __shared__ int32_t cell[kUpLds];
    const double h = ldexp(a.cube->L, -(kLevels + 1));
    const int t = (int)threadIdx.x;
    const int u = (int)ucnt[1];
    if (u == 0) return;
    if (u <= kUpLds) {
        buckets_clear(bk, t);
        __syncthreads();
        for (int j = t; j < u; j += kUpThreads) atomicAdd(&bk.cnt[a.level[list[j]]], 1);
        __syncthreads();
        buckets_scan(bk, t);
        __syncthreads();
        for (int j = t; j < u; j += kUpThreads) {
            const int p = list[j];
            cell[atomicAdd(&bk.cnt[a.level[p]], 1)] = p;
        }
        __syncthreads();
        for (int k = kLevels; k >= 0; --k) {
            const int b0 = bk.off[k], b1 = bk.off[k + 1];
            if (b0 == b1) continue;  // uniform
            for (int j = b0 + t; j < b1; j += kUpThreads) up_node<R>(a, cell[j], h);
            __syncthreads();
        }
    } else {
        for (int k = kLevels; k >= 0; --k) {
            for (int j = t; j < u; j += kUpThreads) {
                const int p = list[j];
                if (a.level[p] == k) up_node<R>(a, p, h);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- octopole
// Third moments for the order-3 walk (Sec. 2.2, the l = 3 term): raw
// S3_abc = sum m y_a y_b y_c about each cell's COM, FP64, components xxx
// xxy xxz xyy xyz xzz yyy yyz yzz zzz.  Leaves from their bodies; internal
// cells level by level, deepest first, from their children by the shift of
// origin (the first moment about a child's COM vanishes):
//   S3_P = sum_k S3_k + (S2_k,ab d_c + S2_k,ac d_b + S2_k,bc d_a) + M_k d_a d_b d_c,
// d = COM_k - COM_P, S2 the raw second moment about the child's COM.  Then
// the traceless octopole O_abc = 15 S3_abc - 3 (T_a d_bc + T_b d_ac +
// T_c d_ab), T_a = S3_axx + S3_ayy + S3_azz, is packed as its seven
// independent components xxx xxy xxz xyy xyz yyy yyz (the others follow
// from the zero traces) and a pad.
__device__ __forceinline__ void com_abs(const Moments &q, int cx, int cy, int cz,
                                        const Cube *cube, double h, double c[3]) {
    c[0] = cube->lo[0] + cx * h + q.c[0];
    c[1] = cube->lo[1] + cy * h + q.c[1];
    c[2] = cube->lo[2] + cz * h + q.c[2];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_oct_leaves(int m, const int32_t *__restrict__ begin,
                                                         const int32_t *__restrict__ count,
                                                         const int32_t *__restrict__ next,
                                                         const int32_t *__restrict__ cx,
                                                         const int32_t *__restrict__ cy,
                                                         const int32_t *__restrict__ cz,
                                                         const Moments *__restrict__ mom,
                                                         const Cube *__restrict__ cube,
                                                         const T *__restrict__ spos,
                                                         const T *__restrict__ smass,
                                                         double *__restrict__ s3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || next[i] != i + 1) return;
    const double h = ldexp(cube->L, -(kLevels + 1));
    double c[3];
    com_abs(mom[i], cx[i], cy[i], cz[i], cube, h, c);
    double o[10] = {};
    for (int j = begin[i]; j < begin[i] + count[i]; ++j) {
        const double y0 = (double)spos[3 * (int64_t)j] - c[0];
        const double y1 = (double)spos[3 * (int64_t)j + 1] - c[1];
        const double y2 = (double)spos[3 * (int64_t)j + 2] - c[2];
        const double mj = (double)smass[j];
        o[0] += mj * y0 * y0 * y0;
        o[1] += mj * y0 * y0 * y1;
        o[2] += mj * y0 * y0 * y2;
        o[3] += mj * y0 * y1 * y1;
        o[4] += mj * y0 * y1 * y2;
        o[5] += mj * y0 * y2 * y2;
        o[6] += mj * y1 * y1 * y1;
        o[7] += mj * y1 * y1 * y2;
        o[8] += mj * y1 * y2 * y2;
        o[9] += mj * y2 * y2 * y2;
    }
    for (int k = 0; k < 10; ++k) s3[10 * (int64_t)i + k] = o[k];
}

__global__ __launch_bounds__(kThreads) void k_oct_level(const int32_t *__restrict__ list, int cnt,
                                                        const int32_t *__restrict__ kids,
                                                        const int32_t *__restrict__ cx,
                                                        const int32_t *__restrict__ cy,
                                                        const int32_t *__restrict__ cz,
                                                        const Moments *__restrict__ mom,
                                                        const Cube *__restrict__ cube,
                                                        double *__restrict__ s3) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const int p = list[t];
    const int32_t *kp = kids + 8 * (int64_t)p;
    if (kp[0] < 0) return;  // a leaf (computed from its bodies)
    const double h = ldexp(cube->L, -(kLevels + 1));
    double cp[3];
    com_abs(mom[p], cx[p], cy[p], cz[p], cube, h, cp);
    double o[10] = {};
    for (int q = 0; q < 8 && kp[q] >= 0; ++q) {
        const int k = kp[q];
        const Moments mk = mom[k];
        double ck[3];
        com_abs(mk, cx[k], cy[k], cz[k], cube, h, ck);
        const double d0 = ck[0] - cp[0], d1 = ck[1] - cp[1], d2 = ck[2] - cp[2];
        const double *t2 = mk.t;  // xx xy xz yy yz zz about the child's COM
        const double *sk = s3 + 10 * (int64_t)k;
        const double M = mk.m;
        o[0] += sk[0] + 3 * t2[0] * d0 + M * d0 * d0 * d0;
        o[1] += sk[1] + 2 * t2[1] * d0 + t2[0] * d1 + M * d0 * d0 * d1;
        o[2] += sk[2] + 2 * t2[2] * d0 + t2[0] * d2 + M * d0 * d0 * d2;
        o[3] += sk[3] + t2[3] * d0 + 2 * t2[1] * d1 + M * d0 * d1 * d1;
        o[4] += sk[4] + t2[4] * d0 + t2[2] * d1 + t2[1] * d2 + M * d0 * d1 * d2;
        o[5] += sk[5] + t2[5] * d0 + 2 * t2[2] * d2 + M * d0 * d2 * d2;
        o[6] += sk[6] + 3 * t2[3] * d1 + M * d1 * d1 * d1;
        o[7] += sk[7] + 2 * t2[4] * d1 + t2[3] * d2 + M * d1 * d1 * d2;
        o[8] += sk[8] + t2[5] * d1 + 2 * t2[4] * d2 + M * d1 * d2 * d2;
        o[9] += sk[9] + 3 * t2[5] * d2 + M * d2 * d2 * d2;
    }
    for (int k = 0; k < 10; ++k) s3[10 * (int64_t)p + k] = o[k];
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_oct_pack(int m, const double *__restrict__ s3,
                                                       R *__restrict__ oct) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double *s = s3 + 10 * (int64_t)i;
    const double tx = s[0] + s[3] + s[5], ty = s[1] + s[6] + s[8], tz = s[2] + s[7] + s[9];
    R *o = oct + 8 * (int64_t)i;
    o[0] = (R)(15 * s[0] - 9 * tx);  // xxx
    o[1] = (R)(15 * s[1] - 3 * ty);  // xxy
    o[2] = (R)(15 * s[2] - 3 * tz);  // xxz
    o[3] = (R)(15 * s[3] - 3 * tx);  // xyy
    o[4] = (R)(15 * s[4]);           // xyz
    o[5] = (R)(15 * s[6] - 9 * ty);  // yyy
    o[6] = (R)(15 * s[7] - 3 * tz);  // yyz
    o[7] = (R)0;
}

template <typename T>
int build_typed(bh_ctx *ctx, bh_tree *t, const T *pos, const T *mass, int n, int B,
                const T *vel, const uint32_t *id, T *pos_out, T *vel_out, T *mass_out,
                uint32_t *id_out, bool resort) {
    hipStream_t st = ctx->stream;
    const int ntiles = div_up(n, kSortTile);
    const int nb = div_up(n, kThreads);
    const int nbbox = nb < 1024 ? nb : 1024;
    const int nkeys = div_up(n, kKeyThreads) < kKeyBlocks ? div_up(n, kKeyThreads) : kKeyBlocks;
    int rc;
    const size_t status_cap0 = t->status.cap, hist_cap0 = t->hist.cap;
    // ---- allocations sized by n
    if ((rc = grow(t->keys_a, 8ull * n)) || (rc = grow(t->keys_b, 8ull * n)) ||
        (rc = grow(t->idx_a, 4ull * n)) || (rc = grow(t->idx_b, 4ull * n)) ||
        (rc = grow(t->delta, (size_t)n + 1)) || (rc = grow(t->nstart, (size_t)n)) ||
        (rc = grow(t->offs, 4ull * (n + 1))) || (rc = grow(t->cube, sizeof(Cube))) ||
        (rc = grow(t->part, 7ull * 8 * nbbox)) || (rc = grow(t->hist, 4ull * 256 * 8 * 4)) ||
        (rc = grow(t->misc, 256 + 4ull * (kLevels + 2) * (nb + 1))) ||
        (rc = grow(t->status, 8ull * 256 * ntiles)) ||
        (rc = grow(t->bodies, sizeof(BodyRec<T>) * (size_t)n)) ||
        (rc = grow(t->anchors, sizeof(Anchor<T>) * (size_t)n)))
        return rc;
    if (!pos_out) {
        if ((rc = grow(t->spos, 3 * sizeof(T) * (size_t)n)) ||
            (rc = grow(t->smass, sizeof(T) * (size_t)n)))
            return rc;
        pos_out = (T *)t->spos.p;
        mass_out = (T *)t->smass.p;
    }
    Cube *cube = (Cube *)t->cube.p;
    // misc: [0] flags, [1] node count, [8..15] sort tile counters, [16..38]
    // segment totals (chain-length sum, then cells per level), [40..47] a
    // copy of the root cube, [64..] per-block sums; [0..48) goes to the host
    // in one copy
    uint32_t *misc = (uint32_t *)t->misc.p;
    uint32_t *flags = misc, *tile_ctr = misc + 8, *seg_tot = misc + 16;
    uint32_t *bsum = misc + 64;
    uint32_t *ucnt = misc + 48;  // upward pass: roots, upper cells, hand-out
    // digit histograms and their scans: all keys, then the movers of a
    // nearly sorted input
    uint32_t *hist = (uint32_t *)t->hist.p, *doff = hist + 2048;
    uint32_t *mhist = hist + 4096, *mdoff = hist + 6144;

    // the digit histograms are left zeroed by the previous build's scans;
    // only fresh memory needs clearing
    if (t->hist.cap != hist_cap0) {
        k_fill_u32<<<8, 256, 0, st>>>(hist, 2048, 0u);
        k_fill_u32<<<8, 256, 0, st>>>(mhist, 2048, 0u);
    }
    if (t->status.cap != status_cap0) {
        // fresh look-back status memory: clear it, or leftover words of
        // whatever used the memory before could carry the current epoch
        const int64_t words = (int64_t)(t->status.cap / 4);
        k_fill_u32<<<(int)((words + 255) / 256), 256, 0, st>>>((uint32_t *)t->status.p, words, 0u);
    }
    k_bbox<T><<<nbbox, kThreads, 0, st>>>(pos, n, (double *)t->part.p);
    k_cube<<<1, kThreads, 0, st>>>((const double *)t->part.p, nbbox, cube, (Cube *)(misc + 40),
                                   flags);
    // the new keys go to the buffer that does not hold the previous build's
    // sorted keys (a nearly sorted rebuild reads those)
    uint64_t *kold = t->sorted_keys;
    uint64_t *knew = kold == (uint64_t *)t->keys_a.p ? (uint64_t *)t->keys_b.p
                                                     : (uint64_t *)t->keys_a.p;
    uint64_t *kother = knew == (uint64_t *)t->keys_a.p ? (uint64_t *)t->keys_b.p
                                                       : (uint64_t *)t->keys_a.p;
    // the all-key digit counts only for the full sort: a rebuild that tries
    // the nearly sorted re-sort counts them only if it falls back
    k_keys<T><<<nkeys, kKeyThreads, 0, st>>>(pos, n, cube, knew, resort ? nullptr : hist,
                                             t->curve);
    if (!resort) k_hist_scan<<<8, 256, 0, st>>>(hist, doff, tile_ctr);
    // one radix sort of n (key, index) pairs, 8 passes of 8 bits: from (ka,
    // va) (va NULL: the input positions), through (kb, vb), ending in (ka,
    // va) again (an even number of passes)
    auto radix = [&](uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb, uint32_t *vspare,
                     int cnt, const uint32_t *offs8) -> uint32_t * {
        const int tiles = div_up(cnt, kSortTile);
        for (int p = 0; p < 8; ++p) {
            const uint32_t ep = ++ctx->epoch;
            k_sort_pass<<<tiles, kSortThreads, 0, st>>>(ka, va, kb, vb, cnt, 8 * p,
                                                        offs8 + 256 * p,
                                                        (unsigned long long *)t->status.p,
                                                        tile_ctr + p, ep & 0x3fffffffu);
            uint64_t *tk = ka;
            ka = kb;
            kb = tk;
            uint32_t *tv = va ? va : vspare;
            va = vb;
            vb = tv;
        }
        return va;
    };
    bool sorted = false;
    t->movers = -1;
    if (resort && kold) {
        // nearly sorted input: stayers, movers, merge (see k_ns_mark)
        const int64_t cap = n / 4 + 1, tcap = n / kNsSample + 1;
        if ((rc = grow(t->mv, 24ull * cap + 24ull * tcap))) return rc;
        uint64_t *mk0 = (uint64_t *)t->mv.p, *mk1 = mk0 + cap, *tk = mk1 + cap, *mtk = tk + tcap;
        uint32_t *mi0 = (uint32_t *)(mtk + tcap), *mi1 = mi0 + cap, *ti = mi1 + cap,
                 *mti = ti + tcap;
        uint8_t *mover = (uint8_t *)t->nstart.p;  // free until the topology
        const int m_old = (int)t->m;
        // the previous build's upward-pass lists (8 m_old bytes) are free
        // until this build's k_leaves: the leaves' out-of-order flags go there
        uint8_t *oflag = (uint8_t *)t->ulist.p;
        k_ns_mark<<<div_up(m_old, kThreads), kThreads, 0, st>>>(
            m_old, (const int32_t *)t->next.p, (const int32_t *)t->level.p,
            (const int32_t *)t->begin.p, (const int32_t *)t->count.p, kold, knew, n, mover, oflag);
        k_ns_reorder<<<div_up(m_old, kThreads), kThreads, 0, st>>>(
            m_old, (const int32_t *)t->begin.p, (const int32_t *)t->count.p, knew, n, mover,
            oflag);
        k_ns_count<<<std::min(kNsCountBlocks, div_up(nb, 4)), 1024, 0, st>>>(n, mover, knew,
                                                                             bsum, mhist);
        k_scan_sums<<<1, 1024, 0, st>>>(bsum, nb, misc + 51);
        // the mover histograms are scanned (and so cleared) on every path
        k_hist_scan<<<8, 256, 0, st>>>(mhist, mdoff, tile_ctr);
        uint32_t *hp = (uint32_t *)ctx->pinned + 56;
        if ((rc = check_launch("resort")) ||
            hipMemcpyAsync(hp, misc + 51, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return rc ? rc : set_error(BH_E_DEVICE, "build: device failure while re-sorting");
        const int nm = (int)hp[0];
        if (nm >= 0 && nm < cap) {
            k_ns_split<<<nb, kThreads, 0, st>>>(n, mover, knew, bsum, kother,
                                                (uint32_t *)t->idx_a.p, mk0, mi0, tk, ti);
            if (nm > 1) radix(mk0, mi0, mk1, mi1, nullptr, nm, mdoff);
            const int ns = n - nm;
            const uint32_t *si = (const uint32_t *)t->idx_a.p;
            uint32_t *oi = (uint32_t *)t->idx_b.p;
            if (nm > 0)
                k_ns_sample<<<div_up(div_up(nm, kNsSample), kThreads), kThreads, 0, st>>>(
                    nm, mk0, mi0, mtk, mti);
            if (ns >= kNsLargeStayers)
                k_ns_merge_stay<kNsPerLaneLarge>
                    <<<div_up(ns, kThreads * kNsPerLaneLarge), kThreads, 0, st>>>(
                        ns, nm, kother, si, mk0, mi0, mtk, mti, knew, oi);
            else if (ns > 0)
                k_ns_merge_stay<kNsPerLaneSmall>
                    <<<div_up(ns, kThreads * kNsPerLaneSmall), kThreads, 0, st>>>(
                        ns, nm, kother, si, mk0, mi0, mtk, mti, knew, oi);
            if (nm > 0)
                k_ns_merge_move<<<div_up(nm, kThreads), kThreads, 0, st>>>(ns, nm, kother, si,
                                                                           mk0, mi0, tk, ti,
                                                                           knew, oi);
            t->sorted_keys = knew;
            t->perm = (uint32_t *)t->idx_b.p;
            t->movers = nm;
            sorted = true;
        }
        // else: too many movers for the merge to pay; the full sort below
        // counts the all-key digit histograms first
    }
    if (!sorted) {
        if (resort) {
            k_keys<T><<<nkeys, kKeyThreads, 0, st>>>(nullptr, n, cube, knew, hist, t->curve);
            k_hist_scan<<<8, 256, 0, st>>>(hist, doff, tile_ctr);
        }
        t->perm = radix(knew, nullptr, kother, (uint32_t *)t->idx_b.p, (uint32_t *)t->idx_a.p, n,
                        doff);
        t->sorted_keys = knew;
    }
    uint64_t *ka = t->sorted_keys;
    uint32_t *va = t->perm;
    if ((rc = check_launch("sort"))) return rc;
    k_gather<T><<<nb, kThreads, 0, st>>>(n, flags, va, pos, mass, vel, id, pos_out, mass_out, vel_out,
                                         id_out);
    // ---- topology
    int8_t *delta = (int8_t *)t->delta.p;
    uint8_t *ns = (uint8_t *)t->nstart.p;
    int32_t *offs = (int32_t *)t->offs.p;
    k_chain<<<nb, kThreads, 0, st>>>(ka, n, B, delta, ns, bsum);
    k_scan_sums<<<kLevels + 2, 1024, 0, st>>>(bsum, nb, seg_tot);
    k_scan_down<<<div_up(n, kDownRanks), kThreads, 0, st>>>(ns, n, bsum, offs, misc + 1);
    if ((rc = check_launch("topology"))) return rc;
    uint32_t *hp = (uint32_t *)ctx->pinned;
    if (hipMemcpyAsync(hp, misc, 4 * 48, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_error(BH_E_DEVICE, "build: device failure while sizing the tree");
    if (hp[0] & 1u) return set_error(BH_E_NONFINITE, "bh_build: non-finite position");
    if (hp[0] & 2u) return set_error(BH_E_DEVICE, "bh_build: internal error (sort permutation)");
    Cube hc;
    memcpy(&hc, hp + 40, sizeof(Cube));
    for (int d = 0; d < 3; ++d) t->lo[d] = hc.lo[d];
    t->L = hc.L;
    if (hp[1] > 0x7fffffffu)  // cannot happen within the host's bound on n
        return set_error(BH_E_DEVICE, "bh_build: internal error (node count above 2^31 - 1)");
    const int m = (int)hp[1];
    t->m = m;
    // cells per level -> level-list bases, depth
    LevelBase lb;
    int lcount[kLevels + 1];
    int acc = 0;
    t->depth = 0;
    for (int k = 0; k <= kLevels; ++k) {
        lcount[k] = (int)hp[16 + 1 + k];
        lb.base[k] = acc;
        t->lvl_cnt[k] = lcount[k];
        t->lvl_base[k] = acc;
        acc += lcount[k];
        if (lcount[k] > 0) t->depth = k;
    }
    if (acc != m || hp[16] != (uint32_t)m)
        return set_error(BH_E_DEVICE, "bh_build: internal error (level counts)");
    // ---- node allocations
    if ((rc = grow(t->hkey, 8ull * m)) || (rc = grow(t->level, 4ull * m)) ||
        (rc = grow(t->begin, 4ull * m)) || (rc = grow(t->count, 4ull * m)) ||
        (rc = grow(t->next, 4ull * m)) || (rc = grow(t->parent, 4ull * m)) ||
        (rc = grow(t->cmask, 4ull * m)) || (rc = grow(t->lvl_list, 4ull * m)) ||
        (rc = grow(t->cx, 4ull * m)) ||
        (rc = grow(t->cy, 4ull * m)) || (rc = grow(t->cz, 4ull * m)) ||
        (rc = grow(t->mom, sizeof(Moments) * (size_t)m)) ||
        (rc = grow(t->kids, 32ull * m)) || (rc = grow(t->ulist, 8ull * m)) ||
        (rc = grow(t->recs, sizeof(typename NodeRecT<T>::type) * (size_t)m)) ||
        (rc = grow(t->kc, 4ull * m)))
        return rc;
    const int nbm = div_up(m, kThreads);
    int32_t *lvl_list = (int32_t *)t->lvl_list.p;
    k_fill_u32<<<div_up(8 * (int64_t)m, kThreads), kThreads, 0, st>>>((uint32_t *)t->kids.p,
                                                                      8 * (int64_t)m, ~0u);
    k_emit<T><<<nb, kEmitThreads, 0, st>>>(ka, pos_out, cube, delta, offs, n, m, bsum, lb,
                                           (uint64_t *)t->hkey.p,
                                    (int32_t *)t->level.p, (int32_t *)t->begin.p,
                                    (int32_t *)t->count.p, (int32_t *)t->next.p,
                                    (int32_t *)t->parent.p, (int32_t *)t->cx.p,
                                    (int32_t *)t->cy.p, (int32_t *)t->cz.p, lvl_list, ucnt,
                                    (int32_t *)t->kids.p, t->curve);
    UpArgs ua;
    ua.m = m;
    ua.kids = (const int4 *)t->kids.p;
    ua.kids_out = (int32_t *)t->kids.p;
    ua.hkey = (const uint64_t *)t->hkey.p;
    ua.level = (const int32_t *)t->level.p;
    ua.begin = (const int32_t *)t->begin.p;
    ua.count = (const int32_t *)t->count.p;
    ua.next = (const int32_t *)t->next.p;
    ua.parent = (const int32_t *)t->parent.p;
    ua.cx = (const int32_t *)t->cx.p;
    ua.cy = (const int32_t *)t->cy.p;
    ua.cz = (const int32_t *)t->cz.p;
    ua.cube = cube;
    ua.mom = (Moments *)t->mom.p;
    ua.cmask = (uint32_t *)t->cmask.p;
    ua.recs = t->recs.p;
    ua.kc = (float *)t->kc.p;
    int32_t *ulist = (int32_t *)t->ulist.p;
    k_leaves<T, T><<<nbm, kThreads, 0, st>>>(ua, pos_out, mass_out,
                                             (BodyRec<T> *)t->bodies.p,
                                             (Anchor<T> *)t->anchors.p, ulist, ucnt);
    // subtrees: about one root per 330 nodes in a Plummer sphere, so about
    // one workgroup each up to 2^22 bodies (a wavefront each: all resident)
    const int nsub = m / 256 < 1 ? 1 : (m / 256 > 8192 ? 8192 : m / 256);
    k_up_sub<T><<<nsub, kSubThreads, 0, st>>>(ua, ulist, ucnt);
    k_up_upper<T><<<1, kUpThreads, 0, st>>>(ua, ulist + m, ucnt);
    t->kids_tree_id = t->build_id;
    t->kc_tree_id = t->build_id;
    return check_launch("tree");
}

}  // namespace

int ensure_octopole(bh_tree *t) {
    if (t->oct_tree_id == t->build_id) return BH_OK;
    const int m = (int)t->m;
    const size_t rs = t->dtype == BH_F32 ? 4 : 8;
    int rc;
    if ((rc = grow(t->s3, 80ull * m)) || (rc = grow(t->oct, 8 * rs * m))) return rc;
    hipStream_t st = t->ctx->stream;
    const int32_t *cx = (const int32_t *)t->cx.p, *cy = (const int32_t *)t->cy.p,
                  *cz = (const int32_t *)t->cz.p;
    const Moments *mom = (const Moments *)t->mom.p;
    const Cube *cube = (const Cube *)t->cube.p;
    double *s3 = (double *)t->s3.p;
    if (t->dtype == BH_F32)
        k_oct_leaves<float><<<div_up(m, kThreads), kThreads, 0, st>>>(
            m, (const int32_t *)t->begin.p, (const int32_t *)t->count.p,
            (const int32_t *)t->next.p, cx, cy, cz, mom, cube, (const float *)t->spos.p,
            (const float *)t->smass.p, s3);
    else
        k_oct_leaves<double><<<div_up(m, kThreads), kThreads, 0, st>>>(
            m, (const int32_t *)t->begin.p, (const int32_t *)t->count.p,
            (const int32_t *)t->next.p, cx, cy, cz, mom, cube, (const double *)t->spos.p,
            (const double *)t->smass.p, s3);
    const int32_t *lvl_list = (const int32_t *)t->lvl_list.p;
    for (int k = t->depth - 1; k >= 0; --k) {
        if (t->lvl_cnt[k] == 0) continue;
        k_oct_level<<<div_up(t->lvl_cnt[k], kThreads), kThreads, 0, st>>>(
            lvl_list + t->lvl_base[k], t->lvl_cnt[k], (const int32_t *)t->kids.p, cx, cy, cz, mom,
            cube, s3);
    }
    if (t->dtype == BH_F32)
        k_oct_pack<float><<<div_up(m, kThreads), kThreads, 0, st>>>(m, s3, (float *)t->oct.p);
    else
        k_oct_pack<double><<<div_up(m, kThreads), kThreads, 0, st>>>(m, s3, (double *)t->oct.p);
    if ((rc = check_launch("octopole"))) return rc;
    t->oct_tree_id = t->build_id;
    return BH_OK;
}

int build_tree(bh_ctx *ctx, bh_tree *t, int curve, const void *pos, const void *mass,
               int dtype, int64_t n, int leaf, const void *vel, const uint32_t *id,
               void *pos_out, void *vel_out, void *mass_out, uint32_t *id_out, bool presorted) {
    // the nearly sorted re-sort needs this tree's previous build (same n,
    // same curve) complete: its sorted keys and its leaves
    const bool resort = presorted && ctx->sort_mode == BH_SORT_ADAPTIVE && t->resort_ok &&
                        t->n == n && t->curve == curve && t->m > 0 &&
                        t->sorted_keys != nullptr;
    t->resort_ok = false;
    t->dtype = dtype;
    t->n = n;
    t->leaf = leaf;
    t->curve = curve;
    t->build_id++;
    int rc;
    if (dtype == BH_F32)
        rc = build_typed<float>(ctx, t, (const float *)pos, (const float *)mass, (int)n, leaf,
                                (const float *)vel, id, (float *)pos_out, (float *)vel_out,
                                (float *)mass_out, id_out, resort);
    else
        rc = build_typed<double>(ctx, t, (const double *)pos, (const double *)mass, (int)n,
                                 leaf, (const double *)vel, id, (double *)pos_out,
                                 (double *)vel_out, (double *)mass_out, id_out, resort);
    t->resort_ok = rc == BH_OK;
    return rc;
}

}  // namespace bh
