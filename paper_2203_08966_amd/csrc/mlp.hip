// Learned acceptance criterion on gfx950: training pairs, training kernels
// and the wave-level MFMA inference used inside the group walk.
//
// The criterion takes one decision per (group, cell): a network predicts
// log10 of the largest error the cell's quadrupole particle-cell term makes
// on the group's bodies in units of the error budget's model M l^3 / d_g^5
// (a coefficient k_C per group and cell), from 10 scale-free features of
// the (box, cell) pair; the cell is accepted iff
// pred + log10(M l^3 / d_g^5) < log10(tau a_min) (and its cube misses the
// box, and l < theta_max d_g).  The walk evaluates the network
// for the candidate cells of a round, one per lane, as one 64-row batch.
//
// Network 10 -> 32 (ReLU) -> 32 (ReLU) -> 1.  FP32 master parameters, flat:
// W1[32][10] b1[32] W2[32][32] b2[32] w3[32] b3 (1441 values).
//
// Inference is batched per wavefront: the 64 lanes' feature rows are one
// 64 x 16 operand (10 features, a constant 1 that carries b1, zero padding),
// split in two 32-sample blocks.  With v_mfma_f32_32x32x16_bf16,
//   H1^T (32 x 32) = W1e (32 x 16) . X^T (16 x 32)        1 MFMA per block
//   H2^T (32 x 32) = W2 (32 x 32) . H1^T + b2             2 MFMAs per block
// and the output layer is a per-lane dot product plus one cross-half add.
// The accumulator layout of the first product (lane l holds sample l%32,
// units 8(v/4) + 4(l/32) + v%4) is used directly as the B operand of the
// second by permuting W2's columns when packing (no data movement).
#include <math.h>

#include "bh_internal.h"
#include "mlp.h"

namespace bh {
namespace {

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// SplitMix64 finaliser (Steele, Lea & Flood 2014) of x + golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// k_C = 1: M l^3 per cell (the error-budget criterion without a network).
__global__ __launch_bounds__(256) void k_cell_kc_plain(int m, const Moments *__restrict__ mom,
                                                       const int32_t *__restrict__ level,
                                                       const Cube *__restrict__ cube,
                                                       float *__restrict__ kc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double side = ldexp(cube->L, -level[i]);
    kc[i] = (float)(mom[i].m * side * side * side);
}

// |a| per sorted rank i from element j of an acceleration array (or of an
// array of norms), j = perm[i] for arrays in caller order, else j = i.
// PERM: perm is given; NORM: norms are read (else accelerations).
constexpr int kAnormUnroll = 8;
template <typename R, bool PERM, bool NORM>
__global__ __launch_bounds__(256) void k_anorm(int n, const R *__restrict__ acc,
                                               const R *__restrict__ norm,
                                               const uint32_t *__restrict__ perm,
                                               float *__restrict__ out,
                                               double *__restrict__ part) {
    // grid-stride over the ranks (a fixed grid: the sum's order is fixed);
    // kAnormUnroll strides at a time, every load issued before the first
    // use, so that a thread's dependent loads (perm, then the element) do
    // not wait one stride after another; the sum keeps the stride order
    double sum = 0.0;
    const int stride = (int)(gridDim.x * blockDim.x);
    auto norm_at = [&](int64_t i) -> float {
        int64_t j = i;
        if constexpr (PERM) j = (int64_t)perm[i];
        if constexpr (NORM) {
            return (float)norm[j];
        } else {
            const R x = acc[3 * j], y = acc[3 * j + 1], z = acc[3 * j + 2];
            return (float)sqrt(x * x + y * y + z * z);
        }
    };
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (int64_t)(kAnormUnroll - 1) * stride < n; i += (int64_t)kAnormUnroll * stride) {
        float v[kAnormUnroll];
#pragma unroll
        for (int u = 0; u < kAnormUnroll; ++u) v[u] = norm_at(i + (int64_t)u * stride);
#pragma unroll
        for (int u = 0; u < kAnormUnroll; ++u) {
            out[i + (int64_t)u * stride] = v[u];
            sum += (double)v[u];
        }
    }
    for (; i < n; i += stride) {
        const float v = norm_at(i);
        out[i] = v;
        sum += (double)v;
    }
    // block sum of the stored norms, FP64: a butterfly within each
    // wavefront (lane 0's result is used), then the four wavefronts in order
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    __shared__ double ws[4];
    if (lane_id() == 0) ws[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// floor = f * (sum of the block sums) / n, one block, fixed order.
__global__ __launch_bounds__(1024) void k_anorm_floor(const double *__restrict__ part, int nblk,
                                                      int n, double f, float *__restrict__ floor_out) {
    __shared__ double s[1024];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 1024) v += part[b];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *floor_out = (float)(f * (s[0] / (double)n));
}

// ------------------------------------------------------------------ training pairs
// One wavefront per group of 64 consecutive sorted ranks [t0 + 64 q, ...),
// over the FP64 tree.  The group's decisions are wave-uniform, so its walk
// is a forward sweep with skip pointers: a multi-body cell whose cube
// misses the box with l < theta_lo d_g is skipped, every other cell opened;
// a cell whose cube misses the box with theta_lo d_g <= l < theta_max d_g is
// a candidate, kept when the hash of (seed, first rank, node) falls below
// `keep`.  A kept pair gets its features and the label
// log10(max_i |a_pc,i - a_exact,i| d_g^5 / (M l^3)) (each lane one body;
// a_exact the direct sum over the cell's bodies; floored at 1e-12).  Pass 1 (feat ==
// nullptr) counts per group; pass 2 writes at offs[q].
__global__ __launch_bounds__(256) void k_group_samples(
    const NodeRec64 *__restrict__ nodes, int m, const BodyRec<double> *__restrict__ bodies,
    const Anchor<double> *__restrict__ anchors, int nbodies, int t0, int t1, double tlo2,
    double tmax2,
    double eps, double keep, uint64_t seed, int32_t *__restrict__ cnt_out,
    const int64_t *__restrict__ offs, int64_t cap_total, float *__restrict__ feat,
    float *__restrict__ label, int32_t *__restrict__ node_out, int32_t *__restrict__ group_out) {
    const int q = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int ng = (t1 - t0 + 63) / 64;
    if (q >= ng) return;  // whole wave
    const int lane = (int)lane_id();
    const int g0 = t0 + 64 * q, g1 = min(g0 + 64, t1);
    const int i = g0 + lane;
    const bool live = i < g1;
    double px = 0, py = 0, pz = 0;  // body position relative to the root corner
    if (live) {
        const BodyRec<double> b = bodies[i];
        const Anchor<double> a = anchors[i];
        px = a.x + b.x;
        py = a.y + b.y;
        pz = a.z + b.z;
    }
    double lo3[3] = {live ? px : 1e300, live ? py : 1e300, live ? pz : 1e300};
    double hi3[3] = {live ? px : -1e300, live ? py : -1e300, live ? pz : -1e300};
    for (int o = 32; o > 0; o >>= 1)
        for (int d = 0; d < 3; ++d) {
            lo3[d] = fmin(lo3[d], __shfl_xor(lo3[d], o));
            hi3[d] = fmax(hi3[d], __shfl_xor(hi3[d], o));
        }
    const double bcx = 0.5 * (lo3[0] + hi3[0]), bcy = 0.5 * (lo3[1] + hi3[1]),
                 bcz = 0.5 * (lo3[2] + hi3[2]);
    const double bhx = 0.5 * (hi3[0] - lo3[0]), bhy = 0.5 * (hi3[1] - lo3[1]),
                 bhz = 0.5 * (hi3[2] - lo3[2]);
    const double e2 = eps * eps;
    const uint64_t keep_lim = (uint64_t)(keep * 9007199254740992.0);  // 2^53
    const int64_t o0 = offs ? offs[q] : 0;
    int k = 0;
    int idx = nodes[0].next == 1 ? m : 1;  // a root leaf has no candidates
    while (idx < m) {
        idx = uniform(idx);
        const NodeRec64 nd = nodes[idx];
        const int nxt = uniform(nd.next);
        if (nd.count == 1) {
            idx = nxt;
            continue;
        }
        const double hs = 0.5 * sqrt(nd.l2);
        const bool overlap = fabs(nd.cx - bcx) <= hs + bhx && fabs(nd.cy - bcy) <= hs + bhy &&
                             fabs(nd.cz - bcz) <= hs + bhz;
        const double ux = (nd.cx + nd.mx) - bcx, uy = (nd.cy + nd.my) - bcy,
                     uz = (nd.cz + nd.mz) - bcz;
        const double tx = fmax(fabs(ux) - bhx, 0.0), ty = fmax(fabs(uy) - bhy, 0.0),
                     tz = fmax(fabs(uz) - bhz, 0.0);
        const double dg2 = tx * tx + ty * ty + tz * tz;
        if (!overlap && nd.l2 < tlo2 * dg2) {
            idx = nxt;
            continue;
        }
        if (!overlap && nd.l2 < tmax2 * dg2 && nd.m > 0.0) {
            const uint64_t hkey = seed ^ (((uint64_t)g0 << 32) | (uint64_t)(uint32_t)idx);
            if ((splitmix64(hkey) >> 11) < keep_lim) {
                if (feat && o0 + k < cap_total) {
                    // this lane's body: exact sum over the cell's bodies and
                    // the cell's quadrupole particle-cell term
                    double err2 = 0.0;
                    if (live) {
                        double ex = 0, ey = 0, ez = 0;
                        for (int j = nd.begin; j < min(nd.begin + nd.count, nbodies); ++j) {
                            const BodyRec<double> sb = bodies[j];
                            const Anchor<double> sa = anchors[j];
                            const double dx = (sa.x + sb.x) - px, dy = (sa.y + sb.y) - py,
                                         dz = (sa.z + sb.z) - pz;
                            const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz + e2);
                            const double w = sb.m * ir * ir * ir;
                            ex += w * dx;
                            ey += w * dy;
                            ez += w * dz;
                        }
                        const double x = px - (nd.cx + nd.mx), y = py - (nd.cy + nd.my),
                                     z = pz - (nd.cz + nd.mz);
                        const double inv = 1.0 / sqrt(x * x + y * y + z * z + e2);
                        const double inv2 = inv * inv, inv3 = inv * inv2, inv5 = inv3 * inv2;
                        const double qzz = -nd.qxx - nd.qyy;
                        const double qx = nd.qxx * x + nd.qxy * y + nd.qxz * z;
                        const double qy = nd.qxy * x + nd.qyy * y + nd.qyz * z;
                        const double qz = nd.qxz * x + nd.qyz * y + qzz * z;
                        const double xqx = x * qx + y * qy + z * qz;
                        const double g = nd.m * inv3 + 2.5 * xqx * inv5 * inv2;
                        const double ax = inv5 * qx - g * x - ex, ay = inv5 * qy - g * y - ey,
                                     az = inv5 * qz - g * z - ez;
                        err2 = ax * ax + ay * ay + az * az;
                    }
                    for (int o = 32; o > 0; o >>= 1) err2 = fmax(err2, __shfl_xor(err2, o));
                    float f[kMlpIn];
                    gfeatures<double>(ux, uy, uz, bhx, bhy, bhz, nd.mx, nd.my, nd.mz, nd.m,
                                      nd.qxx, nd.qxy, nd.qxz, nd.qyy, nd.qyz, nd.l2, nd.count,
                                      nxt == idx + 1, eps, f);
                    if (lane == 0) {
                        const int64_t s = o0 + k;
                        double v = sqrt(err2) * dg2 * dg2 * sqrt(dg2) / (nd.m * nd.l2 * sqrt(nd.l2));
                        v = v > 1e-12 ? v : 1e-12;
                        for (int c = 0; c < kMlpIn; ++c) feat[kMlpIn * s + c] = f[c];
                        label[s] = (float)log10(v);
                        node_out[s] = idx;
                        group_out[s] = g0;
                    }
                }
                ++k;
            }
        }
        idx = nxt == idx + 1 ? nxt : idx + 1;  // a leaf is done; open the rest
    }
    if (cnt_out && lane == 0) cnt_out[q] = k;
}

// exclusive scan of n counts (one block, any n), total at out[n]
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t *__restrict__ c, int n,
                                                      int64_t *__restrict__ out) {
    __shared__ int64_t carry;
    __shared__ int64_t ws[16];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int64_t x = i < n ? c[i] : 0;
        int64_t incl = x;
        const unsigned lane = lane_id();
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t v = __shfl_up(incl, o);
            if ((int)lane >= o) incl += v;
        }
        const int w = threadIdx.x / 64;
        if (lane == 63) ws[w] = incl;
        __syncthreads();
        int64_t pre = carry;
        for (int k = 0; k < w; ++k) pre += ws[k];
        if (i < n) out[i] = pre + incl - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry = pre + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// ------------------------------------------------------------------ training
// One wavefront per block of kTrainBlock samples, in tiles of 32, with FP32
// MFMA (v_mfma_f32_32x32x2_f32: A 32x2, one value per lane at row l%32 and
// k l/32; B 2x32 at k l/32 and column l%32; D 32x32, register v of lane l
// at row 8(v/4) + 4(l/32) + v%4 and column l%32).  Products take hidden
// units down the rows and the tile's samples across the columns, the layout
// of the inference; an accumulator then feeds the next product as its B
// operand register by register, if the product's K runs over the units in
// the order its rows hold them (kappa below).
constexpr int kTrainBlock = 128;  // samples per block
constexpr int kTrainTile = 32;    // samples per MFMA column block

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, const f32x16 &c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// the row (hidden unit) of accumulator register v on a lane of half-wave h
__device__ __forceinline__ int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Gradient of the loss over one minibatch: mean-squared error (quantile 0)
// or the pinball loss of quantile q (derivative 1 - q where the prediction
// exceeds the label, else -q).  Sample j of the batch is sample
// (a * (base + j) + c) mod ns of the set (a permutation of the set per
// epoch).  Each block writes its partial gradient and loss; sums run in a
// fixed order (tiles, then the MFMA's own), so the result is deterministic.
__global__ __launch_bounds__(64) void k_mlp_grad(
    const float *__restrict__ w, const float *__restrict__ X, const float *__restrict__ y,
    int64_t ns, int64_t base, int bs, uint64_t a, uint64_t c, float quantile,
    float *__restrict__ gpart) {
    __shared__ float sw[kMlpParams];
    __shared__ float sa[kMlpHidden][kTrainTile + 1];  // transposes: unit x sample
    __shared__ float sb[kMlpHidden][kTrainTile + 1];
    __shared__ float sx[kTrainTile][16];              // features, 1 (bias slot), 0
    const int l = (int)threadIdx.x;
    const int h = l >> 5, r = l & 31;
    for (int k = l; k < kMlpParams; k += 64) sw[k] = w[k];
    __syncthreads();
    const float *W1 = sw, *b1 = sw + 320, *W2 = sw + 352, *b2 = sw + 1376, *w3 = sw + 1408;
    const float b3 = sw[1440];
    // operands that stay over the tiles
    float A1[8], A2[16], AT[16], b2v[16], w3v[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 2 * i + h;  // feature slot: 0..9 weights, 10 bias, 11..15 zero
        A1[i] = k < kMlpIn ? W1[r * kMlpIn + k] : (k == kMlpIn ? b1[r] : 0.f);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int kap = acc_row(i, h);
        A2[i] = W2[r * kMlpHidden + kap];  // row r of W2, K in row order
        AT[i] = W2[kap * kMlpHidden + r];  // row r of W2^T
        b2v[i] = b2[acc_row(i, h)];
        w3v[i] = w3[acc_row(i, h)];
    }
    f32x16 gW1 = {}, gW2 = {};
    float gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
    for (int t = 0; t < kTrainBlock / kTrainTile; ++t) {
        const int j = blockIdx.x * kTrainBlock + t * kTrainTile + r;  // this lane's sample
        const bool live = j < bs;
        float yy = 0.f;
        if (h == 0) {
            float x[kMlpIn] = {};
            if (live) {
                const uint64_t g = base + (uint64_t)j;
                const int64_t sidx = (int64_t)((a * (g % (uint64_t)ns) + c) % (uint64_t)ns);
                for (int q = 0; q < kMlpIn; ++q) x[q] = X[kMlpIn * sidx + q];
            }
            for (int q = 0; q < 16; ++q) sx[r][q] = q < kMlpIn ? x[q] : (q == kMlpIn ? 1.f : 0.f);
        }
        if (live) {
            const uint64_t g = base + (uint64_t)j;
            yy = y[(int64_t)((a * (g % (uint64_t)ns) + c) % (uint64_t)ns)];
        }
        __syncthreads();
        // forward: z1 = W1e xe, z2 = W2 relu(z1) + b2 (rows: units, columns: samples)
        f32x16 z1 = {};
#pragma unroll
        for (int i = 0; i < 8; ++i) z1 = mfma_f32(A1[i], sx[r][2 * i + h], z1);
        f32x16 z2;
#pragma unroll
        for (int v = 0; v < 16; ++v) z2[v] = b2v[v];
#pragma unroll
        for (int i = 0; i < 16; ++i) z2 = mfma_f32(A2[i], fmaxf(z1[i], 0.f), z2);
        float p = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) p += w3v[v] * fmaxf(z2[v], 0.f);
        const float out = p + __shfl_xor(p, 32) + b3;  // sample r, on both halves
        float dout, lv;
        if (quantile > 0.f) {
            const bool over = out > yy;
            dout = (over ? 1.f - quantile : -quantile) / (float)bs;
            lv = over ? (1.f - quantile) * (out - yy) : quantile * (yy - out);
        } else {
            dout = 2.f * (out - yy) / (float)bs;
            lv = (out - yy) * (out - yy);
        }
        if (!live) dout = lv = 0.f;
        // backward: d2 = dout w3 relu'(z2); d1 = (W2^T d2) relu'(z1)
        f32x16 d2, e1 = {};
#pragma unroll
        for (int v = 0; v < 16; ++v) d2[v] = z2[v] > 0.f ? dout * w3v[v] : 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) e1 = mfma_f32(AT[i], d2[i], e1);
        // dW2 = sum over samples of d2 h1^T: both operands transposed
        // through LDS (row u = r, k = sample)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            sa[acc_row(v, h)][r] = d2[v];
            sb[acc_row(v, h)][r] = fmaxf(z1[v], 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) gW2 = mfma_f32(sa[r][2 * i + h], sb[r][2 * i + h], gW2);
        if (h == 0)  // b2: the row sums of d2
            for (int q = 0; q < kTrainTile; ++q) gb2 += sa[r][q];
        __syncthreads();
        // w3: the row sums of dout h2; then dW1 = sum of d1 xe^T (its bias
        // column is b1's gradient)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            sa[acc_row(v, h)][r] = dout * fmaxf(z2[v], 0.f);
            sb[acc_row(v, h)][r] = z1[v] > 0.f ? e1[v] : 0.f;
        }
        __syncthreads();
        if (h == 0)
            for (int q = 0; q < kTrainTile; ++q) gw3 += sa[r][q];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            gW1 = mfma_f32(sb[r][2 * i + h], r < 16 ? sx[2 * i + h][r] : 0.f, gW1);
        __syncthreads();
        // b3 and the loss: sums over the tile's samples in sample order
        if (h == 0) sa[0][r] = dout;
        __syncthreads();
        if (l == 0) {
            for (int q = 0; q < kTrainTile; ++q) gb3 += sa[0][q];
        }
        __syncthreads();
        if (h == 0) sa[0][r] = lv;
        __syncthreads();
        if (l == 0)
            for (int q = 0; q < kTrainTile; ++q) lsum += sa[0][q];
        __syncthreads();
    }
    float *gp = gpart + (size_t)blockIdx.x * (kMlpParams + 1);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int u = acc_row(v, h);
        if (r < kMlpIn) gp[u * kMlpIn + r] = gW1[v];
        else if (r == kMlpIn) gp[320 + u] = gW1[v];
        gp[352 + u * kMlpHidden + r] = gW2[v];
    }
    if (h == 0) {
        gp[1376 + r] = gb2;
        gp[1408 + r] = gw3;
    }
    if (l == 0) {
        gp[1440] = gb3;
        gp[1441] = lsum;
    }
}

// Sum the partial gradients in block order; Adam step t (1-based).
__global__ __launch_bounds__(256) void k_mlp_adam(const float *__restrict__ gpart, int nblk,
                                                  float *__restrict__ w, float *__restrict__ m1,
                                                  float *__restrict__ m2, float *__restrict__ g_out,
                                                  float *__restrict__ loss_acc, float lr, float b1,
                                                  float b2, float eps, float c1, float c2,
                                                  int apply) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kMlpParams) return;
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += gpart[(size_t)b * (kMlpParams + 1) + k];
    if (k == kMlpParams) {  // loss
        if (loss_acc) loss_acc[0] += g;
        return;
    }
    if (g_out) g_out[k] = g;
    if (!apply) return;
    const float mm = b1 * m1[k] + (1.f - b1) * g;
    const float vv = b2 * m2[k] + (1.f - b2) * g * g;
    m1[k] = mm;
    m2[k] = vv;
    w[k] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ------------------------------------------------------------------ inference
// Pack FP32 master parameters into the per-lane MFMA operand layout, in
// the element type of V.
template <typename V>
__device__ __forceinline__ void mlp_pack_as(const float *__restrict__ w, MlpPacked *__restrict__ p,
                                            int l) {
    using E = typename VecElem<V>::type;
    const float *W1 = w, *b1 = w + 320, *W2 = w + 352, *b2 = w + 1376, *w3 = w + 1408;
    const int row = l & 31, h = l >> 5;
    V v1;
    for (int q = 0; q < 8; ++q) {
        const int k = 8 * h + q;  // feature slot: 0..9 weights, 10 bias, rest 0
        const float v = k < kMlpIn ? W1[row * kMlpIn + k] : (k == kMlpIn ? b1[row] : 0.f);
        v1[q] = (E)v;
    }
    p->a1[l] = __builtin_bit_cast(u32x4, v1);
    for (int c = 0; c < 2; ++c) {
        V v2;
        for (int q = 0; q < 8; ++q) {
            const int unit = q < 4 ? 16 * c + 4 * h + q : 16 * c + 8 + 4 * h + (q - 4);
            v2[q] = (E)W2[row * kMlpHidden + unit];
        }
        p->a2[c][l] = __builtin_bit_cast(u32x4, v2);
    }
    for (int v = 0; v < 16; ++v) {
        const int unit = 8 * (v / 4) + 4 * h + (v % 4);
        p->b2d[l][v] = b2[unit];
        p->w3d[l][v] = w3[unit];
    }
    if (l == 0) p->b3 = w[1440];
}

// both packings: p[BH_MLP_BF16] and p[BH_MLP_FP16]
__global__ __launch_bounds__(64) void k_mlp_pack(const float *__restrict__ w,
                                                 MlpPacked *__restrict__ p) {
    mlp_pack_as<bf16x8>(w, p + BH_MLP_BF16, threadIdx.x);
    mlp_pack_as<f16x8>(w, p + BH_MLP_FP16, threadIdx.x);
}

template <typename V>
__global__ __launch_bounds__(256) void k_mlp_infer(const MlpPacked *__restrict__ p,
                                                   const float *__restrict__ X, int n,
                                                   float *__restrict__ pred) {
    const int wave = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wave * 64 >= n) return;  // whole wave: the MFMAs need every lane
    const int l = (int)lane_id();
    const int i = wave * 64 + l;
    MlpRegs<V> r;
    mlp_load(p, l, r);
    float f[kMlpIn];
    for (int q = 0; q < kMlpIn; ++q) f[q] = i < n ? X[kMlpIn * i + q] : 0.f;
    const float y = mlp_eval(r, f, l);
    if (i < n) pred[i] = y;
}

}  // namespace

// ------------------------------------------------------------------ host side
int mlp_pack(bh_ctx *c) {
    int rc = grow(c->mlp_w, 2 * sizeof(MlpPacked));
    if (rc) return rc;
    k_mlp_pack<<<1, 64, 0, c->stream>>>((const float *)c->mlp_master.p, (MlpPacked *)c->mlp_w.p);
    rc = check_launch("mlp pack");
    if (!rc) {
        c->mlp_loaded = 1;
        c->mlp_version++;  // group-walk predictions made with the old network are stale
    }
    return rc;
}

int mlp_infer(bh_ctx *c, const float *X, int64_t n, int precision, float *pred) {
    const MlpPacked *p = (const MlpPacked *)c->mlp_w.p + precision;
    if (precision == BH_MLP_FP16)
        k_mlp_infer<f16x8><<<div_up(n, 256), 256, 0, c->stream>>>(p, X, (int)n, pred);
    else
        k_mlp_infer<bf16x8><<<div_up(n, 256), 256, 0, c->stream>>>(p, X, (int)n, pred);
    return check_launch("mlp infer");
}

// (every build writes M l^3 with its upward pass: this recomputes it only
// for a tree whose build did not)
int mlp_cells(bh_tree *t) {
    if (t->kc_tree_id == t->build_id) return BH_OK;
    const int m = (int)t->m;
    int rc = grow(t->kc, 4ull * m);
    if (rc) return rc;
    k_cell_kc_plain<<<div_up(m, 256), 256, 0, t->ctx->stream>>>(
        m, (const Moments *)t->mom.p, (const int32_t *)t->level.p, (const Cube *)t->cube.p,
        (float *)t->kc.p);
    if ((rc = check_launch("mlp cells"))) return rc;
    t->kc_tree_id = t->build_id;
    return BH_OK;
}

// blocks of k_anorm (at most; its block sums sit in a fixed-size slot)
constexpr int kAnormBlocks = 1024;

int mlp_anorm(bh_tree *t, const void *acc, const void *norm, bool caller_order,
              double floor_frac) {
    const int n = (int)t->n;
    const int nblk = min(kAnormBlocks, div_up(n, 256));
    const size_t npad = 4ull * (size_t)div_up(n, 64) * 64;  // norms, then block sums, floor
    int rc = grow(t->anorm, npad + 8ull * kAnormBlocks + 8);
    if (rc) return rc;
    const uint32_t *perm = caller_order ? t->perm : nullptr;
    double *part = (double *)((char *)t->anorm.p + npad);
    auto launch = [&](auto zero) {
        using R = decltype(zero);
        const R *a = (const R *)acc, *nm = (const R *)norm;
        float *out = (float *)t->anorm.p;
        hipStream_t st = t->ctx->stream;
        if (perm && norm)
            k_anorm<R, true, true><<<nblk, 256, 0, st>>>(n, a, nm, perm, out, part);
        else if (perm)
            k_anorm<R, true, false><<<nblk, 256, 0, st>>>(n, a, nm, perm, out, part);
        else if (norm)
            k_anorm<R, false, true><<<nblk, 256, 0, st>>>(n, a, nm, perm, out, part);
        else
            k_anorm<R, false, false><<<nblk, 256, 0, st>>>(n, a, nm, perm, out, part);
    };
    if (t->dtype == BH_F32)
        launch(0.0f);
    else
        launch(0.0);
    k_anorm_floor<<<1, 1024, 0, t->ctx->stream>>>(part, nblk, n, floor_frac,
                                                  (float *)(part + kAnormBlocks));
    return check_launch("anorm");
}

const float *mlp_anorm_floor(const bh_tree *t) {
    const size_t npad = 4ull * (size_t)div_up((int)t->n, 64) * 64;
    return (const float *)((const char *)t->anorm.p + npad + 8ull * kAnormBlocks);
}

int mlp_samples(bh_tree *t, double eps, double theta_lo, double theta_max, double keep,
                uint64_t seed, int64_t cap, float *feat, float *label, int32_t *node,
                int32_t *group, int64_t *total) {
    bh_ctx *c = t->ctx;
    const int n = (int)t->n;
    const int ng = div_up(n, 64);
    int rc = grow(c->mlp_scratch, 4ull * ng + 8ull * (ng + 1) + 8);
    if (rc) return rc;
    int32_t *cnt = (int32_t *)c->mlp_scratch.p;
    int64_t *offs = (int64_t *)((char *)c->mlp_scratch.p + 4ull * ng + (4ull * ng) % 8);
    const int nblk = div_up(ng, 4);
    const NodeRec64 *nodes = (const NodeRec64 *)t->recs.p;
    const auto *bodies = (const BodyRec<double> *)t->bodies.p;
    const auto *anchors = (const Anchor<double> *)t->anchors.p;
    k_group_samples<<<nblk, 256, 0, c->stream>>>(nodes, (int)t->m, bodies, anchors, n, 0, n,
                                                 theta_lo * theta_lo, theta_max * theta_max, eps,
                                                 keep, seed, cnt, nullptr, 0, nullptr, nullptr,
                                                 nullptr, nullptr);
    k_scan_counts<<<1, 1024, 0, c->stream>>>(cnt, ng, offs);
    int64_t *hp = (int64_t *)((char *)c->pinned + 2048);
    if ((rc = check_launch("mlp samples")) ||
        hipMemcpyAsync(hp, offs + ng, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return rc ? rc : set_error(BH_E_DEVICE, "sample count copy failed");
    *total = hp[0];
    if (!feat) return BH_OK;
    if (*total > cap)
        return set_error(BH_E_INVALID, "sample capacity too small: need " + std::to_string(*total));
    k_group_samples<<<nblk, 256, 0, c->stream>>>(nodes, (int)t->m, bodies, anchors, n, 0, n,
                                                 theta_lo * theta_lo, theta_max * theta_max, eps,
                                                 keep, seed, nullptr, offs, cap, feat, label, node,
                                                 group);
    return check_launch("mlp samples");
}

int mlp_grad_step(bh_ctx *c, const float *X, const float *y, int64_t ns, int64_t base, int bs,
                  uint64_t a, uint64_t cc, float *g_out, float *loss_acc, bool apply, int step,
                  const MlpTrainCfg &cfg) {
    const int nblk = div_up(bs, kTrainBlock);
    int rc = grow(c->mlp_gpart, 4ull * (kMlpParams + 1) * nblk);
    if (rc) return rc;
    k_mlp_grad<<<nblk, 64, 0, c->stream>>>((const float *)c->mlp_master.p, X, y, ns, base,
                                                    bs, a, cc, cfg.quantile,
                                                    (float *)c->mlp_gpart.p);
    const float c1 = 1.f - powf(cfg.beta1, (float)step), c2 = 1.f - powf(cfg.beta2, (float)step);
    float *mst = (float *)c->mlp_master.p;
    k_mlp_adam<<<div_up(kMlpParams + 1, 256), 256, 0, c->stream>>>(
        (const float *)c->mlp_gpart.p, nblk, mst, mst + kMlpParams, mst + 2 * kMlpParams, g_out,
        loss_acc, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, c1, c2, apply ? 1 : 0);
    return check_launch("mlp train");
}

}  // namespace bh
