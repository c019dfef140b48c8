// Learned acceptance criterion: packed inference weights and the wave-level
// MFMA evaluation in bf16 or fp16 (gfx950, v_mfma_f32_32x32x16_bf16 /
// v_mfma_f32_32x32x16_f16: the same operand layout).
#pragma once

#include <type_traits>

#include "bh_internal.h"

namespace bh {

constexpr int kMlpIn = 10;
constexpr int kMlpHidden = 32;
constexpr int kMlpParams = 1441;  // W1 320, b1 32, W2 1024, b2 32, w3 32, b3 1

struct MlpTrainCfg {
    float lr, beta1, beta2, eps;
    float quantile;  // 0: mean-squared error; in (0, 1): pinball loss
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// element type of an 8-wide MFMA operand
template <typename V> struct VecElem;
template <> struct VecElem<bf16x8> { using type = __bf16; };
template <> struct VecElem<f16x8> { using type = _Float16; };

template <typename V>
__device__ __forceinline__ f32x16 mfma32(const V &a, const V &b, const f32x16 &c) {
    if constexpr (std::is_same<V, f16x8>::value)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Per-lane operands, lane l of the wave:
//  a1[l]    row l%32 of W1e = [W1 | b1 | 0] (hidden unit), feature slots
//           8(l/32) .. +7 (A operand of H1^T = W1e X^T)
//  a2[c][l] row l%32 of W2, K slots 16c + 8(l/32) + q mapped to hidden unit
//           16c + 4(l/32) + q (q < 4) or 16c + 8 + 4(l/32) + q - 4 (q >= 4),
//           which is where the first product leaves those units
//  b2d/w3d  b2 and w3 of the units lane l holds in an accumulator:
//           unit 8(v/4) + 4(l/32) + v%4 for register v
struct MlpPacked {
    u32x4 a1[64];
    u32x4 a2[2][64];
    float b2d[64][16];
    float w3d[64][16];
    float b3;
};

template <typename V>
struct MlpRegs {
    V a1;
    V a2[2];
    float b2d[16];
    float w3d[16];
    float b3;
};

template <typename V>
__device__ __forceinline__ void mlp_load(const MlpPacked *__restrict__ p, int l, MlpRegs<V> &r) {
    r.a1 = __builtin_bit_cast(V, p->a1[l]);
    r.a2[0] = __builtin_bit_cast(V, p->a2[0][l]);
    r.a2[1] = __builtin_bit_cast(V, p->a2[1][l]);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        r.b2d[v] = p->b2d[l][v];
        r.w3d[v] = p->w3d[l][v];
    }
    r.b3 = p->b3;
}

// Prediction for this lane's feature row.  Must be called by all 64 lanes
// of the wave (uniform control flow).
template <typename V>
__device__ __forceinline__ float mlp_eval(const MlpRegs<V> &r, const float *f, int l) {
    using E = typename VecElem<V>::type;
    V lo, hi;
#pragma unroll
    for (int q = 0; q < 8; ++q) lo[q] = (E)f[q];
    hi[0] = (E)f[8];
    hi[1] = (E)f[9];
    hi[2] = (E)1.0f;
#pragma unroll
    for (int q = 3; q < 8; ++q) hi[q] = (E)0.0f;
    const bool upper = l >= 32;
    // samples 0..31 are lanes 0..31, samples 32..63 lanes 32..63; the B
    // operand wants slots 0..7 of a sample in the lower half-wave and slots
    // 8..15 in the upper half: exchange across the halves
    const u32x4 send = __builtin_bit_cast(u32x4, upper ? lo : hi);
    u32x4 recv;
#pragma unroll
    for (int w = 0; w < 4; ++w) recv[w] = __shfl_xor(send[w], 32);
    const V B0 = upper ? __builtin_bit_cast(V, recv) : lo;
    const V B1 = upper ? hi : __builtin_bit_cast(V, recv);
    const f32x16 zero = {};
    const f32x16 d0 = mfma32<V>(r.a1, B0, zero);
    const f32x16 d1 = mfma32<V>(r.a1, B1, zero);
    V h00, h01, h10, h11;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        h00[q] = (E)fmaxf(d0[q], 0.f);
        h01[q] = (E)fmaxf(d0[8 + q], 0.f);
        h10[q] = (E)fmaxf(d1[q], 0.f);
        h11[q] = (E)fmaxf(d1[8 + q], 0.f);
    }
    f32x16 c2;
#pragma unroll
    for (int v = 0; v < 16; ++v) c2[v] = r.b2d[v];
    f32x16 e0 = mfma32<V>(r.a2[0], h00, c2);
    e0 = mfma32<V>(r.a2[1], h01, e0);
    f32x16 e1 = mfma32<V>(r.a2[0], h10, c2);
    e1 = mfma32<V>(r.a2[1], h11, e1);
    float p0 = 0.f, p1 = 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        p0 += r.w3d[v] * fmaxf(e0[v], 0.f);
        p1 += r.w3d[v] * fmaxf(e1[v], 0.f);
    }
    p0 += __shfl_xor(p0, 32);
    p1 += __shfl_xor(p1, 32);
    return (upper ? p1 : p0) + r.b3;
}

// Prediction for this lane's feature row with the packed parameters at p
// (LDS or global memory), for callers short of registers: the two blocks of
// 32 samples one after the other (a loop the compiler keeps rolled), the
// operands read from p where they are used, so that one block's
// accumulators (16 registers) are live at a time.  Must be called by all 64
// lanes of the wave.
template <typename V>
__device__ __forceinline__ float mlp_eval_p(const MlpPacked *__restrict__ p, const float *f, int l) {
    using E = typename VecElem<V>::type;
    // the lane index through an empty asm: the operand loads below then do
    // not look loop-invariant to the caller's loops, so the compiler does
    // not hoist the parameters into registers for a whole walk
    __asm__ volatile("" : "+v"(l));
    V lo, hi;
#pragma unroll
    for (int q = 0; q < 8; ++q) lo[q] = (E)f[q];
    hi[0] = (E)f[8];
    hi[1] = (E)f[9];
    hi[2] = (E)1.0f;
#pragma unroll
    for (int q = 3; q < 8; ++q) hi[q] = (E)0.0f;
    const bool upper = l >= 32;
    // the B operand of sample block b: slots 0..7 of its samples in the lower
    // half-wave, slots 8..15 in the upper half (exchange across the halves)
    const u32x4 send = __builtin_bit_cast(u32x4, upper ? lo : hi);
    u32x4 recv;
#pragma unroll
    for (int w = 0; w < 4; ++w) recv[w] = __shfl_xor(send[w], 32);
    const V Bmine = upper ? hi : lo;
    const V Bother = __builtin_bit_cast(V, recv);
    float out = 0.f;
#pragma unroll 1
    for (int blk = 0; blk < 2; ++blk) {
        // block 0 holds lanes 0..31's samples: lower lanes give their own
        // slots 0..7, upper lanes the received ones; block 1 the reverse
        const V B = (blk == 0) == upper ? Bother : Bmine;
        const V a1 = __builtin_bit_cast(V, p->a1[l]);
        const f32x16 zero = {};
        const f32x16 d = mfma32<V>(a1, B, zero);
        V h0, h1;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            h0[q] = (E)fmaxf(d[q], 0.f);
            h1[q] = (E)fmaxf(d[8 + q], 0.f);
        }
        f32x16 e;
#pragma unroll
        for (int v = 0; v < 16; ++v) e[v] = p->b2d[l][v];
        e = mfma32<V>(__builtin_bit_cast(V, p->a2[0][l]), h0, e);
        e = mfma32<V>(__builtin_bit_cast(V, p->a2[1][l]), h1, e);
        float s = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) s += p->w3d[l][v] * fmaxf(e[v], 0.f);
        s += __shfl_xor(s, 32);
        if ((blk == 1) == upper) out = s;
    }
    return out + p->b3;
}

template <typename R> __device__ __forceinline__ R lg2(R x);
template <> __device__ __forceinline__ float lg2<float>(float x) { return __builtin_amdgcn_logf(x); }
template <> __device__ __forceinline__ double lg2<double>(double x) { return ::log2(x); }

// Features of a (group box, cell) pair for the learned criterion, all
// scale-free (l side, d_g distance from the COM to the box, d_c to the box
// centre, h the box's half-diagonal, n the unit vector from the box centre
// to the COM, g = COM - cell centre, Q the traceless quadrupole):
//   f0 log2(l/d_g) in [-8, 8]     f1 min(log2(d_c/d_g), 8)
//   f2 h / (h + d_g)              f3 n.Q.n / (M l^2)
//   f4 |Q|_F / (M l^2)            f5 g.n / l
//   f6 |g| / l                    f7 log2(count) / 21
//   f8 min(eps / d_g, 1)          f9 1 for a leaf
// u: COM relative to the box centre; b: box half extents; q: xx xy xz yy yz.
// Returns d_g^2.
template <typename R>
__device__ __forceinline__ R gfeatures(R ux, R uy, R uz, R bx, R by, R bz, R gx, R gy, R gz, R m,
                                       R qxx, R qxy, R qxz, R qyy, R qyz, R l2, int count,
                                       bool leaf, R eps, float *f) {
    const R dc2 = ux * ux + uy * uy + uz * uz;
    const R tx = fmax(fabs(ux) - bx, (R)0), ty = fmax(fabs(uy) - by, (R)0),
            tz = fmax(fabs(uz) - bz, (R)0);
    const R dg2 = tx * tx + ty * ty + tz * tz;
    const R dg = sqrt(dg2), h = sqrt(bx * bx + by * by + bz * bz), side = sqrt(l2);
    const R inv_dc = dc2 > (R)0 ? (R)1 / sqrt(dc2) : (R)0;
    const R nx = ux * inv_dc, ny = uy * inv_dc, nz = uz * inv_dc;
    const R qzz = -qxx - qyy;
    const R nqn = nx * (qxx * nx + qxy * ny + qxz * nz) + ny * (qxy * nx + qyy * ny + qyz * nz) +
                  nz * (qxz * nx + qyz * ny + qzz * nz);
    const R qf = sqrt(qxx * qxx + qyy * qyy + qzz * qzz +
                      (R)2 * (qxy * qxy + qxz * qxz + qyz * qyz));
    const R ml2 = m * l2;
    const R f0 = dg2 > (R)0 ? (R)0.5 * lg2<R>(l2 / dg2) : (R)8;
    const R f1 = dg2 > (R)0 ? (R)0.5 * lg2<R>(dc2 / dg2) : (R)8;
    f[0] = (float)fmin(fmax(f0, (R)-8), (R)8);
    f[1] = (float)fmin(f1, (R)8);
    f[2] = h + dg > (R)0 ? (float)(h / (h + dg)) : 0.f;
    f[3] = ml2 > (R)0 ? (float)(nqn / ml2) : 0.f;
    f[4] = ml2 > (R)0 ? (float)(qf / ml2) : 0.f;
    f[5] = (float)((gx * nx + gy * ny + gz * nz) / side);
    f[6] = (float)(sqrt(gx * gx + gy * gy + gz * gz) / side);
    f[7] = (float)(lg2<R>((R)count) * (R)(1.0 / 21.0));
    f[8] = dg > (R)0 ? (float)fmin(eps / dg, (R)1) : 1.f;
    f[9] = leaf ? 1.f : 0.f;
    return dg2;
}

// host entry points (mlp.hip)
int mlp_pack(bh_ctx *c);
// precision: BH_MLP_BF16 or BH_MLP_FP16 (both packings live in c->mlp_w)
int mlp_infer(bh_ctx *c, const float *X, int64_t n, int precision, float *pred);
// training pairs of the learned criterion: groups of 64 consecutive sorted
// ranks, candidates theta_lo <= l/d_g < theta_max kept by hash (FP64 tree)
int mlp_samples(bh_tree *t, double eps, double theta_lo, double theta_max, double keep,
                uint64_t seed, int64_t cap, float *feat, float *label, int32_t *node,
                int32_t *group, int64_t *total);
// M l^3 of every cell (the error budget's k_C = 1 coefficient), cached per
// tree build
int mlp_cells(bh_tree *t);
// |a| per sorted rank into t->anorm from an acceleration array (acc) or an
// array of norms (norm), of the tree's dtype, in caller order (read through
// perm) or in sorted order; also the floor floor_frac * mean |a| (device
// scalar, mlp_anorm_floor)
int mlp_anorm(bh_tree *t, const void *acc, const void *norm, bool caller_order,
              double floor_frac);
const float *mlp_anorm_floor(const bh_tree *t);
int mlp_grad_step(bh_ctx *c, const float *X, const float *y, int64_t ns, int64_t base, int bs,
                  uint64_t a, uint64_t cc, float *g_out, float *loss_acc, bool apply, int step,
                  const MlpTrainCfg &cfg);

}  // namespace bh
