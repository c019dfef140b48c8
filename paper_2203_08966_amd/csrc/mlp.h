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

// host entry points (mlp.hip)
int mlp_pack(bh_ctx *c);
// precision: BH_MLP_BF16 or BH_MLP_FP16 (both packings live in c->mlp_w)
int mlp_infer(bh_ctx *c, const float *X, int64_t n, int precision, float *pred);
int mlp_samples(bh_tree *t, double eps, double theta_lo, double theta_max, double keep,
                uint64_t seed, int64_t cap, float *feat, float *label, int32_t *node,
                int32_t *body, int64_t *total);
// features and k_C M l^3 of every cell (learned: the network; else k_C = 1),
// cached per tree build, eps and parameter version
int mlp_cells(bh_tree *t, double eps, bool learned, int precision);
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
