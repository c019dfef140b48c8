// Integration, energy and direct summation on gfx950.
//
//  kick / drift   KDK leapfrog with a fixed step (Sec. 2.3)
//  energy         E_kin = sum m v^2 / 2, E_pot = sum m phi / 2 (Sec. 2.4, each
//                 pair once), FP64 accumulation in a fixed order
//  direct         O(N * targets) direct sum (Sec. 2.1): in FP64 as the reference
//                 for the tree walk's error, and in the simulation's own
//                 precision as the direct method of Sec. 3 (every pair, no
//                 tree); sources staged through LDS
//  standard units the scaling of Sec. 2.4 (total mass 1, centre-of-mass
//                 frame, virial ratio 1/2, total energy -1/4)
#include <algorithm>
#include <cmath>

#include "bh_internal.h"

namespace bh {
namespace {

// The kicks and drifts stream the 3n components as 16-byte vectors (the
// simulation's buffers are 16-byte aligned), then the last components one
// by one; each component's arithmetic is the same either way.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
    using type = float4;
    static constexpr int N = 4;
};
template <> struct Vec16<double> {
    using type = double2;
    static constexpr int N = 2;
};
template <typename T> __device__ __forceinline__ T &comp(typename Vec16<T>::type &v, int k) {
    return reinterpret_cast<T *>(&v)[k];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kick(int64_t n3, T *__restrict__ v,
                                                   const T *__restrict__ a, T h) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::N;
    const int64_t nv = n3 / W, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = t; i < nv; i += stride) {
        V vv = reinterpret_cast<V *>(v)[i];
        V av = reinterpret_cast<const V *>(a)[i];
#pragma unroll
        for (int k = 0; k < W; ++k) comp<T>(vv, k) += comp<T>(av, k) * h;
        reinterpret_cast<V *>(v)[i] = vv;
    }
    for (int64_t i = nv * W + t; i < n3; i += stride) v[i] += a[i] * h;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kick_drift(int64_t n3, T *__restrict__ x,
                                                         T *__restrict__ v,
                                                         const T *__restrict__ a, T h, T dt) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::N;
    const int64_t nv = n3 / W, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = t; i < nv; i += stride) {
        V vv = reinterpret_cast<V *>(v)[i];
        V av = reinterpret_cast<const V *>(a)[i];
        V xv = reinterpret_cast<V *>(x)[i];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const T vi = comp<T>(vv, k) + comp<T>(av, k) * h;
            comp<T>(vv, k) = vi;
            comp<T>(xv, k) += vi * dt;
        }
        reinterpret_cast<V *>(v)[i] = vv;
        reinterpret_cast<V *>(x)[i] = xv;
    }
    for (int64_t i = nv * W + t; i < n3; i += stride) {
        const T vi = v[i] + a[i] * h;
        v[i] = vi;
        x[i] += vi * dt;
    }
}

// Adds sum(a), sum(b) and sum(c) (per-body interaction counts) into out[0],
// out[1], out[2]: per-thread 64-bit sums, a wavefront reduction, the block's
// wavefronts in LDS, one atomic per block and sum.
__global__ __launch_bounds__(kThreads) void k_count_sum(int64_t n, const uint32_t *__restrict__ a,
                                                        const uint32_t *__restrict__ b,
                                                        const uint32_t *__restrict__ c,
                                                        unsigned long long *__restrict__ out) {
    unsigned long long sa = 0, sb = 0, sc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        sa += a[i];
        sb += b[i];
        sc += c[i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        sa += __shfl_down(sa, off);
        sb += __shfl_down(sb, off);
        sc += __shfl_down(sc, off);
    }
    __shared__ unsigned long long ws[kThreads / 64][3];
    if ((threadIdx.x & 63) == 0) {
        ws[threadIdx.x >> 6][0] = sa;
        ws[threadIdx.x >> 6][1] = sb;
        ws[threadIdx.x >> 6][2] = sc;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int w = 0; w < kThreads / 64; ++w) v += ws[w][threadIdx.x];
        atomicAdd(&out[threadIdx.x], v);
    }
}

// Per-block FP64 partial sums of (m v^2 / 2, m phi / 2).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_energy(int n, const T *__restrict__ v,
                                                     const T *__restrict__ m,
                                                     const T *__restrict__ phi,
                                                     double *__restrict__ part) {
    double ek = 0, ep = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double vx = v[3 * (int64_t)i], vy = v[3 * (int64_t)i + 1], vz = v[3 * (int64_t)i + 2];
        const double mi = m[i];
        ek += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
        ep += 0.5 * mi * (double)phi[i];
    }
    for (int o = 32; o > 0; o >>= 1) {
        ek += __shfl_xor(ek, o);
        ep += __shfl_xor(ep, o);
    }
    __shared__ double s[2][kThreads / 64];
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s[0][w] = ek;
        s[1][w] = ep;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int k = 0; k < kThreads / 64; ++k) {
            a += s[0][k];
            b += s[1][k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// One block of 256: fixed-order tree reduction of the partials.
__global__ __launch_bounds__(256) void k_energy_final(const double *__restrict__ part, int nb,
                                                      double *__restrict__ out) {
    __shared__ double s[2][256];
    double a = 0, b = 0;
    for (int k = threadIdx.x; k < nb; k += 256) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s[0][threadIdx.x] += s[0][threadIdx.x + o];
            s[1][threadIdx.x] += s[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s[0][0];
        out[1] = s[1][0];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_unpermute(int n, int comps,
                                                        const uint32_t *__restrict__ id,
                                                        const T *__restrict__ src,
                                                        T *__restrict__ dst) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t o = id[r];
    for (int c = 0; c < comps; ++c) dst[comps * o + c] = src[comps * (int64_t)r + c];
}

// Direct sum: thread per target, grid.y splits the sources; each block
// stages 256 sources at a time in LDS.  Arithmetic in R (FP64 for the reference sum,
// the simulation's dtype for the direct method); each tile's sums are added
// into FP64 accumulators, and the partial results per split are summed
// afterwards in split order.  targets == nullptr: target t is body t.
template <typename R> struct Src4;
template <> struct Src4<float> { using type = float4; };
template <> struct Src4<double> { using type = double4; };

__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

template <typename T, typename R>
__global__ __launch_bounds__(kThreads) void k_direct(int n, const T *__restrict__ pos,
                                                     const T *__restrict__ mass,
                                                     const int64_t *__restrict__ targets, int nt,
                                                     double e2, int chunk,
                                                     double *__restrict__ part) {
    using V4 = typename Src4<R>::type;
    __shared__ V4 src[kThreads];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ti = t < nt ? (targets ? targets[t] : t) : -1;
    const bool live = ti >= 0 && ti < n;  // out-of-range targets get NaN
    if (!live) ti = -1;
    R xi = 0, yi = 0, zi = 0;
    if (live) {
        xi = (R)pos[3 * ti];
        yi = (R)pos[3 * ti + 1];
        zi = (R)pos[3 * ti + 2];
    }
    const R re2 = (R)e2;
    double ax = 0, ay = 0, az = 0, ph = 0;
    const int j0 = blockIdx.y * chunk;
    const int j1 = min(n, j0 + chunk);
    for (int jb = j0; jb < j1; jb += kThreads) {
        const int j = jb + threadIdx.x;
        if (j < j1) {
            V4 v;
            v.x = (R)pos[3 * (int64_t)j];
            v.y = (R)pos[3 * (int64_t)j + 1];
            v.z = (R)pos[3 * (int64_t)j + 2];
            v.w = (R)mass[j];
            src[threadIdx.x] = v;
        }
        __syncthreads();
        const int cnt = min(kThreads, j1 - jb);
        const int self = (int)(ti - jb);  // tile slot of the target itself
        R tx = 0, ty = 0, tz = 0, tp = 0;
#pragma unroll 4
        for (int k = 0; k < cnt; ++k) {
            const V4 s = src[k];
            const R dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
            const R r2 = dx * dx + dy * dy + dz * dz + re2;
            const R inv = k == self ? (R)0 : inv_sqrt(r2);
            const R minv = s.w * inv;
            const R f = minv * (inv * inv);
            tx += f * dx;
            ty += f * dy;
            tz += f * dz;
            tp -= minv;
        }
        ax += (double)tx;
        ay += (double)ty;
        az += (double)tz;
        ph += (double)tp;
        __syncthreads();
    }
    if (t < nt) {
        double *p = part + 4 * ((int64_t)blockIdx.y * nt + t);
        const double bad = live ? 0.0 : __longlong_as_double(0x7ff8000000000000ll);
        p[0] = ax + bad;
        p[1] = ay + bad;
        p[2] = az + bad;
        p[3] = ph + bad;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_direct_sum(const double *__restrict__ part, int nt,
                                                         int nsplit, T *__restrict__ acc,
                                                         T *__restrict__ phi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double a[4] = {0, 0, 0, 0};
    for (int s = 0; s < nsplit; ++s)
        for (int c = 0; c < 4; ++c) a[c] += part[4 * ((int64_t)s * nt + t) + c];
    acc[3 * (int64_t)t] = (T)a[0];
    acc[3 * (int64_t)t + 1] = (T)a[1];
    acc[3 * (int64_t)t + 2] = (T)a[2];
    if (phi) phi[t] = (T)a[3];
}

// FP64 per-block partial sums of (m, m x, m v) for the standard units.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_moments7(int n, const T *__restrict__ x,
                                                       const T *__restrict__ v,
                                                       const T *__restrict__ m,
                                                       double *__restrict__ part) {
    double q[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double mi = m[i];
        q[0] += mi;
        for (int c = 0; c < 3; ++c) {
            q[1 + c] += mi * (double)x[3 * (int64_t)i + c];
            q[4 + c] += mi * (double)v[3 * (int64_t)i + c];
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < 7; ++c) q[c] += __shfl_xor(q[c], o);
    __shared__ double s[7][kThreads / 64];
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 7; ++c) s[c][w] = q[c];
    __syncthreads();
    if (threadIdx.x < 7) {
        double a = 0;
        for (int k = 0; k < kThreads / 64; ++k) a += s[threadIdx.x][k];
        part[7 * blockIdx.x + threadIdx.x] = a;
    }
}

// One block: fixed-order sums of nb partial rows of k values.
__global__ __launch_bounds__(64) void k_rows_final(const double *__restrict__ part, int nb, int k,
                                                   double *__restrict__ out) {
    if ((int)threadIdx.x >= k) return;
    double a = 0;
    for (int b = 0; b < nb; ++b) a += part[k * b + threadIdx.x];
    out[threadIdx.x] = a;
}

// m /= M; x -= com; v -= vcom (shift and mass scale in FP64, stored in T)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_shift(int n, T *__restrict__ x, T *__restrict__ v,
                                                    T *__restrict__ m, double minv, double cx,
                                                    double cy, double cz, double ux, double uy,
                                                    double uz) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        m[i] = (T)((double)m[i] * minv);
        x[3 * (int64_t)i] = (T)((double)x[3 * (int64_t)i] - cx);
        x[3 * (int64_t)i + 1] = (T)((double)x[3 * (int64_t)i + 1] - cy);
        x[3 * (int64_t)i + 2] = (T)((double)x[3 * (int64_t)i + 2] - cz);
        v[3 * (int64_t)i] = (T)((double)v[3 * (int64_t)i] - ux);
        v[3 * (int64_t)i + 1] = (T)((double)v[3 * (int64_t)i + 1] - uy);
        v[3 * (int64_t)i + 2] = (T)((double)v[3 * (int64_t)i + 2] - uz);
    }
}

// Per-block FP64 partial sums of (m v^2 / 2, m phi / 2) with FP64 phi.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_energy64(int n, const T *__restrict__ v,
                                                       const T *__restrict__ m,
                                                       const double *__restrict__ phi,
                                                       double *__restrict__ part) {
    double q[2] = {0, 0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double vx = v[3 * (int64_t)i], vy = v[3 * (int64_t)i + 1], vz = v[3 * (int64_t)i + 2];
        const double mi = m[i];
        q[0] += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
        q[1] += 0.5 * mi * phi[i];
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < 2; ++c) q[c] += __shfl_xor(q[c], o);
    __shared__ double s[2][kThreads / 64];
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 2; ++c) s[c][w] = q[c];
    __syncthreads();
    if (threadIdx.x < 2) {
        double a = 0;
        for (int k = 0; k < kThreads / 64; ++k) a += s[threadIdx.x][k];
        part[2 * blockIdx.x + threadIdx.x] = a;
    }
}

// x *= a; v *= b (in FP64, stored in T)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale(int64_t n3, T *__restrict__ x,
                                                    T *__restrict__ v, double a, double b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = (T)((double)x[i] * a);
        v[i] = (T)((double)v[i] * b);
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + kThreads - 1) / kThreads;
    return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

int launch_count_sum(hipStream_t s, int64_t n, const uint32_t *a, const uint32_t *b,
                     const uint32_t *c, unsigned long long *out) {
    k_count_sum<<<std::min(grid_for(n), 1024), kThreads, 0, s>>>(n, a, b, c, out);
    return check_launch("count_sum");
}

int launch_kick(hipStream_t s, int dtype, int64_t n, void *vel, const void *acc, double h) {
    if (dtype == BH_F32)
        k_kick<float><<<grid_for(3 * n / 4 + 1), kThreads, 0, s>>>(3 * n, (float *)vel, (const float *)acc, (float)h);
    else
        k_kick<double><<<grid_for(3 * n / 2 + 1), kThreads, 0, s>>>(3 * n, (double *)vel, (const double *)acc, h);
    return check_launch("kick");
}

int launch_kick_drift(hipStream_t s, int dtype, int64_t n, void *pos, void *vel,
                      const void *acc, double h, double dt) {
    if (dtype == BH_F32)
        k_kick_drift<float><<<grid_for(3 * n / 4 + 1), kThreads, 0, s>>>(
            3 * n, (float *)pos, (float *)vel, (const float *)acc, (float)h, (float)dt);
    else
        k_kick_drift<double><<<grid_for(3 * n / 2 + 1), kThreads, 0, s>>>(
            3 * n, (double *)pos, (double *)vel, (const double *)acc, h, dt);
    return check_launch("kick_drift");
}

int launch_energy(hipStream_t s, int dtype, int64_t n, const void *vel, const void *mass,
                  const void *phi, double *red, double *out2) {
    const int nb = 1024;
    if (dtype == BH_F32)
        k_energy<float><<<nb, kThreads, 0, s>>>((int)n, (const float *)vel, (const float *)mass,
                                                (const float *)phi, red);
    else
        k_energy<double><<<nb, kThreads, 0, s>>>((int)n, (const double *)vel,
                                                 (const double *)mass, (const double *)phi, red);
    k_energy_final<<<1, 256, 0, s>>>(red, nb, out2);
    return check_launch("energy");
}

int launch_unpermute(hipStream_t s, int dtype, int64_t n, const uint32_t *id, const void *src,
                     void *dst) {
    if (dtype == BH_F32)
        k_unpermute<float><<<div_up(n, kThreads), kThreads, 0, s>>>((int)n, 3, id,
                                                                   (const float *)src, (float *)dst);
    else
        k_unpermute<double><<<div_up(n, kThreads), kThreads, 0, s>>>(
            (int)n, 3, id, (const double *)src, (double *)dst);
    return check_launch("unpermute");
}

namespace {
// Sources split so that about 2048 blocks are in flight: the number of
// splits and the source chunk per split for n sources and nt targets.
struct DirectSplit {
    int bx, nsplit, chunk;
};

DirectSplit direct_split(int64_t n, int64_t nt) {
    DirectSplit d;
    d.bx = div_up(nt, kThreads);
    d.nsplit = 2048 / d.bx;
    if (d.nsplit < 1) d.nsplit = 1;
    if (d.nsplit > 256) d.nsplit = 256;
    d.chunk = div_up(n, d.nsplit);
    d.chunk = div_up(d.chunk, kThreads) * kThreads;
    d.nsplit = div_up(n, d.chunk);
    return d;
}

// part: 32 * nsplit * nt bytes of device memory (4 doubles per split and target)
template <typename T, typename R, typename O>
int direct_launch(hipStream_t s, const DirectSplit &d, int64_t n, const T *pos, const T *mass,
                  const int64_t *targets, int64_t nt, double eps, O *acc, O *phi, double *part) {
    dim3 grid(d.bx, d.nsplit);
    k_direct<T, R><<<grid, kThreads, 0, s>>>((int)n, pos, mass, targets, (int)nt, eps * eps,
                                             d.chunk, part);
    k_direct_sum<O><<<d.bx, kThreads, 0, s>>>(part, (int)nt, d.nsplit, acc, phi);
    return check_launch("direct");
}

template <typename T, typename R, typename O>
int direct_splits(hipStream_t s, int64_t n, const T *pos, const T *mass,
                  const int64_t *targets, int64_t nt, double eps, O *acc, O *phi,
                  DevBuf &scratch) {
    const DirectSplit d = direct_split(n, nt);
    int rc = grow(scratch, 32ull * d.nsplit * nt);
    if (rc) return rc;
    return direct_launch<T, R, O>(s, d, n, pos, mass, targets, nt, eps, acc, phi,
                                  (double *)scratch.p);
}

// Partial sums of the direct sum for callers that cannot allocate: a fixed
// array in each GPU's global memory, held until the process ends.  Host
// code never uses the array's name as an address: its device address is
// taken once per device (static_scratch_init) and kept in g_static_part.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticScratchBytes / 8];
double *g_static_part[kMaxDevices] = {};
}  // namespace

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(BH_E_DEVICE, "device index beyond the static scratch table");
    if (g_static_part[device]) return BH_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        hipGetLastError();
        return set_error(BH_E_DEVICE, "hipGetSymbolAddress of the static scratch failed");
    }
    g_static_part[device] = (double *)p;
    return BH_OK;
}

int64_t direct_static_max_targets() {
    // direct_split keeps nsplit * nt <= 2048 * kThreads while one split
    // suffices; beyond that one split of 32 bytes per target
    return (int64_t)(kStaticScratchBytes / 32);
}

int launch_direct_static(hipStream_t s, int device, int dtype, int64_t n, const void *pos,
                         const void *mass, const int64_t *targets, int64_t nt, double eps,
                         double *acc, double *phi) {
    if (device < 0 || device >= kMaxDevices || !g_static_part[device])
        return set_error(BH_E_STATE, "static scratch not set up on this device");
    const DirectSplit d = direct_split(n, nt);
    if (32ull * d.nsplit * nt > kStaticScratchBytes)
        return set_error(BH_E_INVALID, "nt too large for the static scratch");
    double *part = g_static_part[device];
    if (dtype == BH_F32)
        return direct_launch<float, double, double>(s, d, n, (const float *)pos,
                                                    (const float *)mass, targets, nt, eps, acc,
                                                    phi, part);
    return direct_launch<double, double, double>(s, d, n, (const double *)pos,
                                                 (const double *)mass, targets, nt, eps, acc,
                                                 phi, part);
}

int launch_direct(hipStream_t s, int dtype, int64_t n, const void *pos, const void *mass,
                  const int64_t *targets, int64_t nt, double eps, double *acc, double *phi,
                  DevBuf &scratch) {
    if (dtype == BH_F32)
        return direct_splits<float, double, double>(s, n, (const float *)pos, (const float *)mass,
                                                    targets, nt, eps, acc, phi, scratch);
    return direct_splits<double, double, double>(s, n, (const double *)pos, (const double *)mass,
                                                 targets, nt, eps, acc, phi, scratch);
}

int launch_direct_all(hipStream_t s, int dtype, int64_t n, const void *pos, const void *mass,
                      double eps, void *acc, void *phi, DevBuf &scratch) {
    if (dtype == BH_F32)
        return direct_splits<float, float, float>(s, n, (const float *)pos, (const float *)mass,
                                                  nullptr, n, eps, (float *)acc, (float *)phi,
                                                  scratch);
    return direct_splits<double, double, double>(s, n, (const double *)pos, (const double *)mass,
                                                 nullptr, n, eps, (double *)acc, (double *)phi,
                                                 scratch);
}

namespace {
template <typename T>
int standard_units_t(hipStream_t s, int64_t n, T *pos, T *vel, T *mass, DevBuf &scratch,
                     DevBuf &work, double *host) {
    const int nb = 256;
    // work: direct-sum acc (3 n) and phi (n), then the partial rows
    int rc = grow(work, 8ull * (4 * n + 7 * nb + 8));
    if (rc) return rc;
    double *wacc = (double *)work.p, *wphi = wacc + 3 * n, *part = wphi + n;
    double *tot = part + 7 * nb;
    auto fetch = [&](int k) -> int {
        if (hipMemcpyAsync(host, tot, 8 * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(BH_E_DEVICE, "standard units: reduction copy failed");
        for (int c = 0; c < k; ++c)
            if (!std::isfinite(host[c]))
                return set_error(BH_E_NONFINITE, "standard units: non-finite input");
        return BH_OK;
    };
    // 1. total mass 1 and the centre-of-mass frame
    k_moments7<T><<<nb, kThreads, 0, s>>>((int)n, pos, vel, mass, part);
    k_rows_final<<<1, 64, 0, s>>>(part, nb, 7, tot);
    if ((rc = fetch(7))) return rc;
    const double M = host[0];
    if (!(M > 0)) return set_error(BH_E_INVALID, "standard units: total mass must be > 0");
    k_shift<T><<<std::min(div_up(n, kThreads), 4096), kThreads, 0, s>>>(
        (int)n, pos, vel, mass, 1.0 / M, host[1] / M, host[2] / M, host[3] / M, host[4] / M,
        host[5] / M, host[6] / M);
    // 2. kinetic and (unsoftened) potential energy
    if ((rc = direct_splits<T, double, double>(s, n, pos, mass, nullptr, n, 0.0, wacc, wphi,
                                               scratch)))
        return rc;
    k_energy64<T><<<nb, kThreads, 0, s>>>((int)n, vel, mass, wphi, part);
    k_rows_final<<<1, 64, 0, s>>>(part, nb, 2, tot);
    if ((rc = fetch(2))) return rc;
    const double ek = host[0], ep = host[1];
    if (!(ek > 0)) return set_error(BH_E_INVALID, "standard units: kinetic energy must be > 0");
    if (!(ep < 0)) return set_error(BH_E_INVALID, "standard units: potential energy must be < 0");
    // 3. velocities to virial ratio 1/2: E_kin = -E_pot / 2, so E = E_pot / 2
    const double qv = std::sqrt(-0.5 * ep / ek);
    // 4. lengths x b, velocities x 1/sqrt(b): E -> E / b = -1/4 for b = -2 E_pot
    const double b = -2.0 * ep;
    k_scale<T><<<std::min(div_up(3 * n, kThreads), 4096), kThreads, 0, s>>>(
        3 * n, pos, vel, b, qv / std::sqrt(b));
    if ((rc = check_launch("standard units"))) return rc;
    host[0] = ek;
    host[1] = ep;
    host[2] = M;
    return BH_OK;
}
}  // namespace

int standard_units(hipStream_t s, int dtype, int64_t n, void *pos, void *vel, void *mass,
                   DevBuf &scratch, DevBuf &work, double *host) {
    if (dtype == BH_F32)
        return standard_units_t<float>(s, n, (float *)pos, (float *)vel, (float *)mass, scratch,
                                       work, host);
    return standard_units_t<double>(s, n, (double *)pos, (double *)vel, (double *)mass, scratch,
                                    work, host);
}

}  // namespace bh
