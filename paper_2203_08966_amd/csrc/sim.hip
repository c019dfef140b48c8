// Integration, energy and direct summation on gfx950.
//
//  kick / drift   KDK leapfrog with a fixed step (Sec. 2.3)
//  energy         E_kin = sum m v^2 / 2, E_pot = sum m phi / 2 (Sec. 2.4, each
//                 pair once), FP64 accumulation in a fixed order
//  direct         FP64 O(N * targets) direct sum (Sec. 2.1), the judge of the
//                 tree walk's error; sources staged through LDS
#include "bh_internal.h"

namespace bh {
namespace {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kick(int64_t n3, T *__restrict__ v,
                                                   const T *__restrict__ a, T h) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] += a[i] * h;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kick_drift(int64_t n3, T *__restrict__ x,
                                                         T *__restrict__ v,
                                                         const T *__restrict__ a, T h, T dt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T vi = v[i] + a[i] * h;
        v[i] = vi;
        x[i] += vi * dt;
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

// Direct sum, FP64: thread per target, grid.y splits the sources; each
// block stages 256 sources at a time in LDS.  Partial results per split are
// summed afterwards in split order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_direct(int n, const T *__restrict__ pos,
                                                     const T *__restrict__ mass,
                                                     const int64_t *__restrict__ targets, int nt,
                                                     double e2, int chunk,
                                                     double *__restrict__ part) {
    __shared__ double4 src[kThreads];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ti = t < nt ? targets[t] : -1;
    const bool live = ti >= 0 && ti < n;  // out-of-range targets get NaN
    if (!live) ti = -1;
    double xi = 0, yi = 0, zi = 0;
    if (live) {
        xi = pos[3 * ti];
        yi = pos[3 * ti + 1];
        zi = pos[3 * ti + 2];
    }
    double ax = 0, ay = 0, az = 0, ph = 0;
    const int j0 = blockIdx.y * chunk;
    const int j1 = min(n, j0 + chunk);
    for (int jb = j0; jb < j1; jb += kThreads) {
        const int j = jb + threadIdx.x;
        if (j < j1) src[threadIdx.x] = make_double4(pos[3 * (int64_t)j], pos[3 * (int64_t)j + 1],
                                                    pos[3 * (int64_t)j + 2], mass[j]);
        __syncthreads();
        const int cnt = min(kThreads, j1 - jb);
        for (int k = 0; k < cnt; ++k) {
            const double4 s = src[k];
            if (jb + k == ti) continue;
            const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
            const double r2 = dx * dx + dy * dy + dz * dz + e2;
            const double r = sqrt(r2);
            const double f = s.w / (r2 * r);
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
            ph -= s.w / r;
        }
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

__global__ __launch_bounds__(kThreads) void k_direct_sum(const double *__restrict__ part, int nt,
                                                         int nsplit, double *__restrict__ acc,
                                                         double *__restrict__ phi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double a[4] = {0, 0, 0, 0};
    for (int s = 0; s < nsplit; ++s)
        for (int c = 0; c < 4; ++c) a[c] += part[4 * ((int64_t)s * nt + t) + c];
    acc[3 * (int64_t)t] = a[0];
    acc[3 * (int64_t)t + 1] = a[1];
    acc[3 * (int64_t)t + 2] = a[2];
    if (phi) phi[t] = a[3];
}

int grid_for(int64_t n) {
    int64_t g = (n + kThreads - 1) / kThreads;
    return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

int launch_kick(hipStream_t s, int dtype, int64_t n, void *vel, const void *acc, double h) {
    if (dtype == BH_F32)
        k_kick<float><<<grid_for(3 * n), kThreads, 0, s>>>(3 * n, (float *)vel, (const float *)acc, (float)h);
    else
        k_kick<double><<<grid_for(3 * n), kThreads, 0, s>>>(3 * n, (double *)vel, (const double *)acc, h);
    return check_launch("kick");
}

int launch_kick_drift(hipStream_t s, int dtype, int64_t n, void *pos, void *vel,
                      const void *acc, double h, double dt) {
    if (dtype == BH_F32)
        k_kick_drift<float><<<grid_for(3 * n), kThreads, 0, s>>>(
            3 * n, (float *)pos, (float *)vel, (const float *)acc, (float)h, (float)dt);
    else
        k_kick_drift<double><<<grid_for(3 * n), kThreads, 0, s>>>(
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

int launch_direct(hipStream_t s, int dtype, int64_t n, const void *pos, const void *mass,
                  const int64_t *targets, int64_t nt, double eps, double *acc, double *phi,
                  DevBuf &scratch) {
    const int bx = div_up(nt, kThreads);
    int nsplit = 2048 / bx;
    if (nsplit < 1) nsplit = 1;
    if (nsplit > 256) nsplit = 256;
    int chunk = div_up(n, nsplit);
    chunk = div_up(chunk, kThreads) * kThreads;
    nsplit = div_up(n, chunk);
    int rc = grow(scratch, 32ull * nsplit * nt);
    if (rc) return rc;
    dim3 grid(bx, nsplit);
    if (dtype == BH_F32)
        k_direct<float><<<grid, kThreads, 0, s>>>((int)n, (const float *)pos, (const float *)mass,
                                                  targets, (int)nt, eps * eps, chunk,
                                                  (double *)scratch.p);
    else
        k_direct<double><<<grid, kThreads, 0, s>>>((int)n, (const double *)pos,
                                                   (const double *)mass, targets, (int)nt,
                                                   eps * eps, chunk, (double *)scratch.p);
    k_direct_sum<<<bx, kThreads, 0, s>>>((const double *)scratch.p, (int)nt, nsplit, acc, phi);
    return check_launch("direct");
}

}  // namespace bh
