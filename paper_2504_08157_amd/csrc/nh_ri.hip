// gfx950 kernels of the RI-velocity diagnostic (paper, section on the RI
// velocity): the speed-weighted centre of each level, the mean tangential
// speed over open annuli (strips) around it, and the maximum of those means
// over strips and levels, with the maximum horizontal speed alongside.
//
// Every level is cut into nb contiguous chunks of lattice columns, one
// workgroup per (chunk, level): a reduction pass for the centre, then a
// histogram pass (strip sums and counts in LDS) for the means.  Partial
// results per workgroup are combined in a fixed order by small final
// kernels; only the LDS histogram additions are unordered.  (Summing the
// lanes of one strip across the wavefront before each LDS update was 2.8x
// slower than one LDS atomic per node: neighbouring lanes span about a dozen
// strips at the benchmark's resolution.)
#include "nh_internal.h"

namespace nh {

constexpr int kRiThreads = 256;

__device__ __forceinline__ double ri_block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int h = kRiThreads / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// s0 = sum m |u|, s1 = sum m |u| x, s2 = sum m |u| y over chunk b of level k
// (m = m_x m_y, the level's 2D quadrature weight up to the level's factor)
__global__ void __launch_bounds__(kRiThreads) ri_centroid_partial(RiParams p, const double *__restrict__ q,
                                                                   double *__restrict__ part)
{
    __shared__ double red[kRiThreads];
    const int b = blockIdx.x, k = blockIdx.y;
    const long nxy = (long)p.nx * p.ny;
    const long chunk = (nxy + p.nb - 1) / p.nb;
    const long i0 = b * chunk, i1 = i0 + chunk < nxy ? i0 + chunk : nxy;
    const double *u = q + p.U + k * nxy, *v = q + 2 * p.U + k * nxy, *w = q + 3 * p.U + k * nxy;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long i = i0 + threadIdx.x; i < i1; i += kRiThreads) {
        const int ix = (int)(i % p.nx), iy = (int)(i / p.nx);
        const double sp = sqrt(u[i] * u[i] + v[i] * v[i] + w[i] * w[i]) * (p.mx[ix] * p.my[iy]);
        s0 += sp;
        s1 += sp * p.x[ix];
        s2 += sp * p.y[iy];
    }
    s0 = ri_block_sum(s0, red);
    s1 = ri_block_sum(s1, red);
    s2 = ri_block_sum(s2, red);
    if (threadIdx.x == 0) {
        double *o = part + ((long)k * p.nb + b) * 3;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

// centre of level k = blockIdx.x from its nb partials (a level at rest: the
// domain midpoint)
__global__ void __launch_bounds__(kRiThreads) ri_centroid_final(RiParams p, const double *__restrict__ part,
                                                                 double *__restrict__ center)
{
    __shared__ double red[kRiThreads];
    const int k = blockIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < p.nb; b += kRiThreads)
        for (int c = 0; c < 3; ++c) s[c] += part[((long)k * p.nb + b) * 3 + c];
    for (int c = 0; c < 3; ++c) s[c] = ri_block_sum(s[c], red);
    if (threadIdx.x == 0) {
        center[k] = s[0] > 0.0 ? s[1] / s[0] : p.xmid;
        center[p.nz + k] = s[0] > 0.0 ? s[2] / s[0] : p.ymid;
    }
}

// Strip of squared radius r2: the j with (j eps)^2 < r2 < ((j+1) eps)^2,
// edges and r2 rounded exactly as written (no fused multiply-add), or -1.
__device__ __forceinline__ double ri_edge2(int j, double eps)
{
    const double b = __dmul_rn((double)j, eps);
    return __dmul_rn(b, b);
}

__device__ __forceinline__ int ri_strip(double r2, double eps, int ns)
{
    if (!(r2 > 0.0) || !(r2 < ri_edge2(ns, eps))) return -1;
    double g = sqrt(r2) / eps;
    int j = g < (double)ns ? (int)g : ns - 1;
    if (j > ns - 1) j = ns - 1;
    while (j > 0 && !(ri_edge2(j, eps) < r2)) --j;
    while (j < ns - 1 && !(r2 < ri_edge2(j + 1, eps))) ++j;
    return (ri_edge2(j, eps) < r2 && r2 < ri_edge2(j + 1, eps)) ? j : -1;
}

// strip sums and counts of chunk b of level k, and its maximum horizontal speed
__global__ void __launch_bounds__(kRiThreads) ri_strip_partial(RiParams p, const double *__restrict__ q,
                                                                const double *__restrict__ center,
                                                                double *__restrict__ ssum, int *__restrict__ scnt,
                                                                double *__restrict__ umax)
{
    extern __shared__ double hist[];                 // [ns] sums, then [ns] counts
    __shared__ double red[kRiThreads];
    int *hcnt = reinterpret_cast<int *>(hist + p.nstrips);
    const int b = blockIdx.x, k = blockIdx.y, ns = p.nstrips;
    for (int j = threadIdx.x; j < ns; j += kRiThreads) {
        hist[j] = 0.0;
        hcnt[j] = 0;
    }
    __syncthreads();
    const long nxy = (long)p.nx * p.ny;
    const long chunk = (nxy + p.nb - 1) / p.nb;
    const long i0 = b * chunk, i1 = i0 + chunk < nxy ? i0 + chunk : nxy;
    const double *u = q + p.U + k * nxy, *v = q + 2 * p.U + k * nxy;
    const double xc = center[k], yc = center[p.nz + k];
    double um = 0.0;
    for (long i = i0 + threadIdx.x; i < i1; i += kRiThreads) {
        const int ix = (int)(i % p.nx), iy = (int)(i / p.nx);
        const double ui = u[i], vi = v[i];
        um = fmax(um, sqrt(ui * ui + vi * vi));
        const double dx = __dsub_rn(p.x[ix], xc), dy = __dsub_rn(p.y[iy], yc);
        const double r2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
        const int j = ri_strip(r2, p.eps, ns);
        if (j >= 0) {
            // |u_h . e_theta|: the horizontal velocity less its radial part
            atomicAdd(&hist[j], fabs(vi * dx - ui * dy) / sqrt(r2));
            atomicAdd(&hcnt[j], 1);
        }
    }
    // block maximum of the horizontal speed
    red[threadIdx.x] = um;
    __syncthreads();
    for (int h = kRiThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const long base = ((long)k * p.nb + b) * ns;
    for (int j = threadIdx.x; j < ns; j += kRiThreads) {
        ssum[base + j] = hist[j];
        scnt[base + j] = hcnt[j];
    }
    if (threadIdx.x == 0) umax[(long)k * p.nb + b] = red[0];
}

// strip means of level k = blockIdx.x from its nb partials
__global__ void __launch_bounds__(kRiThreads) ri_strip_final(RiParams p, const double *__restrict__ ssum,
                                                              const int *__restrict__ scnt, double *__restrict__ ubar,
                                                              int *__restrict__ count)
{
    const int k = blockIdx.x, ns = p.nstrips;
    for (int j = threadIdx.x; j < ns; j += kRiThreads) {
        double s = 0.0;
        int c = 0;
        for (int b = 0; b < p.nb; ++b) {
            s += ssum[((long)k * p.nb + b) * ns + j];
            c += scnt[((long)k * p.nb + b) * ns + j];
        }
        ubar[(long)k * ns + j] = c > 0 ? s / c : 0.0;
        count[(long)k * ns + j] = c;
    }
}

// result = {u_RI, radius of its strip centre, height of its level, max
// horizontal speed}; the largest mean of a populated strip, the first in
// (level, strip) order on ties; {0, -1, -1, .} when no strip is populated
__global__ void __launch_bounds__(kRiThreads) ri_max_final(RiParams p, const double *__restrict__ ubar,
                                                            const int *__restrict__ count,
                                                            const double *__restrict__ umax,
                                                            const double *__restrict__ z, double *__restrict__ result)
{
    __shared__ double rv[kRiThreads];
    __shared__ long ri[kRiThreads];
    __shared__ double red[kRiThreads];
    const long n = (long)p.nz * p.nstrips;
    double best = -1.0;
    long at = -1;
    for (long i = threadIdx.x; i < n; i += kRiThreads)
        if (count[i] > 0 && ubar[i] > best) {   // strided ascending: the first of equals stays
            best = ubar[i];
            at = i;
        }
    double um = 0.0;
    for (long i = threadIdx.x; i < (long)p.nz * p.nb; i += kRiThreads) um = fmax(um, umax[i]);
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = at;
    red[threadIdx.x] = um;
    __syncthreads();
    for (int h = kRiThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int o = threadIdx.x + h;
            const bool take = ri[o] >= 0 && (ri[threadIdx.x] < 0 || rv[o] > rv[threadIdx.x] ||
                                             (rv[o] == rv[threadIdx.x] && ri[o] < ri[threadIdx.x]));
            if (take) {
                rv[threadIdx.x] = rv[o];
                ri[threadIdx.x] = ri[o];
            }
            red[threadIdx.x] = fmax(red[threadIdx.x], red[o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long a = ri[0];
        result[0] = a >= 0 ? rv[0] : 0.0;
        result[1] = a >= 0 ? ((double)(a % p.nstrips) + 0.5) * p.eps : -1.0;
        result[2] = a >= 0 ? z[a / p.nstrips] : -1.0;
        result[3] = red[0];
    }
}

size_t ri_lds_bytes(int nstrips) { return (size_t)nstrips * (sizeof(double) + sizeof(int)); }

hipError_t launch_ri(const RiParams &p, const double *q, bool center_given, double *center, double *ubar,
                     int *count, double *result, const double *z, const RiWork &w, hipStream_t s)
{
    const dim3 grid(p.nb, p.nz), blk(kRiThreads);
    if (!center_given) {
        hipLaunchKernelGGL(ri_centroid_partial, grid, blk, 0, s, p, q, w.cpart);
        hipLaunchKernelGGL(ri_centroid_final, dim3(p.nz), blk, 0, s, p, w.cpart, center);
    }
    hipLaunchKernelGGL(ri_strip_partial, grid, blk, ri_lds_bytes(p.nstrips), s, p, q, (const double *)center,
                       w.ssum, w.scnt, w.umax);
    hipLaunchKernelGGL(ri_strip_final, dim3(p.nz), blk, 0, s, p, w.ssum, w.scnt, ubar, count);
    hipLaunchKernelGGL(ri_max_final, dim3(1), blk, 0, s, p, ubar, count, w.umax, z, result);
    return hipGetLastError();
}

}  // namespace nh
