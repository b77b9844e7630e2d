// gfx950 kernels and the host-driven Krylov loop of the 3D-IMEX split
// (paper, Sec. 2.3: IMEX with the linear fast-wave operator treated
// implicitly, ARK2, matrix-free GMRES).  Here the linear operator is taken
// over all three directions:
//   (L)_rho'   = - rho0 (d/dx u + d/dy v) - d/dz (rho0 w)
//   (L)_u      = - (1/rho0) dp'_L/dx,   (L)_v = - (1/rho0) dp'_L/dy
//   (L)_w      = - (1/rho0) dp'_L/dz - g rho'/rho0 - tau(z) w
//   (L)_theta' = - w dtheta0/dz,        p'_L = gamma p0 (rho'/rho0 + theta'/theta0),
// the vertical terms from the column-walking L_v kernel, the horizontal ones
// from the DSS'd x/y derivative stencils of the explicit path, the damping
// of w in the absorbing layer implicit (the Klemp form of an upper sponge).
// Each stage system (I - a L) x = b is one global system in 5U unknowns,
// solved by restarted GMRES with classical Gram-Schmidt (a second pass when
// the kept norm falls below 1e-2 of the vector's), its dot products reduced
// in a fixed order on the device and its small Hessenberg problem on the
// host; optionally right-preconditioned by the column systems of the 1D
// split (flexible GMRES, since those are solved iteratively).
#include "nh_internal.h"

#include <cmath>
#include <vector>

namespace nh {

// out[f] = a x[f] + c (lv[f] + horizontal and damping terms of L x) at every
// node; lv holds L_v x (u, v rows zero).  Walls: u rows zero at x walls, v
// rows at y walls, w rows at the bottom and top.  lv may alias out.
__global__ void __launch_bounds__(256) l3_combine_kernel(L3Params h, const double *__restrict__ x, const double *lv,
                                                         double *out, double a, double c)
{
    const long nxy = (long)h.nx * h.ny, U = nxy * h.nz;
    const int NC = 2 * h.N + 1;
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < U; I += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(I % h.nx), iy = (int)((I / h.nx) % h.ny), iz = (int)(I / nxy);
        const double *Lv = h.lev + (long)iz * kLevW;
        const double rho0 = Lv[0], p0 = Lv[2], tau = Lv[4], irho0 = Lv[7], ith0 = Lv[8];
        const double gp = h.gamma * p0;
        double dux = 0.0, dpx = 0.0, dvy = 0.0, dpy = 0.0;
        for (int o = 0; o < NC; ++o) {
            const double cf = h.gx[(long)ix * NC + o];
            if (cf == 0.0) continue;
            int j = ix + o - h.N;
            if (j < 0 || j >= h.nx) {
                if (!h.perx) continue;
                j += j < 0 ? h.nx : -h.nx;
            }
            const long J = I + (j - ix);
            dux += cf * x[U + J];
            dpx += cf * (gp * (x[J] * irho0 + x[4 * U + J] * ith0));
        }
        for (int o = 0; o < NC; ++o) {
            const double cf = h.gy[(long)iy * NC + o];
            if (cf == 0.0) continue;
            int j = iy + o - h.N;
            if (j < 0 || j >= h.ny) {
                if (!h.pery) continue;
                j += j < 0 ? h.ny : -h.ny;
            }
            const long J = I + (long)(j - iy) * h.nx;
            dvy += cf * x[2 * U + J];
            dpy += cf * (gp * (x[J] * irho0 + x[4 * U + J] * ith0));
        }
        double Lr = lv[I] - rho0 * (dux + dvy);
        double Lu = -irho0 * dpx, Lvv = -irho0 * dpy;
        double Lw = lv[3 * U + I] - tau * x[3 * U + I];
        const double Lt = lv[4 * U + I];
        if (!h.perx && (ix == 0 || ix == h.nx - 1)) Lu = 0.0;
        if (!h.pery && (iy == 0 || iy == h.ny - 1)) Lvv = 0.0;
        if (iz == 0 || iz == h.nz - 1) Lw = 0.0;
        out[I] = a * x[I] + c * Lr;
        out[U + I] = a * x[U + I] + c * Lu;
        out[2 * U + I] = a * x[2 * U + I] + c * Lvv;
        out[3 * U + I] = a * x[3 * U + I] + c * Lw;
        out[4 * U + I] = a * x[4 * U + I] + c * Lt;
    }
}

hipError_t launch_l3(const L3Params &h, const double *x, double *out, double a, double c, hipStream_t s)
{
    hipError_t e = launch_lv_apply(h.hv, x, out, s, true);
    if (e != hipSuccess) return e;
    const long U = (long)h.nx * h.ny * h.nz;
    long blocks = (U + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(l3_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, h, x, (const double *)out, out,
                       a, c);
    return hipGetLastError();
}

// ---- Krylov kernels on n-vectors.  Partial sums per block, then one block
// sums the partials of each quantity in block order: the same result on
// every call.
constexpr int kKryBlocks = 1024, kKryThreads = 256, kKryMaxV = 34;

__device__ __forceinline__ double kry_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// part[b][j] = sum over block b's elements of V_j . w (j < nv), and
// part[b][nv] = w . w
__global__ void __launch_bounds__(kKryThreads) kry_dots_kernel(const double *__restrict__ V, long stride, int nv,
                                                               const double *__restrict__ w, long n,
                                                               double *__restrict__ part)
{
    __shared__ double red[kKryThreads / 64][kKryMaxV + 1];
    double acc[kKryMaxV + 1];
#pragma unroll
    for (int j = 0; j <= kKryMaxV; ++j) acc[j] = 0.0;
    for (long i = blockIdx.x * (long)kKryThreads + threadIdx.x; i < n; i += (long)gridDim.x * kKryThreads) {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < kKryMaxV; ++j)
            if (j < nv) acc[j] += V[j * stride + i] * wi;
        acc[kKryMaxV] += wi * wi;
    }
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int j = 0; j <= kKryMaxV; ++j) {
        if (j < nv || j == kKryMaxV) {
            const double s = kry_wave_sum(acc[j]);
            if (lane == 0) red[wv][j] = s;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= nv; j += kKryThreads) {
        const int jj = j < nv ? j : kKryMaxV;
        double s = 0.0;
        for (int q = 0; q < kKryThreads / 64; ++q) s += red[q][jj];
        part[(long)blockIdx.x * (kKryMaxV + 1) + j] = s;
    }
}

// out[j] = sum over blocks of part[b][j]: workgroup j sums quantity j, each
// thread a fixed strided subset of the blocks, then a fixed tree
__global__ void __launch_bounds__(kKryThreads) kry_final_kernel(const double *__restrict__ part, int nb,
                                                                double *__restrict__ out)
{
    __shared__ double red[kKryThreads];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kKryThreads) s += part[(long)b * (kKryMaxV + 1) + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kKryThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

struct KryCoef {
    double c[kKryMaxV];
};

// y = s (w - sum_j c_j V_j) (j < nv); with norm != 0 also part[b][0] =
// block sums of the result squared (before the scale s)
__global__ void __launch_bounds__(kKryThreads) kry_axpy_kernel(const double *__restrict__ V, long stride, int nv,
                                                               KryCoef cf, const double *w, double *y, long n,
                                                               double s, int norm, double *__restrict__ part)
{
    __shared__ double red[kKryThreads / 64];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)kKryThreads + threadIdx.x; i < n; i += (long)gridDim.x * kKryThreads) {
        double v = w[i];
#pragma unroll 4
        for (int j = 0; j < nv; ++j) v -= cf.c[j] * V[j * stride + i];
        acc += v * v;
        y[i] = s * v;
    }
    if (!norm) return;
    const double t = kry_wave_sum(acc);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int q = 0; q < kKryThreads / 64; ++q) r += red[q];
        part[(long)blockIdx.x * (kKryMaxV + 1)] = r;
    }
}

namespace {

struct Kry {
    const L3Params &h;
    const G3Work &w;
    hipStream_t s;
    long n;

    // host copies of nv + 1 reduced quantities
    hipError_t fetch(int nv, double *host)
    {
        hipLaunchKernelGGL(kry_final_kernel, dim3(nv + 1), dim3(kKryThreads), 0, s, w.part, kKryBlocks, w.red);
        hipError_t e = hipMemcpyAsync(host, w.red, sizeof(double) * (nv + 1), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    }
    hipError_t dots(const double *V, int nv, const double *x, double *host)
    {
        hipLaunchKernelGGL(kry_dots_kernel, dim3(kKryBlocks), dim3(kKryThreads), 0, s, V, n, nv, x, n, w.part);
        return fetch(nv, host);
    }
    // y = sc (x - sum c_j V_j); returns ||x - sum c_j V_j||^2 when norm
    hipError_t axpy(const double *V, int nv, const double *c, const double *x, double *y, double sc, bool norm,
                    double *n2)
    {
        KryCoef k{};
        for (int j = 0; j < nv; ++j) k.c[j] = c[j];
        hipLaunchKernelGGL(kry_axpy_kernel, dim3(kKryBlocks), dim3(kKryThreads), 0, s, V, n, nv, k, x, y, n, sc,
                           norm ? 1 : 0, w.part);
        if (!norm) return hipGetLastError();
        double h2[2];
        hipError_t e = fetch(0, h2);
        *n2 = h2[0];
        return e;
    }
};

}  // namespace

// z = (I - alpha L_v)^-1 v column by column (column GMRES(10) to rtol 1e-6;
// the Schur form where the column is short enough); u, v rows are copied
static hipError_t column_precond(const L3Params &h, double alpha, const double *v, double *z, hipStream_t s)
{
    GmresArgs g{};
    g.b = v; g.x0 = nullptr; g.x = z; g.alpha = alpha; g.rtol = 1e-6;
    g.restart = kGmresRegM; g.max_restarts = 10; g.iters = nullptr;
    g.schur = h.nz - 2 <= 64 * kGmresSchurSlots ? 1 : 0;
    return launch_gmres(h.hv, g, s);
}

hipError_t gmres3d(const L3Params &h, const G3Work &w, double alpha, const double *b, const double *x0, double *x,
                   int m, int max_restarts, double rtol, bool precond, hipStream_t s, int *iters, double *relres)
{
    const long n = (long)kNF * h.nx * h.ny * h.nz;
    Kry k{h, w, s, n};
    hipError_t e;
    double *V = w.V;   // (m + 1) vectors of n
    double tmp[kKryMaxV + 1];
    // ||b||
    if ((e = k.dots(V, 0, b, tmp)) != hipSuccess) return e;
    const double bn = std::sqrt(tmp[0]);
    *iters = 0;
    *relres = 0.0;
    if (x0 != x) {
        e = hipMemcpyAsync(x, x0 ? x0 : b, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    if (bn == 0.0) {
        const double z = 0.0;
        return k.axpy(V, 0, &z, x, x, 0.0, false, nullptr);   // x = 0
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    for (int cyc = 0; cyc <= max_restarts; ++cyc) {
        // r = b - (x - alpha L x) into V_0
        if ((e = launch_l3(h, x, w.t, 1.0, -alpha, s)) != hipSuccess) return e;
        const double one = 1.0;
        double r2 = 0.0;
        if ((e = k.axpy(w.t, 1, &one, b, V, 1.0, true, &r2)) != hipSuccess) return e;
        const double beta = std::sqrt(r2);
        *relres = beta / bn;
        if (beta <= rtol * bn) return hipSuccess;
        if ((e = k.axpy(V, 0, &one, V, V, 1.0 / beta, false, nullptr)) != hipSuccess) return e;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool conv = false;
        for (; j < m; ++j) {
            double *vj = V + (long)j * n, *vn = V + (long)(j + 1) * n;
            // flexible GMRES: z_j = M^-1 v_j kept, the new direction is A z_j
            const double *zj = vj;
            if (precond) {
                double *zz = w.Z + (long)j * n;
                if ((e = column_precond(h, alpha, vj, zz, s)) != hipSuccess) return e;
                zj = zz;
            }
            if ((e = launch_l3(h, zj, vn, 1.0, -alpha, s)) != hipSuccess) return e;
            // classical Gram-Schmidt, a second pass when the kept norm is small
            double hc[kKryMaxV + 1], h2[kKryMaxV + 1];
            if ((e = k.dots(V, j + 1, vn, hc)) != hipSuccess) return e;
            const double w2 = hc[j + 1];
            double k2 = 0.0;
            if ((e = k.axpy(V, j + 1, hc, vn, vn, 1.0, true, &k2)) != hipSuccess) return e;
            if (k2 < 1e-4 * w2) {
                if ((e = k.dots(V, j + 1, vn, h2)) != hipSuccess) return e;
                for (int i = 0; i <= j; ++i) hc[i] += h2[i];
                if ((e = k.axpy(V, j + 1, h2, vn, vn, 1.0, true, &k2)) != hipSuccess) return e;
            }
            const double hn = std::sqrt(k2);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0) {
                const double sc = 1.0 / hn;
                const double z = 0.0;
                if ((e = k.axpy(V, 0, &z, vn, vn, sc, false, nullptr)) != hipSuccess) return e;
            }
            // Givens rotations
            for (int i = 0; i < j; ++i) {
                const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * a1;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
            }
            const double a0 = H[(size_t)j * m + j], a1 = H[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a0, a1);
            cs[j] = rr > 0.0 ? a0 / rr : 1.0;
            sn[j] = rr > 0.0 ? a1 / rr : 0.0;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++*iters;
            if (std::fabs(g[j + 1]) <= rtol * bn || hn == 0.0) {
                conv = true;
                ++j;
                break;
            }
        }
        // x += V y, H y = g (upper triangular, j columns)
        for (int i = j - 1; i >= 0; --i) {
            double v = g[i];
            for (int l = i + 1; l < j; ++l) v -= H[(size_t)i * m + l] * y[l];
            y[i] = v / H[(size_t)i * m + i];
        }
        std::vector<double> ny(j);
        for (int i = 0; i < j; ++i) ny[i] = -y[i];
        if ((e = k.axpy(precond ? w.Z : V, j, ny.data(), x, x, 1.0, false, nullptr)) != hipSuccess) return e;
        (void)conv;
    }
    // final residual after the last cycle
    if ((e = launch_l3(h, x, w.t, 1.0, -alpha, s)) != hipSuccess) return e;
    const double one = 1.0;
    double r2 = 0.0;
    if ((e = k.axpy(w.t, 1, &one, b, V, 1.0, true, &r2)) != hipSuccess) return e;
    *relres = std::sqrt(r2) / bn;
    return hipSuccess;
}

}  // namespace nh
