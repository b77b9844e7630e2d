// gfx950 kernels and the host-driven Krylov loop of the 3D-IMEX split
// (paper, Sec. 2.3: IMEX with the linear fast-wave operator treated
// implicitly, ARK2, matrix-free GMRES).  Here the linear operator is taken
// over all three directions:
//   (L)_rho'   = - rho0 (d/dx u + d/dy v) - d/dz (rho0 w)
//   (L)_u      = - (1/rho0) dp'_L/dx,   (L)_v = - (1/rho0) dp'_L/dy
//   (L)_w      = - (1/rho0) dp'_L/dz - g rho'/rho0 - tau(z) w
//   (L)_theta' = - w dtheta0/dz,        p'_L = gamma p0 (rho'/rho0 + theta'/theta0),
// the vertical terms from the column-walking L_v kernel, the horizontal ones
// from the DSS'd x/y derivative stencils of the explicit path (a tiled pass
// with the x/y planes staged in LDS), the damping
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
// node, lv holding L_v x (u, v rows zero; lv may alias out, x may not).
// Walls: u rows zero at x walls, v rows at y walls, w rows at the bottom and
// top.  A workgroup of 64 x 8 lattice columns walks a chunk of kL3KZ levels, staging per level the planes of u, v and p'_L of
// its tile plus an N-wide x/y halo in LDS (two buffers, one barrier per
// level); the x and y taps come from LDS, the node's own rho', w, theta' and
// L_v rows from coalesced loads.  All loads of a level are issued two levels
// ahead into register slots indexed at compile time.  Chunks of levels give
// enough workgroups on meshes of few columns.
constexpr int kL3TX = 64, kL3TY = 8, kL3KZ = 8, kL3P = 2;

__device__ __forceinline__ int l3_xcd_block(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

template <int I, int E, class F>
__device__ __forceinline__ void l3_unrolled(F &&f)
{
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        l3_unrolled<I + 1, E>(f);
    }
}

// (lev is h.lev passed again as a restrict pointer so that its per-level
// values are read with scalar loads)
template <int N>
__global__ void __launch_bounds__(kL3TX * kL3TY) l3_tile_kernel(L3Params h, const double *__restrict__ x,
                                                                const double *lv, double *out, double a, double c,
                                                                const double *__restrict__ lev)
{
    constexpr int NC = 2 * N + 1, PX = kL3TX + 2 * N, PY = kL3TY + 2 * N, PS = PX * PY;
    constexpr int NT = kL3TX * kL3TY, NS = (PS + NT - 1) / NT, P = kL3P;
    __shared__ double tile[2][3][PS];   // u, v, p'_L
    const long nxy = (long)h.nx * h.ny;
    const int nz = h.nz;
    const long U = nxy * nz;
    const int ntx = (h.nx + kL3TX - 1) / kL3TX, nty = (h.ny + kL3TY - 1) / kL3TY;
    const int t = l3_xcd_block(blockIdx.x, gridDim.x);
    const int tt = t % (ntx * nty), kc = t / (ntx * nty);
    const int kb = kc * kL3KZ, ke = kb + kL3KZ < nz ? kb + kL3KZ : nz;
    const int tx = threadIdx.x % kL3TX, ty = threadIdx.x / kL3TX;
    const int x0 = (tt % ntx) * kL3TX, y0 = (tt / ntx) * kL3TY;
    const int ix = x0 + tx, iy = y0 + ty;
    const bool own = ix < h.nx && iy < h.ny;
    const long col = own ? ix + (long)iy * h.nx : 0;
    double cx[NC], cy[NC];
#pragma unroll
    for (int o = 0; o < NC; ++o) {
        cx[o] = own ? h.gx[(long)ix * NC + o] : 0.0;
        cy[o] = own ? h.gy[(long)iy * NC + o] : 0.0;
    }
    long sc[NS];
    bool sv[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int s = threadIdx.x + i * NT;
        int jx = x0 - N + s % PX, jy = y0 - N + s / PX;
        bool ok = s < PS;
        if (jx < 0 || jx >= h.nx) {
            ok = ok && h.perx;
            jx = ((jx % h.nx) + h.nx) % h.nx;
        }
        if (jy < 0 || jy >= h.ny) {
            ok = ok && h.pery;
            jy = ((jy % h.ny) + h.ny) % h.ny;
        }
        sv[i] = ok;
        sc[i] = ok ? jx + (long)jy * h.nx : 0;
    }
    auto level = [&](int k) -> long { return (long)(k < ke ? k : ke - 1) * nxy; };
    // slot contents: staged rho', u, v, theta' of NS nodes; own rho', w,
    // theta' of x and of L_v x
    double sr[P][NS], su[P][NS], sv2[P][NS], st[P][NS], ox[P][3], ol[P][3];
    auto load = [&](int p, int k) {
        const long L = level(k);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            sr[p][i] = x[sc[i] + L];
            su[p][i] = x[U + sc[i] + L];
            sv2[p][i] = x[2 * U + sc[i] + L];
            st[p][i] = x[4 * U + sc[i] + L];
        }
        ox[p][0] = x[col + L];
        ox[p][1] = x[3 * U + col + L];
        ox[p][2] = x[4 * U + col + L];
        ol[p][0] = lv[col + L];
        ol[p][1] = lv[3 * U + col + L];
        ol[p][2] = lv[4 * U + col + L];
    };
    l3_unrolled<0, P>([&](auto J) { load(decltype(J)::value, kb + decltype(J)::value); });
    for (int k0 = kb; k0 < ke; k0 += P) {
        l3_unrolled<0, P>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const int k = k0 + j;
            const double *Lv = lev + level(k) / nxy * kLevW;
            const double rho0 = Lv[0], p0 = Lv[2], tau = Lv[4], irho0 = Lv[7], ith0 = Lv[8];
            const double gp = h.gamma * p0;
            double(*T)[PS] = tile[(k - kb) & 1];
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                const int sidx = threadIdx.x + i * NT;
                if (sidx < PS) {
                    T[0][sidx] = sv[i] ? su[j][i] : 0.0;
                    T[1][sidx] = sv[i] ? sv2[j][i] : 0.0;
                    T[2][sidx] = sv[i] ? gp * (sr[j][i] * irho0 + st[j][i] * ith0) : 0.0;
                }
            }
            const double xr = ox[j][0], xw = ox[j][1], xt = ox[j][2];
            const double lr = ol[j][0], lw = ol[j][1], lt = ol[j][2];
            load(j, k + P);
            __syncthreads();
            double dux = 0.0, dpx = 0.0, dvy = 0.0, dpy = 0.0;
#pragma unroll
            for (int o = 0; o < NC; ++o) {
                const int jx = (ty + N) * PX + tx + o, jy = (ty + o) * PX + tx + N;
                dux += cx[o] * T[0][jx];
                dpx += cx[o] * T[2][jx];
                dvy += cy[o] * T[1][jy];
                dpy += cy[o] * T[2][jy];
            }
            const int jo = (ty + N) * PX + tx + N;
            const double xu = T[0][jo], xv = T[1][jo];
            double Lr = lr - rho0 * (dux + dvy);
            double Lu = -irho0 * dpx, Lvv = -irho0 * dpy;
            double Lw = lw - tau * xw;
            if (!h.perx && (ix == 0 || ix == h.nx - 1)) Lu = 0.0;
            if (!h.pery && (iy == 0 || iy == h.ny - 1)) Lvv = 0.0;
            if (k == 0 || k == nz - 1) Lw = 0.0;
            if (own && k < ke) {
                const long I = col + (long)k * nxy;
                out[I] = a * xr + c * Lr;
                out[U + I] = a * xu + c * Lu;
                out[2 * U + I] = a * xv + c * Lvv;
                out[3 * U + I] = a * xw + c * Lw;
                out[4 * U + I] = a * xt + c * lt;
            }
        });
    }
}

hipError_t launch_l3(const L3Params &h, const double *x, double *out, double a, double c, hipStream_t s)
{
    hipError_t e = launch_lv_apply(h.hv, x, out, s, true);
    if (e != hipSuccess) return e;
    const int ntx = (h.nx + kL3TX - 1) / kL3TX, nty = (h.ny + kL3TY - 1) / kL3TY;
    const int nkc = (h.nz + kL3KZ - 1) / kL3KZ;
    const dim3 grid((unsigned)(ntx * nty * nkc)), blk(kL3TX * kL3TY);
    switch (h.N) {
    case 2: hipLaunchKernelGGL(l3_tile_kernel<2>, grid, blk, 0, s, h, x, (const double *)out, out, a, c, h.lev); break;
    case 3: hipLaunchKernelGGL(l3_tile_kernel<3>, grid, blk, 0, s, h, x, (const double *)out, out, a, c, h.lev); break;
    case 4: hipLaunchKernelGGL(l3_tile_kernel<4>, grid, blk, 0, s, h, x, (const double *)out, out, a, c, h.lev); break;
    case 5: hipLaunchKernelGGL(l3_tile_kernel<5>, grid, blk, 0, s, h, x, (const double *)out, out, a, c, h.lev); break;
    case 6: hipLaunchKernelGGL(l3_tile_kernel<6>, grid, blk, 0, s, h, x, (const double *)out, out, a, c, h.lev); break;
    default: return hipErrorInvalidValue;
    }
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
            if (std::fabs(g[j + 1]) <= rtol * bn || hn == 0.0) {   // estimate met (the next cycle checks the true residual)
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
