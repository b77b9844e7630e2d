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
// in a fixed order and its small Hessenberg problem solved on the device;
// optionally right-preconditioned by the column systems of the 1D split
// (flexible GMRES, since those are solved iteratively).
#include "nh_internal.h"

#include <cmath>
#include <vector>

namespace nh {

// out[f] = a x[f] + c (L x)[f] at every node, all of L in one walk (out may
// not alias x).  Walls: u rows zero at x walls, v rows at y walls, w rows at
// the bottom and top.  A workgroup of 64 x 8 lattice columns walks a chunk
// of kL3KZ levels.  Per level it stages the planes of u, v and p'_L of its
// tile plus an N-wide x/y halo in LDS (two buffers, one barrier per level)
// for the x and y taps; the vertical part (L_v) comes from a (2N+1)-level
// window of rho0 w and p'_L of the thread's own column in registers, filled
// with the N levels below the chunk and the N levels above each level as
// the walk goes (taps outside the column see zero inputs), as in the
// column-walking L_v kernel.  All loads of a level, the window's lead level
// included, are issued two levels ahead into register slots indexed at
// compile time.  Chunks of levels give enough workgroups on meshes of few
// columns.
constexpr int kL3TX = 64, kL3TY = 8, kL3KZ = 16, kL3P = 2;

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

// (lev and gz are h.lev and h.hv.gz passed again as restrict pointers so
// that their per-level values are read with scalar loads)
template <int N>
__global__ void __launch_bounds__(kL3TX * kL3TY) l3_tile_kernel(L3Params h, const double *__restrict__ x,
                                                                double *out, double a, double c,
                                                                const double *__restrict__ lev,
                                                                const double *__restrict__ gz, const int *gate)
{
    if (gate && *gate == 0) return;
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
    const double gamma = h.gamma, grav = h.hv.g;
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
    // rho0 w and p'_L of the own column at level kk (zero outside the column)
    auto vert = [&](int kk, double r, double w, double th, double &va, double &vb) {
        const double *L = lev + (long)(kk < 0 ? 0 : kk < nz ? kk : nz - 1) * kLevW;
        const bool in = kk >= 0 && kk < nz;
        va = in ? L[0] * w : 0.0;
        vb = in ? gamma * L[2] * (r * L[7] + th * L[8]) : 0.0;
    };
    // the vertical window: slots o = 0 .. 2N hold levels k - N + o
    double ta[NC], tb[NC];
#pragma unroll
    for (int o = 0; o < 2 * N; ++o) {
        const int kk = kb - N + o;
        const long L = (long)(kk < 0 ? 0 : kk < nz ? kk : nz - 1) * nxy;
        vert(kk, x[col + L], x[3 * U + col + L], x[4 * U + col + L], ta[o], tb[o]);
    }
    // slot contents: staged rho', u, v, theta' of NS nodes; own rho', w,
    // theta' of x at the level and at the window's lead level (level + N)
    double sr[P][NS], su[P][NS], sv2[P][NS], st[P][NS], ox[P][3], oz[P][3];
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
        const int kz = k + N;
        const long Z = (long)(kz < nz ? kz : nz - 1) * nxy;
        oz[p][0] = x[col + Z];
        oz[p][1] = x[3 * U + col + Z];
        oz[p][2] = x[4 * U + col + Z];
    };
    l3_unrolled<0, P>([&](auto J) { load(decltype(J)::value, kb + decltype(J)::value); });
    for (int k0 = kb; k0 < ke; k0 += P) {
        l3_unrolled<0, P>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const int k = k0 + j;
            const double *Lv = lev + level(k) / nxy * kLevW;
            const double rho0 = Lv[0], p0 = Lv[2], dth0 = Lv[3], tau = Lv[4], irho0 = Lv[7], ith0 = Lv[8];
            const double gp = gamma * p0;
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
            vert(k + N, oz[j][0], oz[j][1], oz[j][2], ta[2 * N], tb[2 * N]);
            load(j, k + P);
            // vertical part at level k
            const double *G = gz + (long)(k < ke ? k : ke - 1) * NC;
            double d_rw = 0.0, d_pl = 0.0;
#pragma unroll
            for (int o = 0; o < NC; ++o) {
                d_rw += G[o] * ta[o];
                d_pl += G[o] * tb[o];
            }
#pragma unroll
            for (int o = 0; o < 2 * N; ++o) {
                ta[o] = ta[o + 1];
                tb[o] = tb[o + 1];
            }
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
            double Lr = -d_rw - rho0 * (dux + dvy);
            double Lu = -irho0 * dpx, Lvv = -irho0 * dpy;
            double Lw = -d_pl * irho0 - grav * xr * irho0 - tau * xw;
            const double Lt = -xw * dth0;
            if (!h.perx && (ix == 0 || ix == h.nx - 1)) Lu = 0.0;
            if (!h.pery && (iy == 0 || iy == h.ny - 1)) Lvv = 0.0;
            if (k == 0 || k == nz - 1) Lw = 0.0;
            if (own && k < ke) {
                const long I = col + (long)k * nxy;
                out[I] = a * xr + c * Lr;
                out[U + I] = a * xu + c * Lu;
                out[2 * U + I] = a * xv + c * Lvv;
                out[3 * U + I] = a * xw + c * Lw;
                out[4 * U + I] = a * xt + c * Lt;
            }
        });
    }
}

hipError_t launch_l3(const L3Params &h, const double *x, double *out, double a, double c, hipStream_t s,
                     const int *gate)
{
    const int ntx = (h.nx + kL3TX - 1) / kL3TX, nty = (h.ny + kL3TY - 1) / kL3TY;
    const int nkc = (h.nz + kL3KZ - 1) / kL3KZ;
    const dim3 grid((unsigned)(ntx * nty * nkc)), blk(kL3TX * kL3TY);
    switch (h.N) {
    case 2: hipLaunchKernelGGL(l3_tile_kernel<2>, grid, blk, 0, s, h, x, out, a, c, h.lev, h.hv.gz, gate); break;
    case 3: hipLaunchKernelGGL(l3_tile_kernel<3>, grid, blk, 0, s, h, x, out, a, c, h.lev, h.hv.gz, gate); break;
    case 4: hipLaunchKernelGGL(l3_tile_kernel<4>, grid, blk, 0, s, h, x, out, a, c, h.lev, h.hv.gz, gate); break;
    case 5: hipLaunchKernelGGL(l3_tile_kernel<5>, grid, blk, 0, s, h, x, out, a, c, h.lev, h.hv.gz, gate); break;
    case 6: hipLaunchKernelGGL(l3_tile_kernel<6>, grid, blk, 0, s, h, x, out, a, c, h.lev, h.hv.gz, gate); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- Krylov kernels on n-vectors.  Dot products are summed per block into
// quantity-major partials, then by one workgroup in a fixed order: the same
// result on every call.  The Hessenberg problem, the rotations and the
// convergence test live on the device (G3State), so the host queues the
// launches of a cycle ahead of their results; launches past the end of the
// process see their gate flag at 0 and return at once.
constexpr int kKryBlocks = 1024, kKryThreads = 256, kKryMaxV = 34, kKryCtl = 1024;

__device__ __forceinline__ double kry_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// part[j][b] = sum over block b's elements of V_j . w (j < NV), and
// part[NV][b] = w . w.  All loads of an iteration are unconditional (the
// index of a lane past the end is clamped and its weight zeroed after the
// loads), so they are in flight together; for short bases each lane takes
// UF elements a grid stride apart, so that every CU still has enough bytes
// in flight to run at memory speed.
template <int NV>
__global__ void __launch_bounds__(kKryThreads) kry_dots_kernel(const double *__restrict__ V, long stride,
                                                               const double *__restrict__ w, long n,
                                                               double *__restrict__ part, const int *gate)
{
    constexpr int UF = NV <= 1 ? 4 : NV <= 3 ? 2 : 1;
    if (gate && *gate == 0) return;
    __shared__ double red[kKryThreads / 64][NV + 1];
    double acc[NV + 1];
#pragma unroll
    for (int j = 0; j <= NV; ++j) acc[j] = 0.0;
    const long S = (long)gridDim.x * kKryThreads;
    for (long i0 = blockIdx.x * (long)kKryThreads + threadIdx.x; i0 < n; i0 += S * UF) {
        long ii[UF];
        double wi[UF], vv[NV > 0 ? NV : 1][UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) ii[u] = i0 + u * S < n ? i0 + u * S : n - 1;
#pragma unroll
        for (int u = 0; u < UF; ++u) wi[u] = w[ii[u]];
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int u = 0; u < UF; ++u) vv[j][u] = V[j * stride + ii[u]];
#pragma unroll
        for (int u = 1; u < UF; ++u)
            if (i0 + u * S >= n) wi[u] = 0.0;
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            acc[NV] += wi[u] * wi[u];
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] += vv[j][u] * wi[u];
        }
    }
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int j = 0; j <= NV; ++j) {
        const double s = kry_wave_sum(acc[j]);
        if (lane == 0) red[wv][j] = s;
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= NV; j += kKryThreads) {
        double s = 0.0;
        for (int q = 0; q < kKryThreads / 64; ++q) s += red[q][j];
        part[(long)j * kKryBlocks + blockIdx.x] = s;
    }
}

template <int NV>
static void launch_dots(int nv, const double *V, long n, const double *x, double *part, const int *gate,
                        hipStream_t s)
{
    if constexpr (NV <= kG3MaxRestart) {
        if (nv == NV)
            hipLaunchKernelGGL(kry_dots_kernel<NV>, dim3(kKryBlocks), dim3(kKryThreads), 0, s, V, n, x, n, part,
                               gate);
        else
            launch_dots<NV + 1>(nv, V, n, x, part, gate, s);
    }
}

// y = s (w - sum_j c_j V_j) for j < nv, nv = *nvp when given, s = *sc when
// given (else 1), coefficients c in device memory; with norm also part[0][b]
// = block sums of (w - sum_j c_j V_j)^2.  y may alias w.
__global__ void __launch_bounds__(kKryThreads) kry_axpy_kernel(const double *__restrict__ V, long stride, int nv,
                                                               const int *nvp, const double *cf, const double *w,
                                                               double *y, long n, const double *sc, int norm,
                                                               double *__restrict__ part, const int *gate)
{
    if (gate && *gate == 0) return;
    __shared__ double red[kKryThreads / 64];
    const int nvv = nvp ? *nvp : nv;
    const double s = sc ? *sc : 1.0;
    double acc = 0.0;
    for (long i = blockIdx.x * (long)kKryThreads + threadIdx.x; i < n; i += (long)gridDim.x * kKryThreads) {
        double v = w[i];
#pragma unroll 4
        for (int j = 0; j < nvv; ++j) v -= cf[j] * V[j * stride + i];
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
        part[blockIdx.x] = r;
    }
}

// The nq quantities of the block partials summed into out (LDS): wave v
// sums quantities v, v + 16, ..., each lane a fixed strided subset of the
// blocks, then a fixed butterfly.  Ends with a barrier.
__device__ void kry_reduce(const double *__restrict__ part, int nq, double *out)
{
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int q = wv; q < nq; q += kKryCtl / 64) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < kKryBlocks / 64; ++b) s += part[(long)q * kKryBlocks + b * 64 + lane];
        s = kry_wave_sum(s);
        if (lane == 0) out[q] = s;
    }
    __syncthreads();
}

__device__ void g3_publish(const G3State *st, G3Status *hs)
{
    volatile G3Status *v = hs;
    v->go = st->go;
    v->open = st->open;
    v->iters = st->iters;
    v->relres = st->relres;
    __threadfence_system();
}

// Start of a solve: ||b|| from the partials of b . b
__global__ void __launch_bounds__(kKryCtl) g3_begin_kernel(G3State *st, const double *__restrict__ part,
                                                           G3Status *hs)
{
    __shared__ double red[1];
    kry_reduce(part, 1, red);
    if (threadIdx.x != 0) return;
    const double bn = sqrt(red[0]);
    st->bn = bn;
    st->bzero = bn == 0.0;
    st->open = bn > 0.0;
    st->go = 0;
    st->pass2 = 0;
    st->ncols = 0;
    st->iters = 0;
    st->relres = 0.0;
    st->one = 1.0;
    st->zero = 0.0;
    g3_publish(st, hs);
}

// Start of a cycle: beta = ||r|| from the partials of the residual; the solve
// ends when beta <= rtol ||b||, else (unless this is the final check) the
// Arnoldi process starts from V_0 = r / beta.
__global__ void __launch_bounds__(kKryCtl) g3_cycle_kernel(G3State *st, const double *__restrict__ part,
                                                           double rtol, int final, G3Status *hs)
{
    if (st->open == 0) return;
    __shared__ double red[1];
    kry_reduce(part, 1, red);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(red[0]), bn = st->bn;
    st->relres = beta / bn;
    st->ncols = 0;
    st->pass2 = 0;
    if (beta <= rtol * bn) {
        st->open = 0;
        st->go = 0;
    } else {
        st->go = final ? 0 : 1;
        st->scale = 1.0 / beta;
        st->gv[0] = beta;
        for (int i = 1; i <= kG3MaxRestart; ++i) st->gv[i] = 0.0;
    }
    g3_publish(st, hs);
}

// Column j of the Hessenberg matrix from the partials of V_i . w (i <= j) and
// w . w (pass 1) or of the second pass.  The norm of the kept part is
// ||w||^2 - sum h_i^2 when that keeps at least 1e-4 of ||w||^2 (the vector
// is then written normalised by the combination that orthogonalises it);
// otherwise a second pass orthogonalises the kept part again and its norm
// comes from that pass.  Then the earlier rotations, a new one, the rotated
// residual and the convergence test.
__global__ void __launch_bounds__(kKryCtl) g3_column_kernel(G3State *st, const double *__restrict__ part, int j,
                                                            int m, double rtol, int pass, G3Status *hs)
{
    if (pass == 1 ? st->go == 0 : st->pass2 == 0) return;
    __shared__ double red[kKryMaxV + 1];
    kry_reduce(part, j + 2, red);
    if (threadIdx.x != 0) return;
    double h2 = 0.0;
    for (int i = 0; i <= j; ++i) h2 += red[i] * red[i];
    const double w2 = red[j + 1];
    double k2 = w2 - h2;
    if (pass == 1) {
        for (int i = 0; i <= j; ++i) st->coef[i] = red[i];
        if (!(k2 >= 1e-4 * w2)) {   // second pass
            for (int i = 0; i <= j; ++i) st->hc[i] = red[i];
            st->pass2 = 1;
            st->scale = 1.0;
            return;
        }
        for (int i = 0; i <= j; ++i) st->hc[i] = red[i];
        st->pass2 = 0;
    } else {
        for (int i = 0; i <= j; ++i) {
            st->coef[i] = red[i];
            st->hc[i] += red[i];
        }
    }
    const double hn = k2 > 0.0 ? sqrt(k2) : 0.0;
    st->scale = hn > 0.0 ? 1.0 / hn : 0.0;
    double *H = st->H;
    constexpr int R = kG3MaxRestart;
    for (int i = 0; i <= j; ++i) H[i * R + j] = st->hc[i];
    H[(j + 1) * R + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a0 = H[i * R + j], a1 = H[(i + 1) * R + j];
        H[i * R + j] = st->cs[i] * a0 + st->sn[i] * a1;
        H[(i + 1) * R + j] = -st->sn[i] * a0 + st->cs[i] * a1;
    }
    const double a0 = H[j * R + j], a1 = H[(j + 1) * R + j];
    const double rr = hypot(a0, a1);
    st->cs[j] = rr > 0.0 ? a0 / rr : 1.0;
    st->sn[j] = rr > 0.0 ? a1 / rr : 0.0;
    H[j * R + j] = rr;
    H[(j + 1) * R + j] = 0.0;
    st->gv[j + 1] = -st->sn[j] * st->gv[j];
    st->gv[j] = st->cs[j] * st->gv[j];
    st->iters += 1;
    st->ncols = j + 1;
    // estimate met (the next cycle checks the true residual), breakdown or
    // the restart length reached
    if (fabs(st->gv[j + 1]) <= rtol * st->bn || hn == 0.0 || j + 1 == m) {
        st->go = 0;
        st->pass2 = 0;
    }
    g3_publish(st, hs);
}

// End of a cycle: H y = g over the cycle's columns (upper triangular), and
// the coefficients -y of the update x += Z y (Z = V unpreconditioned)
__global__ void __launch_bounds__(64) g3_end_kernel(G3State *st)
{
    const int nc = st->ncols;
    if (nc == 0 || threadIdx.x != 0) return;
    constexpr int R = kG3MaxRestart;
    double y[kG3MaxRestart];
    for (int i = nc - 1; i >= 0; --i) {
        double v = st->gv[i];
        for (int l = i + 1; l < nc; ++l) v -= st->H[i * R + l] * y[l];
        y[i] = v / st->H[i * R + i];
    }
    for (int i = 0; i < nc; ++i) st->coef[i] = -y[i];
}

namespace {

struct Kry {
    const G3Work &w;
    hipStream_t s;
    long n;

    void dots(const double *V, int nv, const double *x, const int *gate)
    {
        launch_dots<0>(nv, V, n, x, w.part, gate, s);
    }
    // y = sc (x - sum_j cf_j V_j)
    void axpy(const double *V, int nv, const int *nvp, const double *cf, const double *x, double *y,
              const double *sc, bool norm, const int *gate)
    {
        hipLaunchKernelGGL(kry_axpy_kernel, dim3(kKryBlocks), dim3(kKryThreads), 0, s, V, n, nv, nvp, cf, x, y, n, sc,
                           norm ? 1 : 0, w.part, gate);
    }
};

}  // namespace

// z = (I - alpha L_v)^-1 v column by column (column GMRES(10) to rtol 1e-6;
// the Schur form where the column is short enough); u, v rows are copied
static hipError_t column_precond(const L3Params &h, double alpha, const double *v, double *z, const int *gate,
                                 hipStream_t s)
{
    GmresArgs g{};
    g.b = v; g.x0 = nullptr; g.x = z; g.alpha = alpha; g.rtol = 1e-6;
    g.restart = kGmresRegM; g.max_restarts = 10; g.iters = nullptr;
    g.schur = h.nz - 2 <= 64 * kGmresSchurSlots ? 1 : 0;
    g.gate = gate;
    return launch_gmres(h.hv, g, s);
}

// The host queues one Arnoldi step while the previous one runs: before it
// queues step j it waits for the event after step j - 2 (the cycle start for
// j = 1) and reads the status the kernels wrote, so at most one step is
// queued past the end of the process, and that one does nothing.  One
// stream synchronisation per solve reads the result.
hipError_t gmres3d(const L3Params &h, const G3Work &w, double alpha, const double *b, const double *x0, double *x,
                   int m, int max_restarts, double rtol, bool precond, hipStream_t s, int *iters, double *relres)
{
    const long n = (long)kNF * h.nx * h.ny * h.nz;
    Kry k{w, s, n};
    hipError_t e;
    G3State *st = w.state;
    double *V = w.V;   // (m + 1) vectors of n
    *iters = 0;
    *relres = 0.0;
    // ||b||, x = x0 (or b); x = 0 when b = 0
    k.dots(V, 0, b, nullptr);
    hipLaunchKernelGGL(g3_begin_kernel, dim3(1), dim3(kKryCtl), 0, s, st, (const double *)w.part, w.status_dev);
    if (x0 != x) k.axpy(V, 0, nullptr, nullptr, x0 ? x0 : b, x, nullptr, false, nullptr);
    k.axpy(V, 0, nullptr, nullptr, x, x, &st->zero, false, &st->bzero);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    auto mark = [&](int i) { return hipEventRecord(w.ev[i & 1], s); };
    for (int cyc = 0; cyc <= max_restarts + 1; ++cyc) {
        const bool final = cyc == max_restarts + 1;
        // r = b - (x - alpha L x) into V_0, ||r||, then V_0 = r / ||r||
        if ((e = launch_l3(h, x, w.t, 1.0, -alpha, s, &st->open)) != hipSuccess) return e;
        k.axpy(w.t, 1, nullptr, &st->one, b, V, nullptr, true, &st->open);
        hipLaunchKernelGGL(g3_cycle_kernel, dim3(1), dim3(kKryCtl), 0, s, st, (const double *)w.part, rtol,
                           final ? 1 : 0, w.status_dev);
        if (final) break;
        k.axpy(V, 0, nullptr, nullptr, V, V, &st->scale, false, &st->go);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(0)) != hipSuccess) return e;
        bool waited = false;
        for (int j = 0; j < m; ++j) {
            if (j >= 1) {
                if ((e = hipEventSynchronize(w.ev[(j - 1) & 1])) != hipSuccess) return e;
                waited = true;
                if (w.status->go == 0) break;
            }
            double *vj = V + (long)j * n, *vn = V + (long)(j + 1) * n;
            // flexible GMRES: z_j = M^-1 v_j kept, the new direction is A z_j
            const double *zj = vj;
            if (precond) {
                double *zz = w.Z + (long)j * n;
                if ((e = column_precond(h, alpha, vj, zz, &st->go, s)) != hipSuccess) return e;
                zj = zz;
            }
            if ((e = launch_l3(h, zj, vn, 1.0, -alpha, s, &st->go)) != hipSuccess) return e;
            // classical Gram-Schmidt, the second pass gated on the first's verdict
            k.dots(V, j + 1, vn, &st->go);
            hipLaunchKernelGGL(g3_column_kernel, dim3(1), dim3(kKryCtl), 0, s, st, (const double *)w.part, j, m, rtol,
                               1, w.status_dev);
            k.axpy(V, j + 1, nullptr, st->coef, vn, vn, &st->scale, false, &st->go);
            k.dots(V, j + 1, vn, &st->pass2);
            hipLaunchKernelGGL(g3_column_kernel, dim3(1), dim3(kKryCtl), 0, s, st, (const double *)w.part, j, m, rtol,
                               2, w.status_dev);
            k.axpy(V, j + 1, nullptr, st->coef, vn, vn, &st->scale, false, &st->pass2);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = mark(j + 1)) != hipSuccess) return e;
        }
        if (!waited && (e = hipEventSynchronize(w.ev[0])) != hipSuccess) return e;
        // x += Z y over the cycle's columns
        hipLaunchKernelGGL(g3_end_kernel, dim3(1), dim3(64), 0, s, st);
        k.axpy(precond ? w.Z : V, 0, &st->ncols, st->coef, x, x, nullptr, false, &st->ncols);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (w.status->open == 0) break;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *iters = w.status->iters;
    *relres = w.status->relres;
    return hipSuccess;
}

}  // namespace nh
