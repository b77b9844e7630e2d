// gfx950 kernel of the tensor hyper-diffusion term H_q = -(div tau grad)^2 q
// (alpha = 2), with tau = (J E) diag(nu_i lambda_i^-1) (J E)^T from the
// eigendecomposition of the metric tensor and nu_i = c_i^(1/2) dx_i^2 / dt^(1/2)
// (paper, section on tensor-based hyper-diffusion).
//
// On the axis-aligned box elements of the lattice, J and G are diagonal and
// tau = diag(tau_x, tau_y, tau_z) per element, each direction's value set by
// its rank among the element's extents.  The continuous-Galerkin weak form
// of div tau grad with the co-located LGL quadrature, after direct stiffness
// summation and the inverse diagonal mass, then separates into one assembled
// 1D operator per direction: (L q)_x = -m_x^-1 K_x q along x lines with
// K_x = sum_e (tau_x,e / a_e) D^T W D and m_x = sum_e a_e W (a_e the half
// length of element e), and likewise for y and z, provided the ranks do not
// change across the mesh (the host checks this).  Row p of each operator is
// a (2N+1)-tap stencil over the nodes p - N .. p + N of the line; the host
// assembles the rows, wraps periodic directions and leaves taps past a wall
// at zero.
#include "nh_internal.h"

namespace nh {

// Workgroups are handed to the 8 XCDs round robin (b mod 8), each with its
// own L2: give XCD x the contiguous range [x q + min(x, r), ...) of the n
// logical blocks (q = n / 8, r = n mod 8), so that blocks running together on
// one XCD cover neighbouring rows and their y taps hit that L2.
__device__ __forceinline__ int hd_xcd_block(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

// out[f] = scale * L q[f] (out[f] += ... with ACC) for the 5 fields of
// q [5][U].  Tiled column walk: a workgroup of 64 x 16 lattice columns of one
// field walks up the levels; the plane of its tile plus an N-wide x/y halo
// is staged in LDS per level (two planes, one barrier per level), and the z
// taps are accumulated per thread from the staged planes' own nodes (or, at
// orders 5 and 6, taken from a register window of the thread's column).  Halo nodes past a wall are staged as zeros (their coefficients
// are zero); periodic directions wrap.  Measured on a 512 x 512 x 81 lattice
// (N = 4): 64 x 16 tiles beat 64 x 4, 64 x 8, 32 x 8 and 128 x 4 (fewer halo
// re-reads per node), and staging beats reading the x and y taps through
// the caches.
constexpr int kHdTX = 64, kHdTY = 16;
constexpr int kHdRunMaxN = 4;

template <int I, int E, class F>
__device__ __forceinline__ void hd_static_for(F &&f)
{
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        hd_static_for<I + 1, E>(f);
    }
}
// Prefetch depth in levels: 4, or 2 at N = 6 where 4 would spill registers.
// Measured on the 512 x 512 x 81 lattice (N = 4), both passes of H_q:
// 1.26 ms at depth 1, 1.07 at 2, 1.10 at 3, 1.03 at 4.
template <int N>
constexpr int hd_prefetch() { return N >= 6 ? 2 : 4; }

// With wallmask set, the wall-normal velocity rows are left out (zero, or
// unchanged when accumulating): u on the x walls, v on the y walls, w at the
// bottom and top levels, the no-flux condition imposed on the whole tendency.
template <int N, bool ACC, int P = hd_prefetch<N>()>
__global__ void __launch_bounds__(kHdTX * kHdTY) hd_laplace_tile_kernel(HyperParams h, const double *__restrict__ q,
                                                                        double *__restrict__ out, double scale,
                                                                        const double *__restrict__ sz, int wallmask)
{
    constexpr int NC = 2 * N + 1, PX = kHdTX + 2 * N, PY = kHdTY + 2 * N;
    constexpr int NT = kHdTX * kHdTY, NS = (PX * PY + NT - 1) / NT;
    __shared__ double tile[2][PY * PX];
    const long nxy = (long)h.nx * h.ny;
    const int nz = h.nz;
    const long U = nxy * nz;
    const int ntx = (h.nx + kHdTX - 1) / kHdTX, nty = (h.ny + kHdTY - 1) / kHdTY;
    const int t = hd_xcd_block(blockIdx.x, gridDim.x);
    const int f = t / (ntx * nty), tt = t - f * ntx * nty;
    const int tx = threadIdx.x % kHdTX, ty = threadIdx.x / kHdTX;
    const int x0 = (tt % ntx) * kHdTX, y0 = (tt / ntx) * kHdTY;
    const int ix = x0 + tx, iy = y0 + ty;
    const bool own = ix < h.nx && iy < h.ny;
    const long col = own ? ix + (long)iy * h.nx : 0;
    // this column's wall-normal rows: every level (u, v on a wall column) or
    // the bottom and top levels (w)
    const bool colwall = wallmask && ((f == 1 && !h.perx && (ix == 0 || ix == h.nx - 1)) ||
                                      (f == 2 && !h.pery && (iy == 0 || iy == h.ny - 1)));
    const bool zwall = wallmask && f == 3;
    const double *qf = q + (long)f * U;
    double *of = out + (long)f * U;
    double cx[NC], cy[NC];
#pragma unroll
    for (int o = 0; o < NC; ++o) {
        cx[o] = own ? h.sx[(long)ix * NC + o] : 0.0;
        cy[o] = own ? h.sy[(long)iy * NC + o] : 0.0;
    }
    // lattice column of each staged node this thread handles; nodes past a
    // wall (and the padding of the last pass) read column 0 and stage zero
    long sc[NS];
    bool sv[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int s = threadIdx.x + i * NT;
        int jx = x0 - N + s % PX, jy = y0 - N + s / PX;
        bool ok = s < PX * PY;
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
    // Orders up to kHdRunMaxN accumulate the z taps as running sums fed from
    // the staged planes (no second read of the thread's column; 3-5 % faster
    // per H_q at N = 4); higher orders keep a register window of the column,
    // which needs fewer registers there (the running sums spill at N = 5, 6).
    if constexpr (N <= kHdRunMaxN) {
        // Every stream is loaded P levels ahead of its use into a ring of P
        // register slots indexed at compile time (the level loop is unrolled by
        // P, so no value is copied while its load is in flight), unconditionally
        // (levels outside the column are clamped) and masked only where it is
        // consumed: every wait in the loop is then for loads issued P levels
        // earlier.  Slot k mod P holds the staged plane of level k (pre) and,
        // accumulating, the output column at level k - N (apre).
        auto level = [&](int lv) -> long { return (long)(lv < 0 ? 0 : (lv < nz ? lv : nz - 1)) * nxy; };
        // With h.stream the output column (read when accumulating, then
        // written) bypasses the caches: touched once, it should not displace
        // the staged planes' halos from L2.
        auto ld_out = [&](const double *a) -> double {
            if (h.stream) return __builtin_nontemporal_load(a);
            return *a;
        };
        double pre[P][NS], apre[ACC ? P : 1];
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int i = 0; i < NS; ++i) pre[p][i] = qf[sc[i] + level(p)];
            if constexpr (ACC) apre[p] = ld_out(of + col + level(p - N));
        }
        // Running sums of the thread's column: za[o] collects L q at level
        // k - N + o.  The node of level k, read from the staged plane, adds its
        // z tap to each of the 2N + 1 levels it reaches and its x/y part to its
        // own level; level k - N is then complete and is written.  The z values
        // come from the plane already in LDS instead of a second read of the
        // column from memory.
        double za[NC];
#pragma unroll
        for (int o = 0; o < NC; ++o) za[o] = 0.0;
        for (int k0 = 0; k0 < nz + N; k0 += P) {
            hd_static_for<0, P>([&](auto J) {
                constexpr int j = decltype(J)::value;
                const int k = k0 + j;   // levels k >= nz add nothing; levels m >= nz are not written
                double *tl = tile[k & 1];
#pragma unroll
                for (int i = 0; i < NS; ++i)
                    if (threadIdx.x + i * NT < PX * PY) tl[threadIdx.x + i * NT] = sv[i] ? pre[j][i] : 0.0;
#pragma unroll
                for (int i = 0; i < NS; ++i) pre[j][i] = qf[sc[i] + level(k + P)];
                __syncthreads();
                if (k < nz) {
                    double ax = 0.0, ay = 0.0;
#pragma unroll
                    for (int o = 0; o < NC; ++o) {
                        ax += cx[o] * tl[(ty + N) * PX + tx + o];
                        ay += cy[o] * tl[(ty + o) * PX + tx + N];
                    }
                    const double qk = tl[(ty + N) * PX + tx + N];
#pragma unroll
                    for (int o = 0; o < NC; ++o) {
                        const int lv = k - N + o;   // level whose row takes q(k) with tap 2N - o
                        if (lv >= 0 && lv < nz) za[o] += sz[(long)lv * NC + 2 * N - o] * qk;
                    }
                    za[N] += ax + ay;
                }
                const int m = k - N;
                if (m >= 0 && m < nz) {
                    double v = scale * za[0];
                    if (colwall || (zwall && (m == 0 || m == nz - 1))) v = 0.0;
                    if constexpr (ACC) v = apre[j] + v;
                    if (own) {
                        if (h.stream) __builtin_nontemporal_store(v, of + col + (long)m * nxy);
                        else of[col + (long)m * nxy] = v;
                    }
                }
#pragma unroll
                for (int o = 0; o < 2 * N; ++o) za[o] = za[o + 1];
                za[2 * N] = 0.0;
                if constexpr (ACC) apre[j] = ld_out(of + col + level(k + P - N));
            });
        }
    } else {
        // Every stream is loaded P levels ahead of its use into a ring of P
        // register slots indexed at compile time (the level loop is unrolled by
        // P, so no value is copied while its load is in flight), unconditionally
        // (levels past the top are clamped) and masked only where it is consumed:
        // every wait in the loop is then for loads issued P levels earlier.  Slot
        // k mod P holds the staged plane of level k (pre), the own column of q at
        // level k + N + 1 (wpre) and, accumulating, that of out at level k (apre).
        auto level = [&](int lv) -> long { return (long)(lv < nz ? lv : nz - 1) * nxy; };
        // With h.stream the output column (read when accumulating, then
        // written) bypasses the caches: touched once, it should not displace
        // the staged planes' halos from L2.
        auto ld_out = [&](const double *a) -> double {
            if (h.stream) return __builtin_nontemporal_load(a);
            return *a;
        };
        double pre[P][NS], wpre[P], apre[ACC ? P : 1];
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int i = 0; i < NS; ++i) pre[p][i] = qf[sc[i] + level(p)];
            wpre[p] = qf[col + level(N + 1 + p)];
            if constexpr (ACC) apre[p] = ld_out(of + col + level(p));
        }
        double win[NC];   // levels k - N .. k + N of the thread's column
#pragma unroll
        for (int o = 0; o < N; ++o) win[o] = 0.0;
#pragma unroll
        for (int o = 0; o <= N; ++o) win[N + o] = o < nz ? qf[col + level(o)] : 0.0;
        for (int k0 = 0; k0 < nz; k0 += P) {
            hd_static_for<0, P>([&](auto J) {
                constexpr int j = decltype(J)::value;
                const int k = k0 + j;   // levels k >= nz of the last pass compute nothing that is kept
                double *tl = tile[k & 1];
#pragma unroll
                for (int i = 0; i < NS; ++i)
                    if (threadIdx.x + i * NT < PX * PY) tl[threadIdx.x + i * NT] = sv[i] ? pre[j][i] : 0.0;
#pragma unroll
                for (int i = 0; i < NS; ++i) pre[j][i] = qf[sc[i] + level(k + P)];
                __syncthreads();
                const double *Sk = sz + level(k) / nxy * NC;
                double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
                for (int o = 0; o < NC; ++o) {
                    az += Sk[o] * win[o];
                    ax += cx[o] * tl[(ty + N) * PX + tx + o];
                    ay += cy[o] * tl[(ty + o) * PX + tx + N];
                }
                double v = scale * (ax + ay + az);
                if (colwall || (zwall && (k == 0 || k == nz - 1))) v = 0.0;
                if constexpr (ACC) v = apre[j] + v;
                if (own && k < nz) {
                    if (h.stream) __builtin_nontemporal_store(v, of + col + (long)k * nxy);
                    else of[col + (long)k * nxy] = v;
                }
#pragma unroll
                for (int o = 0; o < 2 * N; ++o) win[o] = win[o + 1];
                win[2 * N] = k + N + 1 < nz ? wpre[j] : 0.0;
                wpre[j] = qf[col + level(k + N + 1 + P)];
                if constexpr (ACC) apre[j] = ld_out(of + col + level(k + P));
            });
        }
    }
}

template <int N>
static void hd_launch(const HyperParams &h, const double *q, double *out, double scale, bool accumulate,
                      bool wallmask, hipStream_t s)
{
    const int ntx = (h.nx + kHdTX - 1) / kHdTX, nty = (h.ny + kHdTY - 1) / kHdTY;
    const dim3 grid((unsigned)(ntx * nty * kNF)), blk(kHdTX * kHdTY);
    if (accumulate)
        hipLaunchKernelGGL((hd_laplace_tile_kernel<N, true>), grid, blk, 0, s, h, q, out, scale, h.sz,
                           wallmask ? 1 : 0);
    else
        hipLaunchKernelGGL((hd_laplace_tile_kernel<N, false>), grid, blk, 0, s, h, q, out, scale, h.sz,
                           wallmask ? 1 : 0);
}

hipError_t launch_hd_laplace(const HyperParams &h, const double *q, double *out, double scale, bool accumulate,
                             bool wallmask, hipStream_t s)
{
    switch (h.N) {
    case 1: hd_launch<1>(h, q, out, scale, accumulate, wallmask, s); break;
    case 2: hd_launch<2>(h, q, out, scale, accumulate, wallmask, s); break;
    case 3: hd_launch<3>(h, q, out, scale, accumulate, wallmask, s); break;
    case 4: hd_launch<4>(h, q, out, scale, accumulate, wallmask, s); break;
    case 5: hd_launch<5>(h, q, out, scale, accumulate, wallmask, s); break;
    case 6: hd_launch<6>(h, q, out, scale, accumulate, wallmask, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nh
