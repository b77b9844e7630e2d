// gfx950 kernels of the 1D-IMEX (HEVI) time step: the vertical linear
// operator L_v, the ARK2 stage combinations, and a batched matrix-free GMRES
// that solves (I - alpha L_v) x = b independently in every lattice column.
//
// The IMEX split of Sec. 2.3 treats the fast waves implicitly; in the HEVI
// form only their vertical part is implicit.  L_v is the linearisation of S
// about the resting hydrostatic reference restricted to z-derivatives:
//   (L_v x)_rho'   = - d/dz (rho0 w)
//   (L_v x)_w      = - (1/rho0) d/dz p'_L - g rho'/rho0,   p'_L = gamma p0 (rho'/rho0 + theta'/theta0)
//   (L_v x)_theta' = - w d(theta0)/dz
//   (L_v x)_u = (L_v x)_v = 0,
// with the same DSS'd vertical derivative as the right-hand side (the
// mass-weighted average of the one-sided element derivatives, a (2N+1)-point
// stencil per level) and the w-rows zero at z = 0 and z = H.  It couples only
// the nodes of one column and its coefficients depend on z alone.
//
// GMRES (Sec. 2.3: matrix-free, fewer than 20 Krylov vectors): restarted
// GMRES(m), modified Gram-Schmidt, Givens rotations, stopping when the
// residual estimate satisfies ||b - A x|| <= rtol ||b||.  One wavefront owns
// one column: the column's 3 n_z unknowns are spread over the 64 lanes
// (unknown u on lane u mod 64), the Krylov basis lives in LDS, dot products
// are wave reductions.  A column never waits for another column.
#include "nh_internal.h"

#include <math.h>

namespace nh {

// ---------------------------------------------------------------- L_v on a state
// y = L_v x on [5][U]; one thread per node, z-neighbours read along the
// column (stride n_x n_y), coalesced along x.
__global__ void lv_apply_kernel(HeviParams h, const double *__restrict__ x, double *__restrict__ y)
{
    const long nxy = (long)h.nx * h.ny;
    const long U = nxy * h.nz;
    const int NC = 2 * h.N + 1;
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < U; I += (long)gridDim.x * blockDim.x) {
        const int k = (int)(I / nxy);
        const double *L = h.lev + (long)k * kLevW;
        const double *G = h.gz + (long)k * NC;
        double d_rw = 0.0, d_pl = 0.0;
        for (int o = -h.N; o <= h.N; ++o) {
            const int kk = k + o;
            if (kk < 0 || kk >= h.nz) continue;
            const double c = G[o + h.N];
            if (c == 0.0) continue;
            const double *Lk = h.lev + (long)kk * kLevW;
            const long J = I + (long)o * nxy;
            d_rw += c * (Lk[0] * x[3 * U + J]);
            d_pl += c * (h.gamma * Lk[2] * (x[J] * Lk[7] + x[4 * U + J] * Lk[8]));
        }
        const double rp = x[I], w = x[3 * U + I];
        y[I] = -d_rw;
        y[U + I] = 0.0;
        y[2 * U + I] = 0.0;
        y[3 * U + I] = (k == 0 || k == h.nz - 1) ? 0.0 : -d_pl * L[7] - h.g * rp * L[7];
        y[4 * U + I] = -w * L[3];
    }
}

// ---------------------------------------------------------------- combinations
// out = base + sum_j c[j] * src[j] (j < nsrc), elementwise on [5][U].
__global__ void axpy_multi_kernel(long n, const double *__restrict__ base, int nsrc, LinComb lc,
                                  double *__restrict__ out)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double r = base[i];
        for (int j = 0; j < nsrc; ++j) r += lc.c[j] * lc.src[j][i];
        out[i] = r;
    }
}

// ---------------------------------------------------------------- GMRES
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// y = (I - alpha L_v) x for one column, x and y in LDS (field-major
// [rho'(z), w(z), theta'(z)]), tmp: 2 n_z scratch for rho0 w and p'_L.
__device__ void column_apply(const HeviParams &h, double alpha, const double *x, double *y, double *tmp,
                             const double *slev, const double *sgz)
{
    const int nz = h.nz, lane = threadIdx.x, NC = 2 * h.N + 1;
    for (int k = lane; k < nz; k += 64) {
        const double *L = slev + k * kLevW;
        tmp[k] = L[0] * x[nz + k];
        tmp[nz + k] = h.gamma * L[2] * (x[k] * L[7] + x[2 * nz + k] * L[8]);
    }
    __syncthreads();
    for (int k = lane; k < nz; k += 64) {
        const double *L = slev + k * kLevW;
        const double *G = sgz + k * NC;
        double d_rw = 0.0, d_pl = 0.0;
        for (int o = -h.N; o <= h.N; ++o) {
            const int kk = k + o;
            if (kk < 0 || kk >= nz) continue;
            d_rw += G[o + h.N] * tmp[kk];
            d_pl += G[o + h.N] * tmp[nz + kk];
        }
        const double lr = -d_rw;
        const double lw = (k == 0 || k == nz - 1) ? 0.0 : -d_pl * L[7] - h.g * x[k] * L[7];
        const double lt = -x[nz + k] * L[3];
        y[k] = x[k] - alpha * lr;
        y[nz + k] = x[nz + k] - alpha * lw;
        y[2 * nz + k] = x[2 * nz + k] - alpha * lt;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(64) gmres_column_kernel(HeviParams h, GmresArgs g)
{
    extern __shared__ double smem[];
    const int nz = h.nz, NU = 3 * nz, m = g.restart, lane = threadIdx.x;
    const int NC = 2 * h.N + 1;
    double *V = smem;                       // (m+1) x NU Krylov basis
    double *w = V + (size_t)(m + 1) * NU;   // NU
    double *xs = w + NU;                    // NU current iterate
    double *tmp = xs + NU;                  // 2 nz
    double *H = tmp + 2 * nz;               // (m+1) x m Hessenberg
    double *cs = H + (m + 1) * m;           // m
    double *sn = cs + m;                    // m
    double *gv = sn + m;                    // m+1
    double *slev = gv + (m + 1);            // nz x kLevW
    double *sgz = slev + nz * kLevW;        // nz x NC

    for (int i = lane; i < nz * kLevW; i += 64) slev[i] = h.lev[i];
    for (int i = lane; i < nz * NC; i += 64) sgz[i] = h.gz[i];

    const long nxy = (long)h.nx * h.ny;
    const long U = nxy * nz;
    const int fld[3] = {0, 3, 4};
    for (long col = blockIdx.x; col < nxy; col += gridDim.x) {
        // load b (into w) and the initial guess (into xs)
        for (int u = lane; u < NU; u += 64) {
            const int f = u / nz, k = u % nz;
            const long I = col + (long)k * nxy;
            w[u] = g.b[fld[f] * U + I];
            xs[u] = g.x0 ? g.x0[f * U + I] : w[u];
        }
        __syncthreads();
        double bn = 0.0;
        for (int u = lane; u < NU; u += 64) bn += w[u] * w[u];
        bn = sqrt(wave_sum(bn));
        const double tol = g.rtol * bn;
        int iters = 0;
        bool conv = bn == 0.0;
        if (conv)
            for (int u = lane; u < NU; u += 64) xs[u] = 0.0;
        for (int rs = 0; rs <= g.max_restarts && !conv; ++rs) {
            // r = b - A x  ->  V[0]
            column_apply(h, g.alpha, xs, V, tmp, slev, sgz);
            double rn = 0.0;
            for (int u = lane; u < NU; u += 64) {
                const double r = w[u] - V[u];
                V[u] = r;
                rn += r * r;
            }
            rn = sqrt(wave_sum(rn));
            if (rn <= tol) { conv = true; break; }
            for (int u = lane; u < NU; u += 64) V[u] /= rn;
            if (lane == 0) gv[0] = rn;
            __syncthreads();
            int j = 0;
            double res = rn;
            for (; j < m; ++j) {
                double *vj1 = V + (size_t)(j + 1) * NU;
                column_apply(h, g.alpha, V + (size_t)j * NU, vj1, tmp, slev, sgz);
                // modified Gram-Schmidt
                for (int i = 0; i <= j; ++i) {
                    const double *vi = V + (size_t)i * NU;
                    double d = 0.0;
                    for (int u = lane; u < NU; u += 64) d += vj1[u] * vi[u];
                    d = wave_sum(d);
                    for (int u = lane; u < NU; u += 64) vj1[u] -= d * vi[u];
                    if (lane == 0) H[i * m + j] = d;
                }
                double nn = 0.0;
                for (int u = lane; u < NU; u += 64) nn += vj1[u] * vj1[u];
                nn = sqrt(wave_sum(nn));
                if (lane == 0) H[(j + 1) * m + j] = nn;
                if (nn > 0.0)
                    for (int u = lane; u < NU; u += 64) vj1[u] /= nn;
                __syncthreads();
                // Givens rotations on column j of H (every lane keeps the same copy)
                if (lane == 0) {
                    for (int i = 0; i < j; ++i) {
                        const double a = H[i * m + j], bb = H[(i + 1) * m + j];
                        H[i * m + j] = cs[i] * a + sn[i] * bb;
                        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
                    }
                    const double a = H[j * m + j], bb = H[(j + 1) * m + j];
                    const double r = sqrt(a * a + bb * bb);
                    const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? bb / r : 0.0;
                    cs[j] = c;
                    sn[j] = s;
                    H[j * m + j] = r;
                    H[(j + 1) * m + j] = 0.0;
                    gv[j + 1] = -s * gv[j];
                    gv[j] = c * gv[j];
                }
                __syncthreads();
                res = fabs(gv[j + 1]);
                ++iters;
                if (res <= tol || nn == 0.0) { ++j; break; }
            }
            // back substitution y = H^-1 g (lane 0), x += V y
            if (lane == 0) {
                for (int i = j - 1; i >= 0; --i) {
                    double s = gv[i];
                    for (int l = i + 1; l < j; ++l) s -= H[i * m + l] * gv[l];
                    gv[i] = s / H[i * m + i];
                }
            }
            __syncthreads();
            for (int u = lane; u < NU; u += 64) {
                double acc = xs[u];
                for (int i = 0; i < j; ++i) acc += gv[i] * V[(size_t)i * NU + u];
                xs[u] = acc;
            }
            __syncthreads();
            if (res <= tol) {
                // confirm with the true residual
                column_apply(h, g.alpha, xs, V, tmp, slev, sgz);
                double tn = 0.0;
                for (int u = lane; u < NU; u += 64) {
                    const double r = w[u] - V[u];
                    tn += r * r;
                }
                tn = sqrt(wave_sum(tn));
                conv = tn <= tol;
            }
        }
        for (int u = lane; u < NU; u += 64) {
            const int f = u / nz, k = u % nz;
            const long I = col + (long)k * nxy;
            g.x[fld[f] * U + I] = xs[u];
        }
        // u and v rows of (I - alpha L_v) are the identity
        for (int k = lane; k < nz; k += 64) {
            const long I = col + (long)k * nxy;
            g.x[U + I] = g.b[U + I];
            g.x[2 * U + I] = g.b[2 * U + I];
        }
        if (lane == 0) {
            if (g.iters) g.iters[col] = conv ? iters : -iters - 1;
        }
        __syncthreads();
    }
}

static int grid_for(long n, int block)
{
    long gsz = (n + block - 1) / block;
    if (gsz > 65535) gsz = 65535;
    if (gsz < 1) gsz = 1;
    return (int)gsz;
}

size_t gmres_lds_bytes(int nz, int N, int restart)
{
    const int NU = 3 * nz, m = restart;
    const size_t n = (size_t)(m + 1) * NU + 2 * (size_t)NU + 2 * nz + (m + 1) * m + 2 * m + (m + 1) +
                     (size_t)nz * kLevW + (size_t)nz * (2 * N + 1);
    return n * sizeof(double);
}

hipError_t launch_lv_apply(const HeviParams &h, const double *x, double *y, hipStream_t s)
{
    const long U = (long)h.nx * h.ny * h.nz;
    hipLaunchKernelGGL(lv_apply_kernel, dim3(grid_for(U, 256)), dim3(256), 0, s, h, x, y);
    return hipGetLastError();
}

hipError_t launch_axpy_multi(long n, const double *base, int nsrc, const LinComb &lc, double *out,
                             hipStream_t s)
{
    hipLaunchKernelGGL(axpy_multi_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, base, nsrc, lc, out);
    return hipGetLastError();
}

hipError_t launch_gmres(const HeviParams &h, const GmresArgs &g, hipStream_t s)
{
    const long ncol = (long)h.nx * h.ny;
    const size_t lds = gmres_lds_bytes(h.nz, h.N, g.restart);
    const int grid = (int)(ncol < 8192 ? ncol : 8192);
    hipLaunchKernelGGL(gmres_column_kernel, dim3(grid), dim3(64), lds, s, h, g);
    return hipGetLastError();
}

}  // namespace nh
