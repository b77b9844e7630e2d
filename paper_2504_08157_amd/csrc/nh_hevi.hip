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
// (unknown u on lane u mod 64), dot products are wave reductions, and a
// column never waits for another column.  For m = 10 (and 3 n_z <= 256) the
// Krylov basis lives in registers; otherwise in LDS.
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

// ---------------------------------------------------------------- GMRES, register basis
// The same restarted GMRES with the Krylov basis in registers: unknown u of
// the column sits in slot u / 64 of lane u mod 64 (S slots cover 64 S
// unknowns), and the loops over basis vectors are unrolled so that every
// basis access is a register.  LDS holds only the level tables, one vector
// for the lane exchange of L_v and the small Hessenberg data, so many more
// columns run per CU than with the basis in LDS.
template <int M, int S>
__global__ void __launch_bounds__(64) gmres_reg_kernel(HeviParams h, GmresArgs g)
{
    extern __shared__ double smem[];
    const int nz = h.nz, NU = 3 * nz, lane = threadIdx.x;
    const int NC = 2 * h.N + 1;
    double *slev = smem;                  // nz x kLevW
    double *sgz = slev + nz * kLevW;      // nz x NC
    double *xb = sgz + nz * NC;           // NU: the vector L_v is applied to
    double *tmp = xb + NU;                // 2 nz: rho0 w and p'_L
    double *H = tmp + 2 * nz;             // (M+1) x M
    double *cs = H + (M + 1) * M;         // M
    double *sn = cs + M;                  // M
    double *gv = sn + M;                  // M+1

    for (int i = lane; i < nz * kLevW; i += 64) slev[i] = h.lev[i];
    for (int i = lane; i < nz * NC; i += 64) sgz[i] = h.gz[i];
    __syncthreads();

    // y = (I - alpha L_v) x on register vectors (slot s: unknown lane + 64 s)
    auto apply = [&](const double *x, double *y) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int u = lane + 64 * s;
            if (u < NU) xb[u] = x[s];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int k = lane; k < nz; k += 64) {
            const double *L = slev + k * kLevW;
            tmp[k] = L[0] * xb[nz + k];
            tmp[nz + k] = h.gamma * L[2] * (xb[k] * L[7] + xb[2 * nz + k] * L[8]);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int u = lane + 64 * s;
            double r = 0.0;
            if (u < NU) {
                const int f = u / nz, k = u - f * nz;
                const double *L = slev + k * kLevW;
                double lv;
                if (f == 0) {
                    const double *G = sgz + k * NC;
                    double d = 0.0;
                    for (int o = -h.N; o <= h.N; ++o) {
                        const int kk = k + o;
                        if (kk >= 0 && kk < nz) d += G[o + h.N] * tmp[kk];
                    }
                    lv = -d;
                } else if (f == 1) {
                    if (k == 0 || k == nz - 1) {
                        lv = 0.0;
                    } else {
                        const double *G = sgz + k * NC;
                        double d = 0.0;
                        for (int o = -h.N; o <= h.N; ++o) {
                            const int kk = k + o;
                            if (kk >= 0 && kk < nz) d += G[o + h.N] * tmp[nz + kk];
                        }
                        lv = -d * L[7] - h.g * xb[k] * L[7];
                    }
                } else {
                    lv = -xb[nz + k] * L[3];
                }
                r = x[s] - g.alpha * lv;
            }
            y[s] = r;
        }
        // the exchange vector is rewritten by the next apply
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    auto dot = [&](const double *a, const double *c) __attribute__((always_inline)) {
        double d = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) d += a[s] * c[s];
        return wave_sum(d);
    };

    const long nxy = (long)h.nx * h.ny;
    const long U = nxy * nz;
    const int fld[3] = {0, 3, 4};
    for (long col = blockIdx.x; col < nxy; col += gridDim.x) {
        double bv[S], xs[S], V[M + 1][S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int u = lane + 64 * s;
            bv[s] = 0.0;
            xs[s] = 0.0;
            if (u < NU) {
                const int f = u / nz, k = u - f * nz;
                const long I = col + (long)k * nxy;
                bv[s] = g.b[fld[f] * U + I];
                xs[s] = g.x0 ? g.x0[f * U + I] : bv[s];
            }
        }
        const double bn = sqrt(dot(bv, bv));
        const double tol = g.rtol * bn;
        int iters = 0;
        bool conv = bn == 0.0;
        if (conv)
#pragma unroll
            for (int s = 0; s < S; ++s) xs[s] = 0.0;
        for (int rs = 0; rs <= g.max_restarts && !conv; ++rs) {
            apply(xs, V[0]);
#pragma unroll
            for (int s = 0; s < S; ++s) V[0][s] = bv[s] - V[0][s];
            const double rn = sqrt(dot(V[0], V[0]));
            if (rn <= tol) { conv = true; break; }
#pragma unroll
            for (int s = 0; s < S; ++s) V[0][s] /= rn;
            if (lane == 0) gv[0] = rn;
            int jn = 0;
            double res = rn;
            bool done = false;
            // fully unrolled (basis indices are registers): no early exit,
            // the remaining steps are skipped by a wave-uniform flag
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (!done) {
                    apply(V[j], V[j + 1]);
#pragma unroll
                    for (int i = 0; i <= j; ++i) {
                        const double d = dot(V[j + 1], V[i]);
#pragma unroll
                        for (int s = 0; s < S; ++s) V[j + 1][s] -= d * V[i][s];
                        if (lane == 0) H[i * M + j] = d;
                    }
                    const double nn = sqrt(dot(V[j + 1], V[j + 1]));
                    if (nn > 0.0)
#pragma unroll
                        for (int s = 0; s < S; ++s) V[j + 1][s] /= nn;
                    if (lane == 0) {
                        H[(j + 1) * M + j] = nn;
                        for (int i = 0; i < j; ++i) {
                            const double a = H[i * M + j], bb = H[(i + 1) * M + j];
                            H[i * M + j] = cs[i] * a + sn[i] * bb;
                            H[(i + 1) * M + j] = -sn[i] * a + cs[i] * bb;
                        }
                        const double a = H[j * M + j], bb = H[(j + 1) * M + j];
                        const double r = sqrt(a * a + bb * bb);
                        const double c = r > 0.0 ? a / r : 1.0, sg = r > 0.0 ? bb / r : 0.0;
                        cs[j] = c;
                        sn[j] = sg;
                        H[j * M + j] = r;
                        H[(j + 1) * M + j] = 0.0;
                        gv[j + 1] = -sg * gv[j];
                        gv[j] = c * gv[j];
                    }
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    res = fabs(gv[j + 1]);
                    ++iters;
                    jn = j + 1;
                    done = res <= tol || nn == 0.0;
                }
            }
            // back substitution y = H^-1 g (lane 0), x += V y
            if (lane == 0) {
                for (int i = jn - 1; i >= 0; --i) {
                    double sacc = gv[i];
                    for (int l = i + 1; l < jn; ++l) sacc -= H[i * M + l] * gv[l];
                    gv[i] = sacc / H[i * M + i];
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (i < jn) {
                    const double yi = gv[i];
#pragma unroll
                    for (int s = 0; s < S; ++s) xs[s] += yi * V[i][s];
                }
            }
            if (res <= tol) {
                // confirm with the true residual
                double t[S];
                apply(xs, t);
#pragma unroll
                for (int s = 0; s < S; ++s) t[s] = bv[s] - t[s];
                conv = sqrt(dot(t, t)) <= tol;
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int u = lane + 64 * s;
            if (u < NU) {
                const int f = u / nz, k = u - f * nz;
                g.x[fld[f] * U + col + (long)k * nxy] = xs[s];
            }
        }
        for (int k = lane; k < nz; k += 64) {
            const long I = col + (long)k * nxy;
            g.x[U + I] = g.b[U + I];
            g.x[2 * U + I] = g.b[2 * U + I];
        }
        if (lane == 0 && g.iters) g.iters[col] = conv ? iters : -iters - 1;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
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
    if (g.restart == kGmresRegM && 3 * h.nz <= 64 * kGmresRegSlots) {
        // register basis: LDS for the level tables, the exchange vector and
        // the Hessenberg data only
        const size_t lds = sizeof(double) * ((size_t)h.nz * kLevW + (size_t)h.nz * (2 * h.N + 1) + 3 * h.nz +
                                             2 * h.nz + (kGmresRegM + 1) * kGmresRegM + 2 * kGmresRegM +
                                             kGmresRegM + 1);
        const int grid = (int)(ncol < 32768 ? ncol : 32768);
        hipLaunchKernelGGL((gmres_reg_kernel<kGmresRegM, kGmresRegSlots>), dim3(grid), dim3(64), lds, s, h, g);
        return hipGetLastError();
    }
    const size_t lds = gmres_lds_bytes(h.nz, h.N, g.restart);
    const int grid = (int)(ncol < 8192 ? ncol : 8192);
    hipLaunchKernelGGL(gmres_column_kernel, dim3(grid), dim3(64), lds, s, h, g);
    return hipGetLastError();
}

}  // namespace nh
