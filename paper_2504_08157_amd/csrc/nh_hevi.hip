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

#include <utility>

namespace nh {

// ---------------------------------------------------------------- L_v on a state
// y = L_v x on [5][U].  One thread per lattice column walks up the levels
// (lv_walk: the (2N+1)-level window of the two stencil inputs rho0 w and
// p'_L in registers), so every value of x is read once and every value of y
// written once, coalesced along x.  Level data and stencil rows are
// wave-uniform.  With uv false the (zero) u and v rows are not written.
// Residual form (RESID): x holds (rho', w, theta') as [3][U] and the
// kernel writes the residual of (I - alpha L_v) x = b,
// y = b - x + alpha L_v x, in fields 0, 3, 4 of [5][U] (b also [5][U]).
template <int N, bool RESID>
__global__ void __launch_bounds__(256) lv_apply_kernel(HeviParams h, const double *__restrict__ x,
                                                       double *__restrict__ y, bool uv, double alpha,
                                                       const double *__restrict__ b)
{
    const long nxy = (long)h.nx * h.ny;
    const long col = blockIdx.x * 256L + threadIdx.x;
    if (col >= nxy) return;
    const long U = nxy * h.nz;
    lv_walk<N>(h, col, 0, h.nz, x, RESID ? U : 3 * U, RESID ? 2 * U : 4 * U,
               [&](int k, double l0, double l3, double l4, double xr, double xw, double xt) {
                   const long I = col + (long)k * nxy;
                   if constexpr (RESID) {
                       y[I] = b[I] - xr + alpha * l0;
                       y[3 * U + I] = b[3 * U + I] - xw + alpha * l3;
                       y[4 * U + I] = b[4 * U + I] - xt + alpha * l4;
                   } else {
                       y[I] = l0;
                       if (uv) {
                           y[U + I] = 0.0;
                           y[2 * U + I] = 0.0;
                       }
                       y[3 * U + I] = l3;
                       y[4 * U + I] = l4;
                   }
               });
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
    if (g.gate && *g.gate == 0) return;
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
// Wave-wide sums in registers (no LDS traffic): gfx950 lane swaps between
// register pairs and DPP butterflies inside 16-lane rows.

// DPP lane move with every source lane valid.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double join_d(unsigned lo, unsigned hi)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// gfx950 lane swaps between two registers (one 16-lane row is a "row"):
// swap32: a <- [a lanes 0-31, b lanes 0-31], b <- [a lanes 32-63, b lanes 32-63]
// swap16: a <- [a row 0, b row 0, a row 2, b row 2], b <- [a row 1, b row 1, a row 3, b row 3]
__device__ __forceinline__ void swap32(double &a, double &b)
{
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = join_d(lo[0], hi[0]);
    b = join_d(lo[1], hi[1]);
}

__device__ __forceinline__ void swap16(double &a, double &b)
{
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = join_d(lo[0], hi[0]);
    b = join_d(lo[1], hi[1]);
}

// every lane of each 16-lane row <- the sum over its row
__device__ __forceinline__ double row_sum(double v)
{
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return v;
}

template <int L>
__device__ __forceinline__ double lane_value(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return join_d((unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, L),
                  (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), L));
}

template <class F, int... J>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, J...>)
{
    (f(std::integral_constant<int, J>{}), ...);
}

// f(integral_constant<int, j>) for j = 0 .. n-1, in order
template <int n, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, n>{});
}

// v[i] <- sum over the wave of v[i] for i < CNT, four sums at a time: the
// halves and then the rows of the four registers are exchanged and added
// (each register then carries one sum per row), one row reduction follows,
// and each sum is read from its row.  Fixed order of additions.
template <int CNT, int K>
__device__ __forceinline__ void wave_sum_t(double (&v)[K])
{
    static_for<(CNT + 3) / 4>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = 4 * decltype(qc)::value;
        double a = v[q], b = 0.0, c = 0.0, d = 0.0;
        if constexpr (q + 1 < CNT) b = v[q + 1];
        if constexpr (q + 2 < CNT) c = v[q + 2];
        if constexpr (q + 3 < CNT) d = v[q + 3];
        swap32(a, b);
        swap32(c, d);
        double p = a + b, r = c + d;   // lanes 0-31: sums q, q+2; lanes 32-63: q+1, q+3
        swap16(p, r);
        const double t = row_sum(p + r);   // rows 0..3: sums q, q+2, q+1, q+3
        v[q] = lane_value<0>(t);
        if constexpr (q + 1 < CNT) v[q + 1] = lane_value<32>(t);
        if constexpr (q + 2 < CNT) v[q + 2] = lane_value<16>(t);
        if constexpr (q + 3 < CNT) v[q + 3] = lane_value<48>(t);
    });
}

// one sum, left in every lane
__device__ __forceinline__ double wave_sum1(double v)
{
    double a = v, b = v;
    swap32(a, b);
    double p = a + b, r = p;
    swap16(p, r);
    return row_sum(p + r);
}
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// The same restarted GMRES with the Krylov basis in registers: unknown u of
// the column sits in slot u / 64 of lane u mod 64 (S slots cover 64 S
// unknowns) and the loops over basis vectors are unrolled, so every basis
// access is a register.  Orthogonalisation is classical Gram-Schmidt with a
// re-orthogonalisation test in the manner of Daniel, Gragg, Kaufman and
// Stewart (1976): the dot products and |w|^2 are reduced together in one
// round, the new norm follows from Pythagoras, and a second pass runs only
// where the projection kept less than 1 % of |w| (one reduction round per
// step instead of one per basis vector; the restart length of 10 keeps the
// accumulated loss of orthogonality near 1e-13).  The Arnoldi process runs on L_v itself, which
// spans the same Krylov space as A = I - alpha L_v (H_A = I - alpha H_L) but
// without the identity part that the projection would cancel every step.
// The Hessenberg column is rotated in registers on every lane; lane 0 keeps
// the triangular factor and the rotations in LDS for the back substitution.
// LDS holds the level coefficients, the lane exchange of L_v, b and x.
template <int M, int S>
__global__ void __launch_bounds__(64) gmres_reg_kernel(HeviParams h, GmresArgs g)
{
    if (g.gate && *g.gate == 0) return;
    extern __shared__ double smem[];
    const int nz = h.nz, NU = 3 * nz, N = h.N, NC = 2 * N + 1, lane = threadIdx.x;
    const int NP = nz + 2 * N;            // padded length of the L_v intermediates
    double *slc = smem;                   // nz x 5: rho0, p0, d theta0/dz, 1/rho0, 1/theta0
    double *sgz = slc + nz * 5;           // nz x NC
    double *xb = sgz + nz * NC;           // NU: the vector L_v is applied to
    double *tp = xb + NU;                 // 2 NP: rho0 w and p'_L, N zeros on both ends
    double *sb = tp + 2 * NP;             // NU: right-hand side
    double *sx = sb + NU;                 // NU: iterate
    double *R = sx + NU;                  // M x M triangular factor, R[i M + j]
    double *cs = R + M * M;               // M
    double *sn = cs + M;                  // M
    double *gv = sn + M;                  // M: rotated residual

    for (int k = lane; k < nz; k += 64) {
        const double *L = h.lev + k * kLevW;
        slc[k * 5 + 0] = L[0];
        slc[k * 5 + 1] = L[2];
        slc[k * 5 + 2] = L[3];
        slc[k * 5 + 3] = L[7];
        slc[k * 5 + 4] = L[8];
    }
    for (int i = lane; i < nz * NC; i += 64) sgz[i] = h.gz[i];
    for (int i = lane; i < 2 * NP; i += 64) tp[i] = 0.0;
    __syncthreads();

    // slot s of this lane: field sf (0 rho', 1 w, 2 theta', 3 unused), level sk
    int sf[S], sk[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int u = lane + 64 * s;
        sf[s] = u < NU ? u / nz : 3;
        sk[s] = u < NU ? u - sf[s] * nz : 0;
    }

    // y = L_v x on register vectors
    auto apply = [&](const double (&x)[S], double (&y)[S]) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (sf[s] < 3) xb[lane + 64 * s] = x[s];
        wave_sync();
        for (int k = lane; k < nz; k += 64) {
            const double *L = slc + k * 5;
            tp[N + k] = L[0] * xb[nz + k];
            tp[NP + N + k] = h.gamma * L[1] * (xb[k] * L[3] + xb[2 * nz + k] * L[4]);
        }
        wave_sync();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int f = sf[s], k = sk[s];
            const double *L = slc + k * 5;
            double lv = 0.0;
            if (f == 0 || (f == 1 && k > 0 && k < nz - 1)) {
                const double *G = sgz + k * NC;
                const double *T = tp + (f == 0 ? 0 : NP) + k;
                double d = 0.0;
                for (int o = 0; o < NC; ++o) d += G[o] * T[o];
                lv = f == 0 ? -d : -d * L[3] - h.g * xb[k] * L[3];
            } else if (f == 2) {
                lv = -xb[nz + k] * L[2];
            }
            y[s] = lv;
        }
        // the exchange vectors are rewritten by the next apply
        wave_sync();
    };

    const long nxy = (long)h.nx * h.ny;
    const long U = nxy * nz;
    // offset of slot s's node in b and x (fields rho', w, theta' are state
    // fields 0, 3, 4) and in x0 ([3][U])
    auto ob = [&](int s) { return (sf[s] == 0 ? 0 : sf[s] == 1 ? 3 * U : 4 * U) + (long)sk[s] * nxy; };
    auto o0 = [&](int s) { return sf[s] * U + (long)sk[s] * nxy; };
    for (long col = blockIdx.x; col < nxy; col += gridDim.x) {
        double bn2 = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (sf[s] < 3) {
                const double bb = g.b[ob(s) + col];
                sb[lane + 64 * s] = bb;
                sx[lane + 64 * s] = g.x0 ? g.x0[o0(s) + col] : bb;
                bn2 += bb * bb;
            }
        }
        const double bn = sqrt(wave_sum1(bn2));
        const double tol = g.rtol * bn;
        int iters = 0;
        bool conv = bn == 0.0;
        if (conv)
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (sf[s] < 3) sx[lane + 64 * s] = 0.0;
        // guess choice: the residual norm of the default start x = b, to be
        // compared with that of the given guess at the first restart
        bool choose = g.pick && g.x0 && !conv;
        double rdef = 0.0;
        if (choose) {
            double t[S], y[S];
#pragma unroll
            for (int s = 0; s < S; ++s) t[s] = sf[s] < 3 ? sb[lane + 64 * s] : 0.0;
            apply(t, y);
            double r2 = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double r = sf[s] < 3 ? sb[lane + 64 * s] - (t[s] - g.alpha * y[s]) : 0.0;
                r2 += r * r;
            }
            rdef = sqrt(wave_sum1(r2));
        }
        for (int rs = 0; rs <= g.max_restarts && !conv; ++rs) {
            double V[M + 1][S];
            {
                double t[S];
#pragma unroll
                for (int s = 0; s < S; ++s) t[s] = sf[s] < 3 ? sx[lane + 64 * s] : 0.0;
                apply(t, V[0]);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    V[0][s] = sf[s] < 3 ? sb[lane + 64 * s] - (t[s] - g.alpha * V[0][s]) : 0.0;
            }
            double rn2 = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) rn2 += V[0][s] * V[0][s];
            const double rn = sqrt(wave_sum1(rn2));
            if (choose) {
                // keep the guess with the smaller residual: start again
                // from x = b if the given one is worse
                choose = false;
                if (rdef < rn) {
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (sf[s] < 3) sx[lane + 64 * s] = sb[lane + 64 * s];
                    --rs;
                    continue;
                }
            }
            if (rn <= tol) { conv = true; break; }
            {
                const double inv = 1.0 / rn;
#pragma unroll
                for (int s = 0; s < S; ++s) V[0][s] *= inv;
            }
            double gj = rn, res = rn;
            int jn = 0;
            bool done = false;
            // one instance per step (basis indices are registers): no early
            // exit, the remaining steps are skipped by a wave-uniform flag
            static_for<M>([&](auto jc) __attribute__((always_inline)) {
                constexpr int j = decltype(jc)::value;
                if (!done) {
                    apply(V[j], V[j + 1]);
                    // Gram-Schmidt: the dots with V_0..V_j and |w|^2 in one
                    // batched reduction; |w - V h| from Pythagoras unless the
                    // projection kept less than 1 % of |w| (the new vector's
                    // loss of orthogonality is then above ~100 eps), in
                    // which case the pass is repeated and the norm taken
                    // directly
                    double hc[M + 2];
#pragma unroll
                    for (int i = 0; i <= M + 1; ++i) {
                        hc[i] = 0.0;
                        if (i <= j)
#pragma unroll
                            for (int s = 0; s < S; ++s) hc[i] += V[j + 1][s] * V[i][s];
                        if (i == j + 1)
#pragma unroll
                            for (int s = 0; s < S; ++s) hc[i] += V[j + 1][s] * V[j + 1][s];
                    }
                    wave_sum_t<j + 2>(hc);
                    const double w2 = hc[j + 1];
                    double p2 = 0.0;
#pragma unroll
                    for (int i = 0; i <= j; ++i) {
                        p2 += hc[i] * hc[i];
#pragma unroll
                        for (int s = 0; s < S; ++s) V[j + 1][s] -= hc[i] * V[i][s];
                    }
                    double nn2 = w2 - p2;
                    if (nn2 < 1e-4 * w2) {
                        double e[M + 1];
#pragma unroll
                        for (int i = 0; i <= M; ++i) {
                            e[i] = 0.0;
                            if (i <= j)
#pragma unroll
                                for (int s = 0; s < S; ++s) e[i] += V[j + 1][s] * V[i][s];
                        }
                        wave_sum_t<j + 1>(e);
#pragma unroll
                        for (int i = 0; i <= j; ++i) {
#pragma unroll
                            for (int s = 0; s < S; ++s) V[j + 1][s] -= e[i] * V[i][s];
                            hc[i] += e[i];
                        }
                        double t2 = 0.0;
#pragma unroll
                        for (int s = 0; s < S; ++s) t2 += V[j + 1][s] * V[j + 1][s];
                        nn2 = wave_sum1(t2);
                    }
                    const double nn = sqrt(nn2);
                    if (nn > 0.0) {
                        const double inv = 1.0 / nn;
#pragma unroll
                        for (int s = 0; s < S; ++s) V[j + 1][s] *= inv;
                    }
                    // column j of the Hessenberg matrix of A = I - alpha L_v
                    // from that of L_v, the earlier rotations, the new one
#pragma unroll
                    for (int i = 0; i <= j; ++i) hc[i] = (i == j ? 1.0 : 0.0) - g.alpha * hc[i];
                    const double sub = -g.alpha * nn;
#pragma unroll
                    for (int i = 0; i < j; ++i) {
                        const double c = cs[i], sg = sn[i], a = hc[i], bb = hc[i + 1];
                        hc[i] = c * a + sg * bb;
                        hc[i + 1] = -sg * a + c * bb;
                    }
                    const double a = hc[j];
                    const double r = sqrt(a * a + sub * sub);
                    const double c = r > 0.0 ? a / r : 1.0, sg = r > 0.0 ? sub / r : 0.0;
                    if (lane == 0) {
#pragma unroll
                        for (int i = 0; i < j; ++i) R[i * M + j] = hc[i];
                        R[j * M + j] = r;
                        cs[j] = c;
                        sn[j] = sg;
                        gv[j] = c * gj;
                    }
                    wave_sync();
                    gj = -sg * gj;
                    res = fabs(gj);
                    ++iters;
                    jn = j + 1;
                    done = res <= tol || nn == 0.0;
                }
            });
            // back substitution y = R^-1 g on every lane, x += V y
            double y[M];
#pragma unroll
            for (int i = M - 1; i >= 0; --i) {
                y[i] = 0.0;
                if (i < jn) {
                    double acc = gv[i];
#pragma unroll
                    for (int l = i + 1; l < M; ++l)
                        if (l < jn) acc -= R[i * M + l] * y[l];
                    y[i] = acc / R[i * M + i];
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (sf[s] < 3) {
                    double acc = sx[lane + 64 * s];
#pragma unroll
                    for (int i = 0; i < M; ++i) acc += y[i] * V[i][s];
                    sx[lane + 64 * s] = acc;
                }
            }
            if (res <= tol) {
                // confirm with the true residual
                double t[S], w[S];
#pragma unroll
                for (int s = 0; s < S; ++s) t[s] = sf[s] < 3 ? sx[lane + 64 * s] : 0.0;
                apply(t, w);
                double tn2 = 0.0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const double d = sf[s] < 3 ? sb[lane + 64 * s] - (t[s] - g.alpha * w[s]) : 0.0;
                    tn2 += d * d;
                }
                conv = sqrt(wave_sum1(tn2)) <= tol;
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (sf[s] < 3) g.x[ob(s) + col] = sx[lane + 64 * s];
        for (int k = lane; k < nz; k += 64) {
            const long I = col + (long)k * nxy;
            g.x[U + I] = g.b[U + I];
            g.x[2 * U + I] = g.b[2 * U + I];
        }
        if (lane == 0 && g.iters) g.iters[col] = conv ? iters : -iters - 1;
        wave_sync();
    }
}

// ---------------------------------------------------------------- GMRES, Schur form
// The same column system solved through its Schur complement in w.  With
// (I - alpha L_v) x = b written per field, the rho' and theta' rows give
// rho' = b_rho + alpha L_rw w and theta' = b_th + alpha L_tw w
// (L_rw w = -d/dz (rho0 w), L_tw w = -w d theta0/dz), so the interior w rows
// become (I - alpha^2 M) w = b_w + alpha L_w(b_rho + alpha L_rw w_wall,
// b_th + alpha L_tw w_wall) with M w = L_w(L_rw w, L_tw w) and L_w the w row
// of L_v acting on (rho', theta'); the wall values of w are b_w (their rows
// of L_v are zero).  GMRES runs on the n_z - 2 interior w values (Arnoldi on
// M, H = I - alpha^2 H_M), one register slot per 64 of them.  The full-system
// residual of the reconstructed (rho', w, theta') is the Schur residual on
// the interior w rows and zero elsewhere, so the stopping test
// ||b - A x|| <= rtol ||b|| is the same as for the full form (||b|| over
// all 3 n_z unknowns).
template <int M, int S>
__global__ void __launch_bounds__(64) gmres_schur_kernel(HeviParams h, GmresArgs g)
{
    if (g.gate && *g.gate == 0) return;
    extern __shared__ double smem[];
    const int nz = h.nz, N = h.N, NC = 2 * N + 1, lane = threadIdx.x;
    const int NP = nz + 2 * N;
    double *slc = smem;                   // nz x 5: rho0, p0, d theta0/dz, 1/rho0, 1/theta0
    double *sgz = slc + nz * 5;           // nz x NC
    double *ww = sgz + nz * NC;           // nz: w at every level
    double *tp = ww + nz;                 // 2 NP: rho0 w and p'_L, N zeros on both ends
    double *rt = tp + 2 * NP;             // nz: rho' component
    double *tt = rt + nz;                 // nz: theta' component
    double *br = tt + nz;                 // nz: b_rho
    double *bt = br + nz;                 // nz: b_theta
    double *bw = bt + nz;                 // nz: b_w
    double *sb = bw + nz;                 // 64 S: reduced right-hand side
    double *sx = sb + 64 * S;             // 64 S: iterate
    double *R = sx + 64 * S;              // M x M triangular factor
    double *cs = R + M * M;
    double *sn = cs + M;
    double *gv = sn + M;

    for (int k = lane; k < nz; k += 64) {
        const double *L = h.lev + k * kLevW;
        slc[k * 5 + 0] = L[0];
        slc[k * 5 + 1] = L[2];
        slc[k * 5 + 2] = L[3];
        slc[k * 5 + 3] = L[7];
        slc[k * 5 + 4] = L[8];
    }
    for (int i = lane; i < nz * NC; i += 64) sgz[i] = h.gz[i];
    for (int i = lane; i < 2 * NP; i += 64) tp[i] = 0.0;
    __syncthreads();

    // slot s of this lane holds interior level sk (1 .. nz-2), or nothing (0)
    int sk[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = 1 + lane + 64 * s;
        sk[s] = k <= nz - 2 ? k : 0;
    }
    const double beta = g.alpha * g.alpha;

    // From ww (w at every level): rt = rb + c L_rw ww, tt = tb + c L_tw ww at
    // every level (rb, tb may be null), and, if y is given, y[s] = L_w(rt, tt)
    // at the lane's interior levels.
    auto chain = [&](double c, const double *rb, const double *tb, double (*y)[S]) __attribute__((always_inline)) {
        for (int k = lane; k < nz; k += 64) tp[N + k] = slc[k * 5] * ww[k];
        wave_sync();
        for (int k = lane; k < nz; k += 64) {
            const double *L = slc + k * 5;
            const double *G = sgz + k * NC;
            const double *T = tp + k;
            double d = 0.0;
            for (int o = 0; o < NC; ++o) d += G[o] * T[o];
            const double r = (rb ? rb[k] : 0.0) - c * d;
            const double th = (tb ? tb[k] : 0.0) - c * ww[k] * L[2];
            rt[k] = r;
            tt[k] = th;
            tp[NP + N + k] = h.gamma * L[1] * (r * L[3] + th * L[4]);
        }
        wave_sync();
        if (y) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = sk[s];
                double v = 0.0;
                if (k > 0) {
                    const double *G = sgz + k * NC;
                    const double *T = tp + NP + k;
                    double d = 0.0;
                    for (int o = 0; o < NC; ++o) d += G[o] * T[o];
                    v = -d * slc[k * 5 + 3] - h.g * rt[k] * slc[k * 5 + 3];
                }
                (*y)[s] = v;
            }
        }
        // the exchange arrays are rewritten by the next call
        wave_sync();
    };
    // y = M x for interior vectors x in registers (walls zero)
    auto apply = [&](const double (&x)[S], double (&y)[S]) __attribute__((always_inline)) {
        for (int k = lane; k < nz; k += 64)
            if (k == 0 || k == nz - 1) ww[k] = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (sk[s] > 0) ww[sk[s]] = x[s];
        wave_sync();
        chain(1.0, nullptr, nullptr, &y);
    };

    const long nxy = (long)h.nx * h.ny;
    const long U = nxy * nz;
    for (long col = blockIdx.x; col < nxy; col += gridDim.x) {
        double bn2 = 0.0;
        for (int k = lane; k < nz; k += 64) {
            const long I = col + (long)k * nxy;
            const double a = g.b[I], w = g.b[3 * U + I], t = g.b[4 * U + I];
            br[k] = a;
            bw[k] = w;
            bt[k] = t;
            bn2 += a * a + w * w + t * t;
        }
        const double bn = sqrt(wave_sum1(bn2));
        const double tol = g.rtol * bn;
        // reduced right-hand side: b_w + alpha L_w(b_rho + alpha L_rw w_wall, b_th + alpha L_tw w_wall)
        for (int k = lane; k < nz; k += 64) ww[k] = (k == 0 || k == nz - 1) ? bw[k] : 0.0;
        wave_sync();
        {
            double y[S];
            chain(g.alpha, br, bt, &y);
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (sk[s] > 0) {
                    sb[lane + 64 * s] = bw[sk[s]] + g.alpha * y[s];
                    sx[lane + 64 * s] = g.x0 ? g.x0[U + col + (long)sk[s] * nxy] : bw[sk[s]];
                }
        }
        int iters = 0;
        bool conv = bn == 0.0;
        if (conv)
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (sk[s] > 0) sx[lane + 64 * s] = 0.0;
        // guess choice (as in the full form), on the reduced system: the
        // residual of the default start w = b_w
        bool choose = g.pick && g.x0 && !conv;
        double rdef = 0.0;
        if (choose) {
            double t[S], y[S];
#pragma unroll
            for (int s = 0; s < S; ++s) t[s] = sk[s] > 0 ? bw[sk[s]] : 0.0;
            apply(t, y);
            double r2 = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double r = sk[s] > 0 ? sb[lane + 64 * s] - (t[s] - beta * y[s]) : 0.0;
                r2 += r * r;
            }
            rdef = sqrt(wave_sum1(r2));
        }
        for (int rs = 0; rs <= g.max_restarts && !conv; ++rs) {
            double V[M + 1][S];
            {
                double t[S];
#pragma unroll
                for (int s = 0; s < S; ++s) t[s] = sk[s] > 0 ? sx[lane + 64 * s] : 0.0;
                apply(t, V[0]);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    V[0][s] = sk[s] > 0 ? sb[lane + 64 * s] - (t[s] - beta * V[0][s]) : 0.0;
            }
            double rn2 = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) rn2 += V[0][s] * V[0][s];
            const double rn = sqrt(wave_sum1(rn2));
            if (choose) {
                choose = false;
                if (rdef < rn) {
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (sk[s] > 0) sx[lane + 64 * s] = bw[sk[s]];
                    --rs;
                    continue;
                }
            }
            if (rn <= tol) { conv = true; break; }
            {
                const double inv = 1.0 / rn;
#pragma unroll
                for (int s = 0; s < S; ++s) V[0][s] *= inv;
            }
            double gj = rn, res = rn;
            int jn = 0;
            bool done = false;
            static_for<M>([&](auto jc) __attribute__((always_inline)) {
                constexpr int j = decltype(jc)::value;
                if (!done) {
                    apply(V[j], V[j + 1]);
                    double hc[M + 2];
#pragma unroll
                    for (int i = 0; i <= M + 1; ++i) {
                        hc[i] = 0.0;
                        if (i <= j)
#pragma unroll
                            for (int s = 0; s < S; ++s) hc[i] += V[j + 1][s] * V[i][s];
                        if (i == j + 1)
#pragma unroll
                            for (int s = 0; s < S; ++s) hc[i] += V[j + 1][s] * V[j + 1][s];
                    }
                    wave_sum_t<j + 2>(hc);
                    const double w2 = hc[j + 1];
                    double p2 = 0.0;
#pragma unroll
                    for (int i = 0; i <= j; ++i) {
                        p2 += hc[i] * hc[i];
#pragma unroll
                        for (int s = 0; s < S; ++s) V[j + 1][s] -= hc[i] * V[i][s];
                    }
                    double nn2 = w2 - p2;
                    if (nn2 < 1e-4 * w2) {
                        double e[M + 1];
#pragma unroll
                        for (int i = 0; i <= M; ++i) {
                            e[i] = 0.0;
                            if (i <= j)
#pragma unroll
                                for (int s = 0; s < S; ++s) e[i] += V[j + 1][s] * V[i][s];
                        }
                        wave_sum_t<j + 1>(e);
#pragma unroll
                        for (int i = 0; i <= j; ++i) {
#pragma unroll
                            for (int s = 0; s < S; ++s) V[j + 1][s] -= e[i] * V[i][s];
                            hc[i] += e[i];
                        }
                        double t2 = 0.0;
#pragma unroll
                        for (int s = 0; s < S; ++s) t2 += V[j + 1][s] * V[j + 1][s];
                        nn2 = wave_sum1(t2);
                    }
                    const double nn = sqrt(nn2 > 0.0 ? nn2 : 0.0);
                    if (nn > 0.0) {
                        const double inv = 1.0 / nn;
#pragma unroll
                        for (int s = 0; s < S; ++s) V[j + 1][s] *= inv;
                    }
#pragma unroll
                    for (int i = 0; i <= j; ++i) hc[i] = (i == j ? 1.0 : 0.0) - beta * hc[i];
                    const double sub = -beta * nn;
#pragma unroll
                    for (int i = 0; i < j; ++i) {
                        const double c = cs[i], sg = sn[i], a = hc[i], bb = hc[i + 1];
                        hc[i] = c * a + sg * bb;
                        hc[i + 1] = -sg * a + c * bb;
                    }
                    const double a = hc[j];
                    const double r = sqrt(a * a + sub * sub);
                    const double c = r > 0.0 ? a / r : 1.0, sg = r > 0.0 ? sub / r : 0.0;
                    if (lane == 0) {
#pragma unroll
                        for (int i = 0; i < j; ++i) R[i * M + j] = hc[i];
                        R[j * M + j] = r;
                        cs[j] = c;
                        sn[j] = sg;
                        gv[j] = c * gj;
                    }
                    wave_sync();
                    gj = -sg * gj;
                    res = fabs(gj);
                    ++iters;
                    jn = j + 1;
                    done = res <= tol || nn == 0.0;
                }
            });
            double y[M];
#pragma unroll
            for (int i = M - 1; i >= 0; --i) {
                y[i] = 0.0;
                if (i < jn) {
                    double acc = gv[i];
#pragma unroll
                    for (int l = i + 1; l < M; ++l)
                        if (l < jn) acc -= R[i * M + l] * y[l];
                    y[i] = acc / R[i * M + i];
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (sk[s] > 0) {
                    double acc = sx[lane + 64 * s];
#pragma unroll
                    for (int i = 0; i < M; ++i) acc += y[i] * V[i][s];
                    sx[lane + 64 * s] = acc;
                }
            }
            if (res <= tol) {
                double t[S], w[S];
#pragma unroll
                for (int s = 0; s < S; ++s) t[s] = sk[s] > 0 ? sx[lane + 64 * s] : 0.0;
                apply(t, w);
                double tn2 = 0.0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const double d = sk[s] > 0 ? sb[lane + 64 * s] - (t[s] - beta * w[s]) : 0.0;
                    tn2 += d * d;
                }
                conv = sqrt(wave_sum1(tn2)) <= tol;
            }
        }
        // reconstruct rho' and theta' from the full w column
        for (int k = lane; k < nz; k += 64)
            if (k == 0 || k == nz - 1) ww[k] = bw[k];
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (sk[s] > 0) ww[sk[s]] = sx[lane + 64 * s];
        wave_sync();
        chain(g.alpha, br, bt, nullptr);
        for (int k = lane; k < nz; k += 64) {
            const long I = col + (long)k * nxy;
            g.x[I] = rt[k];
            g.x[3 * U + I] = ww[k];
            g.x[4 * U + I] = tt[k];
            g.x[U + I] = g.b[U + I];
            g.x[2 * U + I] = g.b[2 * U + I];
        }
        if (lane == 0 && g.iters) g.iters[col] = conv ? iters : -iters - 1;
        wave_sync();
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

template <bool RESID>
static hipError_t launch_lv(const HeviParams &h, const double *x, double *y, hipStream_t s, bool uv, double alpha,
                            const double *b)
{
    const long nxy = (long)h.nx * h.ny;
    const dim3 grid((unsigned)((nxy + 255) / 256)), blk(256);
    switch (h.N) {
    case 1: hipLaunchKernelGGL((lv_apply_kernel<1, RESID>), grid, blk, 0, s, h, x, y, uv, alpha, b); break;
    case 2: hipLaunchKernelGGL((lv_apply_kernel<2, RESID>), grid, blk, 0, s, h, x, y, uv, alpha, b); break;
    case 3: hipLaunchKernelGGL((lv_apply_kernel<3, RESID>), grid, blk, 0, s, h, x, y, uv, alpha, b); break;
    case 4: hipLaunchKernelGGL((lv_apply_kernel<4, RESID>), grid, blk, 0, s, h, x, y, uv, alpha, b); break;
    case 5: hipLaunchKernelGGL((lv_apply_kernel<5, RESID>), grid, blk, 0, s, h, x, y, uv, alpha, b); break;
    case 6: hipLaunchKernelGGL((lv_apply_kernel<6, RESID>), grid, blk, 0, s, h, x, y, uv, alpha, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lv_apply(const HeviParams &h, const double *x, double *y, hipStream_t s, bool uv)
{
    return launch_lv<false>(h, x, y, s, uv, 0.0, nullptr);
}

hipError_t launch_lv_resid(const HeviParams &h, double alpha, const double *b, const double *x3, double *y,
                           hipStream_t s)
{
    return launch_lv<true>(h, x3, y, s, false, alpha, b);
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
    if (g.schur) {
        if (g.restart != kGmresRegM || h.nz - 2 > 64 * kGmresSchurSlots) return hipErrorInvalidValue;
        const size_t lds = sizeof(double) * ((size_t)h.nz * 5 + (size_t)h.nz * (2 * h.N + 1) + 6 * (size_t)h.nz +
                                             2 * (h.nz + 2 * h.N) + 2 * 64 * kGmresSchurSlots +
                                             kGmresRegM * kGmresRegM + 3 * kGmresRegM);
        const int grid = (int)(ncol < 32768 ? ncol : 32768);
        if (h.nz - 2 <= 64)
            hipLaunchKernelGGL((gmres_schur_kernel<kGmresRegM, 1>), dim3(grid), dim3(64), lds, s, h, g);
        else
            hipLaunchKernelGGL((gmres_schur_kernel<kGmresRegM, kGmresSchurSlots>), dim3(grid), dim3(64), lds, s, h, g);
        return hipGetLastError();
    }
    if (g.restart == kGmresRegM && 3 * h.nz <= 64 * kGmresRegSlots) {
        // register basis: LDS for the level tables, the exchange vector and
        // the Hessenberg data only
        const size_t lds = sizeof(double) * ((size_t)h.nz * 5 + (size_t)h.nz * (2 * h.N + 1) + 9 * h.nz +
                                             2 * (h.nz + 2 * h.N) + kGmresRegM * kGmresRegM + 3 * kGmresRegM);
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
