// gfx950 kernels of the per-column MLP that predicts the initial guess of
// the HEVI column solves: feature extraction and resampling, FP16 MFMA
// forward GEMMs with FP32 accumulation, FP32 backward, Adam.
//
// Network: x (208: 198 features zero-padded) -> SiLU(W1 x + b1) (256)
//          -> SiLU(W2 h1 + b2) (256) -> y = W3 h2 + b3 + S x (256: 195 used),
// with a linear bypass S [256][208]: the exact map from the features to the
// correction is linear for a fixed column grid and alpha ((I - alpha L_v)^-1
// - I), the hidden layers carry its dependence on those.
// Features of a column with right-hand side b (fields rho', w, theta' on the
// n_z lattice levels): the default start x0 = b leaves the residual
// r = alpha L_v b, and the exact correction x - b = (I - alpha L_v)^-1 r is a
// linear function of r alone.  r is made dimensionless level by level
// (rho'/rho0, w/c0 with c0 = sqrt(gamma p0 / rho0), theta'/theta0), divided
// by one column scale s (RMS of the dimensionless r over the column's 3 n_z
// values) and resampled linearly in z to the 65 canonical levels (LGL nodes
// of 16 equal order-4 elements of the column): features 0 .. 194; then 3
// scalars (alpha / 10, 100 alpha c0(z_0) / H, log10 H / 5), zeros to 207.
// s itself is not a feature: the correction is homogeneous of degree one in
// r, so the map from r / s does not depend on s.  The correction is thus predicted
// relative to its own size, not to the size of b.
// Output: the dimensionless correction on the canonical levels,
// x0 = b + D s resample^-1(y), with the w correction zero on the walls.
#include "nh_internal.h"

#include <hip/hip_fp16.h>
#include <math.h>

namespace nh {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- features
// canonical level c of a column with lattice levels z[0..nz-1]: interval and weight
__device__ __forceinline__ void canon_interp(const double *z, int nz, double zc, int *k0, double *t)
{
    int lo = 0, hi = nz - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (z[mid] <= zc) lo = mid; else hi = mid;
    }
    *k0 = lo;
    *t = (zc - z[lo]) / (z[lo + 1] - z[lo]);
    if (*t < 0.0) *t = 0.0;
    if (*t > 1.0) *t = 1.0;
}

// Dimension factor of field f (0: rho', 1: w, 2: theta') at lattice level k.
__device__ __forceinline__ double dim_factor(const MlpColParams &p, int f, int k)
{
    const double *L = p.lev + (long)k * kLevW;
    if (f == 0) return L[0];
    if (f == 2) return L[1];
    return sqrt(p.gamma * L[2] / L[0]);
}

// 64 columns per workgroup of 512 threads: lane = column (every load reads
// 64 consecutive columns of one level, coalesced), the 8 waves split the
// levels of the scale sum and the canonical levels of the resampling; the
// features of the 64 columns are assembled in LDS and written out as whole
// rows.  The interpolation intervals of the canonical levels and the
// inverse dimension factors of every level are tabulated in LDS first
// (dynamic LDS: 3 n_z doubles).  The residual of the start is rscale * lb
// (fields 0, 3, 4 of [5][U]); the targets are the correction x - base of
// that start, base = b ([5][U]) or a previous guess ([3][U], base3).
__global__ void __launch_bounds__(512) mlp_features_kernel(MlpColParams p, const double *__restrict__ base,
                                                           bool base3, const double *__restrict__ lb,
                                                           double rscale, const double *__restrict__ x, long col0,
                                                           long ncol, _Float16 *__restrict__ feat,
                                                           double *__restrict__ scale, float *__restrict__ tgt)
{
    constexpr int NWV = 8;   // waves
    __shared__ _Float16 sf[64][kMlpIn];
    __shared__ double spart[NWV][64];
    __shared__ int sk0[kMlpNC];
    __shared__ double st[kMlpNC];
    extern __shared__ double sdinv[];   // [3][n_z]
    const int nz = p.nz;
    const long nxy = (long)p.nx * p.ny;
    const long U = nxy * nz;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int fld[3] = {0, 3, 4};
    const double H = p.z[nz - 1] - p.z[0];
    for (int i = threadIdx.x; i < 3 * nz; i += 64 * NWV) sdinv[i] = 1.0 / dim_factor(p, i / nz, i % nz);
    for (int c = threadIdx.x; c < kMlpNC; c += 64 * NWV)
        canon_interp(p.z, nz, p.z[0] + H * p.zc[c], &sk0[c], &st[c]);
    __syncthreads();
    const long r0 = (long)blockIdx.x * 64;
    const long r = r0 + lane;
    const bool ok = r < ncol;
    const long col = col0 + (ok ? r : 0);
    // s = RMS over the column of the dimensionless residual
    double a = 0.0;
#pragma unroll 4
    for (int k = q; k < nz; k += NWV) {
        const long I = col + (long)k * nxy;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const double l = rscale * lb[fld[f] * U + I] * sdinv[f * nz + k];
            a += l * l;
        }
    }
    spart[q][lane] = a;
    __syncthreads();
    double ssum = 0.0;
#pragma unroll
    for (int w = 0; w < NWV; ++w) ssum += spart[w][lane];
    const double s = sqrt(ssum / (3.0 * nz)) + 1e-300;
#pragma unroll 3
    for (int c = q; c < kMlpNC; c += NWV) {
        const int k0 = sk0[c];
        const double t = st[c];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const long I0 = fld[f] * U + col + (long)k0 * nxy, I1 = I0 + nxy;
            const double d0 = sdinv[f * nz + k0], d1 = sdinv[f * nz + k0 + 1];
            const double vl = (1.0 - t) * (rscale * lb[I0] * d0) + t * (rscale * lb[I1] * d1);
            sf[lane][f * kMlpNC + c] = (_Float16)(vl / s);
            if (tgt && ok) {
                const long B0 = (base3 ? f : fld[f]) * U + col + (long)k0 * nxy, B1 = B0 + nxy;
                const double vx = (1.0 - t) * ((x[I0] - base[B0]) * d0) + t * ((x[I1] - base[B1]) * d1);
                tgt[r * kMlpOut + f * kMlpNC + c] = (float)(vx / s);
            }
        }
    }
    if (q == 0) {
        sf[lane][kMlpNF] = (_Float16)(p.alpha / 10.0);
        sf[lane][kMlpNF + 1] = (_Float16)(100.0 * p.alpha * dim_factor(p, 1, 0) / H);
        sf[lane][kMlpNF + 2] = (_Float16)(log10(H) / 5.0);
        for (int i = kMlpNF + 3; i < kMlpIn; ++i) sf[lane][i] = (_Float16)0.0f;
        if (ok) scale[r] = s;
    } else if (tgt && ok) {
        for (int i = kMlpNF + q - 1; i < kMlpOut; i += NWV - 1) tgt[r * kMlpOut + i] = 0.0f;
    }
    __syncthreads();
    // rows of 208 halves = 104 words; threads write consecutive words
    const long nrow = ncol - r0 < 64 ? ncol - r0 : 64;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&sf[0][0]);
    uint32_t *dst = reinterpret_cast<uint32_t *>(feat + r0 * kMlpIn);
    for (long i = threadIdx.x; i < nrow * (kMlpIn / 2); i += 64 * NWV) dst[i] = src[i];
}

// x0 = b + D s (y resampled from the canonical to the lattice levels); the
// w correction is zero on the bottom and top levels, and a non-finite
// prediction falls back to x0 = b.  64 columns per workgroup of 512
// threads: the used outputs of the 64 rows of y are staged in LDS, lane =
// column (b reads and x0 writes coalesced), the 8 waves split the levels.
// Per-level tables (dynamic LDS: 4 n_z doubles and n_z ints): the canonical
// interval and weight of each lattice level and its dimension factors.
__global__ void __launch_bounds__(512) mlp_guess_kernel(MlpColParams p, const double *__restrict__ b, long col0,
                                                        long ncol, const float *__restrict__ y,
                                                        const double *__restrict__ scale, double *__restrict__ x0)
{
    __shared__ float sy[64][kMlpNF + 1];
    extern __shared__ double sg[];
    const int nz = p.nz;
    double *tg = sg;              // [n_z] interpolation weight
    double *dg = sg + nz;         // [3][n_z] dimension factors
    int *lg = (int *)(sg + 4 * nz);   // [n_z] canonical interval
    const long nxy = (long)p.nx * p.ny;
    const long U = nxy * nz;
    const int fld[3] = {0, 3, 4};
    const double H = p.z[nz - 1] - p.z[0];
    for (int k = threadIdx.x; k < nz; k += 512) {
        const double zh = (p.z[k] - p.z[0]) / H;
        int lo = 0, hi = kMlpNC - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (p.zc[mid] <= zh) lo = mid; else hi = mid;
        }
        double t = (zh - p.zc[lo]) / (p.zc[lo + 1] - p.zc[lo]);
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        lg[k] = lo;
        tg[k] = t;
        for (int f = 0; f < 3; ++f) dg[f * nz + k] = dim_factor(p, f, k);
    }
    const long r0 = (long)blockIdx.x * 64;
    const long nrow = ncol - r0 < 64 ? ncol - r0 : 64;
    for (long i = threadIdx.x; i < nrow * kMlpNF; i += 512) {
        const long rr = i / kMlpNF;
        const int c = (int)(i - rr * kMlpNF);
        sy[rr][c] = y[(r0 + rr) * kMlpOut + c];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    if (lane >= nrow) return;
    const long r = r0 + lane;
    const double s = scale[r];
#pragma unroll 2
    for (int k = q; k < nz; k += 8) {
        const long I = col0 + r + (long)k * nxy;
        const int lo = lg[k];
        const double t = tg[k];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float *yr = &sy[lane][f * kMlpNC];
            double d = (1.0 - t) * yr[lo] + t * yr[lo + 1];
            if (!isfinite(d) || (f == 1 && (k == 0 || k == nz - 1))) d = 0.0;
            x0[f * U + I] = b[fld[f] * U + I] + dg[f * nz + k] * s * d;
        }
    }
}

// acc += A B^T over one 32-wide k slice held as 8 halves per lane, as two
// v_mfma_f32_16x16x16_f16 (halves 0-3, then 4-7 of both operands: the same
// k values pair up).  The single-instruction v_mfma_f32_16x16x32_f16 form
// gave run-to-run different results in the fused inference kernel although
// its LDS accesses are race-free between barriers; that build spills MFMA
// operands and rewrites their registers right behind the instruction, so
// it is not used.
__device__ __forceinline__ float4v mfma_k32(const half8 &a, const half8 &b, float4v c)
{
    const half4 al = {a[0], a[1], a[2], a[3]}, ah = {a[4], a[5], a[6], a[7]};
    const half4 bl = {b[0], b[1], b[2], b[3]}, bh = {b[4], b[5], b[6], b[7]};
    c = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, c, 0, 0, 0);
}

// ---------------------------------------------------------------- forward GEMM (MFMA)
// C[M x 256] = A[M x K] W[256 x K]^T (+ A2[M x K2] W2[256 x K2]^T) + bias,
// FP16 operands, FP32 accumulation on v_mfma_f32_16x16x16_f16 (two per
// 32-wide K slice, one for a 16-wide remainder).  Workgroup: 64 rows and all 256
// outputs, 4 waves (wave w: outputs 64 w .. 64 w + 63, 4 x 4 MFMA tiles).
// The K loop stages 32-wide slices of A (64 x 32, shared by the 4 waves) in
// LDS; each wave loads its own W fragments straight from memory (W is a
// few hundred KB and stays in L2).  The next slice of both is loaded into
// registers while the current one is multiplied.  A lane's A and B operands
// hold the same 8 (or 4) k values, so the pairing inside the instruction is
// consistent.  The optional second product (the linear bypass of the last
// layer) is accumulated first, into the same registers.  Epilogue: Z (FP32
// pre-activation, skipped when null) and, when act != 0, H = SiLU(Z) in
// FP16.  Requires M % 64 == 0, K % 16 == 0, K2 % 16 == 0.
__global__ void __launch_bounds__(256) gemm_rows_kernel(const _Float16 *__restrict__ A,
                                                        const _Float16 *__restrict__ W,
                                                        const float *__restrict__ bias, int K,
                                                        const _Float16 *__restrict__ A2,
                                                        const _Float16 *__restrict__ W2, int K2,
                                                        float *__restrict__ Z, _Float16 *__restrict__ Hout, int act)
{
    __shared__ half8 sA[64 * 4];    // [row][k octet]
    half4 *sA4 = reinterpret_cast<half4 *>(sA);
    const int t = threadIdx.x, wave = t / 64, lane = t % 64;
    const long m0 = (long)blockIdx.x * 64;
    const int r16 = lane % 16, g = lane / 16;
    float4v acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = float4v{0.f, 0.f, 0.f, 0.f};

    auto run = [&](const _Float16 *Ap, const _Float16 *Wp, int KK) {
        const int K32 = KK & ~31;
        // thread t stages octet t % 4 of A row t / 4; lane (r16, g) of wave w
        // reads k octet g of W rows 64 w + 16 c + r16
        const _Float16 *ga = Ap + (m0 + t / 4) * KK + (t % 4) * 8;
        const _Float16 *gw = Wp + (long)(64 * wave + r16) * KK + 8 * g;
        if (K32 > 0) {
            half8 ra = *(const half8 *)ga;
            half8 bv[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = *(const half8 *)(gw + (long)16 * c * KK);
            for (int k = 0; k < K32; k += 32) {
                __syncthreads();   // the previous slice has been read
                sA[t] = ra;
                __syncthreads();
                half8 bn[4];
                if (k + 32 < K32) {
                    ra = *(const half8 *)(ga + k + 32);
#pragma unroll
                    for (int c = 0; c < 4; ++c) bn[c] = *(const half8 *)(gw + (long)16 * c * KK + k + 32);
                }
                half8 av[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = sA[(16 * a + r16) * 4 + g];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[a][c] = mfma_k32(av[a], bv[c], acc[a][c]);
                if (k + 32 < K32)
#pragma unroll
                    for (int c = 0; c < 4; ++c) bv[c] = bn[c];
            }
        }
        if (KK > K32) {
            // 16-wide remainder: quads instead of octets
            const half4 ra = *(const half4 *)(Ap + (m0 + t / 4) * KK + K32 + (t % 4) * 4);
            const _Float16 *gw4 = Wp + (long)(64 * wave + r16) * KK + K32 + 4 * g;
            half4 bv[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = *(const half4 *)(gw4 + (long)16 * c * KK);
            __syncthreads();
            sA4[t] = ra;
            __syncthreads();
            half4 av[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = sA4[(16 * a + r16) * 4 + g];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x16f16(av[a], bv[c], acc[a][c], 0, 0, 0);
        }
    };
    // the bypass product first (the fused inference kernel accumulates in
    // the same order)
    if (A2) run(A2, W2, K2);
    run(A, W, K);

    // output layout: lane holds rows 4 (lane / 16) + i, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long row = m0 + 16 * a + 4 * g + i;
                const int col = 64 * wave + 16 * c + r16;
                const float z = acc[a][c][i] + bias[col];
                if (Z) Z[row * 256 + col] = z;
                if (act) Hout[row * 256 + col] = (_Float16)(z / (1.0f + expf(-z)));
            }
}

// ---------------------------------------------------------------- fused inference
// The guess x0 of 64 columns per workgroup of 512 threads (8 waves) with
// everything between the right-hand side and x0 kept in LDS: the features
// of the 64 columns (computed as in mlp_features_kernel), the three layers
// on v_mfma_f32_16x16x16_f16 with the A operands read from LDS (wave w:
// outputs 32 w .. 32 w + 31 of the 64 rows; W fragments from memory, where
// they stay L2 resident), and the resampling of the output to the lattice
// levels (as in mlp_guess_kernel).  Layer 1 and the linear bypass share one
// pass over the features, after which one LDS region holds in turn the
// features, H1, H2 and the output rows (about 58 KB per workgroup, two
// workgroups per CU).  The MFMA operands and the order of accumulation are
// those of gemm_rows_kernel, so the guess equals that of the separate
// kernels.
constexpr int kLdF = kMlpIn + 8;    // LDS row of the features (halves), padded
constexpr int kLdH = kMlpHid + 8;   // LDS row of the activations (halves), padded
// the shared region: features, then H1, H2, output rows (the largest)
constexpr int kRegBytes = 64 * (kMlpNF + 1) * 4;
static_assert(64 * kLdF * 2 <= kRegBytes && 64 * kLdH * 2 <= kRegBytes && kRegBytes % 16 == 0, "region sizes");

// x0 = base + D s (network of the residual r of the start base,
// dimensionless) per column: base is b ([5][U], fields 0, 3, 4), whose
// residual is r = alpha L_v b (first pass), or the previous guess ([3][U],
// base3), whose residual is r = b - base + alpha L_v base (refinement pass).
// NV = 0: r is read from lb (fields 0, 3, 4 of [5][U]) times rscale.
// NV = N > 0: r is computed here -- each wave walks a contiguous chunk of the
// column's levels with lv_walk -- and kept dimensionless as FP32 rows
// [3][n_z][64] in the shared region until the resampling (n_z <= 65, the
// region's size).  x0 may be base (each element is read before it is
// written, by the same thread; the walk only reads the workgroup's own
// columns).
constexpr int kMlpFusedNz = kRegBytes / (3 * 64 * 4);

template <int NV>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) mlp_infer_kernel(MlpColParams p, HeviParams hp,
                                                        MlpWeights wt, const double *base, bool base3,
                                                        const double *b, const double *lb, double rscale, long col0,
                                                        long ncol, double *x0)
{
    constexpr int NWV = 8;
    __shared__ __align__(16) unsigned char sreg[kRegBytes];
    _Float16 *sf = reinterpret_cast<_Float16 *>(sreg);   // features [64][kLdF]
    _Float16 *sh = reinterpret_cast<_Float16 *>(sreg);   // H1, then H2 [64][kLdH]
    __shared__ double spart[NWV][64];
    __shared__ double sscale[64];
    __shared__ int sk0[kMlpNC];
    __shared__ double st[kMlpNC];
    extern __shared__ double stab[];
    const int nz = p.nz;
    double *sdinv = stab;              // [3][n_z] inverse dimension factors
    double *dg = stab + 3 * nz;        // [3][n_z] dimension factors
    double *tg = stab + 6 * nz;        // [n_z] canonical weight of each lattice level
    int *lg = (int *)(stab + 7 * nz);  // [n_z] canonical interval of each lattice level
    float *sy = reinterpret_cast<float *>(sreg);   // [64][kMlpNF + 1] outputs, after the last layer

    const long nxy = (long)p.nx * p.ny;
    const long U = nxy * nz;
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const int fld[3] = {0, 3, 4};
    const double H = p.z[nz - 1] - p.z[0];

    // ---- tables
    for (int i = tid; i < 3 * nz; i += 64 * NWV) {
        sdinv[i] = 1.0 / dim_factor(p, i / nz, i % nz);
        dg[i] = dim_factor(p, i / nz, i % nz);
    }
    for (int c = tid; c < kMlpNC; c += 64 * NWV) canon_interp(p.z, nz, p.z[0] + H * p.zc[c], &sk0[c], &st[c]);
    for (int k = tid; k < nz; k += 64 * NWV) {
        const double zh = (p.z[k] - p.z[0]) / H;
        int lo = 0, hi = kMlpNC - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (p.zc[mid] <= zh) lo = mid; else hi = mid;
        }
        double t = (zh - p.zc[lo]) / (p.zc[lo + 1] - p.zc[lo]);
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        lg[k] = lo;
        tg[k] = t;
    }
    __syncthreads();

    // ---- features (lane = column, the waves split the levels)
    const long r0 = (long)blockIdx.x * 64;
    const long nrow = ncol - r0 < 64 ? ncol - r0 : 64;
    const long r = r0 + lane;
    const long col = col0 + (lane < nrow ? r : r0);
    float *rbuf = reinterpret_cast<float *>(sreg);   // NV > 0: residual rows [3][n_z][64]
    {
        double a = 0.0;
        if constexpr (NV > 0) {
            auto resid = [&](int k, double l0, double l3, double l4, double xr, double xw, double xt) {
                const long I = col + (long)k * nxy;
                double v[3] = {p.alpha * l0, p.alpha * l3, p.alpha * l4};
                if (base3) {
                    v[0] = b[I] - xr + v[0];
                    v[1] = b[3 * U + I] - xw + v[1];
                    v[2] = b[4 * U + I] - xt + v[2];
                }
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const double d = v[f] * sdinv[f * nz + k];
                    rbuf[(f * nz + k) * 64 + lane] = (float)d;
                    a += d * d;
                }
            };
            // a contiguous chunk of levels per wave, walked with a window
            // (computing each level from its own 2N+1 neighbours instead
            // measured slower: 0.57 against 0.38 ms per pass)
            const long xw = base3 ? U : 3 * U, xt = base3 ? 2 * U : 4 * U;
            const int chunk = (nz + NWV - 1) / NWV;
            const int ka = q * chunk, kb = min(nz, ka + chunk);
            if (ka < kb) lv_walk<NV>(hp, col, ka, kb, base, xw, xt, resid);
        } else {
#pragma unroll 4
            for (int k = q; k < nz; k += NWV) {
                const long I = col + (long)k * nxy;
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const double l = rscale * lb[fld[f] * U + I] * sdinv[f * nz + k];
                    a += l * l;
                }
            }
        }
        spart[q][lane] = a;
    }
    __syncthreads();
    double ssum = 0.0;
#pragma unroll
    for (int w = 0; w < NWV; ++w) ssum += spart[w][lane];
    const double s = sqrt(ssum / (3.0 * nz)) + 1e-300;
    _Float16 *fr = sf + lane * kLdF;
    if constexpr (NV > 0) {
        // canonical levels c = q, q + 8, ... of this lane's column from the
        // residual rows, held in registers until every wave has read them
        constexpr int NCW = (kMlpNC + NWV - 1) / NWV;
        _Float16 hv[NCW][3];
#pragma unroll
        for (int j = 0; j < NCW; ++j) {
            const int c = q + j * NWV;
            if (c < kMlpNC) {
                const int k0 = sk0[c];
                const double t = st[c];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const double v0 = rbuf[(f * nz + k0) * 64 + lane], v1 = rbuf[(f * nz + k0 + 1) * 64 + lane];
                    hv[j][f] = (_Float16)(((1.0 - t) * v0 + t * v1) / s);
                }
            }
        }
        __syncthreads();   // every wave has read the residual rows
#pragma unroll
        for (int j = 0; j < NCW; ++j) {
            const int c = q + j * NWV;
            if (c < kMlpNC)
#pragma unroll
                for (int f = 0; f < 3; ++f) fr[f * kMlpNC + c] = hv[j][f];
        }
    } else {
#pragma unroll 3
        for (int c = q; c < kMlpNC; c += NWV) {
            const int k0 = sk0[c];
            const double t = st[c];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const long I0 = fld[f] * U + col + (long)k0 * nxy, I1 = I0 + nxy;
                const double d0 = sdinv[f * nz + k0], d1 = sdinv[f * nz + k0 + 1];
                const double vl = (1.0 - t) * (rscale * lb[I0] * d0) + t * (rscale * lb[I1] * d1);
                fr[f * kMlpNC + c] = (_Float16)(vl / s);
            }
        }
    }
    if (q == 0) {
        fr[kMlpNF] = (_Float16)(p.alpha / 10.0);
        fr[kMlpNF + 1] = (_Float16)(100.0 * p.alpha * dim_factor(p, 1, 0) / H);
        fr[kMlpNF + 2] = (_Float16)(log10(H) / 5.0);
        for (int i = kMlpNF + 3; i < kMlpIn; ++i) fr[i] = (_Float16)0.0f;
        sscale[lane] = s;
    }
    __syncthreads();

    // ---- layers
    const int wave = q, r16 = lane % 16, g = lane / 16;
    float4v acc[4][2], acc3[4][2];   // current layer; last layer (bypass first)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            acc[a][c] = float4v{0.f, 0.f, 0.f, 0.f};
            acc3[a][c] = float4v{0.f, 0.f, 0.f, 0.f};
        }
    // C += S[64 x KK] (LDS, row stride ld) Wp[32 w .. 32 w + 31][KK]^T for
    // up to two (W, C) pairs sharing the A fragments
    auto mma = [&](const _Float16 *S, int ld, int KK, const _Float16 *Wa, float4v (&Ca)[4][2],
                   const _Float16 *Wb, float4v (&Cb)[4][2]) __attribute__((always_inline)) {
        const int K32 = KK & ~31;
        const long wrow = (long)(32 * wave + r16) * KK;
        if (K32 > 0) {
            half8 ba[2], bb[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                ba[c] = *(const half8 *)(Wa + wrow + (long)16 * c * KK + 8 * g);
                if (Wb) bb[c] = *(const half8 *)(Wb + wrow + (long)16 * c * KK + 8 * g);
            }
#pragma unroll 1
            for (int k = 0; k < K32; k += 32) {
                half8 na[2], nb[2];
                if (k + 32 < K32)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        na[c] = *(const half8 *)(Wa + wrow + (long)16 * c * KK + k + 32 + 8 * g);
                        if (Wb) nb[c] = *(const half8 *)(Wb + wrow + (long)16 * c * KK + k + 32 + 8 * g);
                    }
                half8 av[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = *(const half8 *)(S + (16 * a + r16) * ld + k + 8 * g);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        Ca[a][c] = mfma_k32(av[a], ba[c], Ca[a][c]);
                        if (Wb) Cb[a][c] = mfma_k32(av[a], bb[c], Cb[a][c]);
                    }
                if (k + 32 < K32)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        ba[c] = na[c];
                        if (Wb) bb[c] = nb[c];
                    }
            }
        }
        if (KK > K32) {
            half4 ba[2], bb[2], av[4];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                ba[c] = *(const half4 *)(Wa + wrow + (long)16 * c * KK + K32 + 4 * g);
                if (Wb) bb[c] = *(const half4 *)(Wb + wrow + (long)16 * c * KK + K32 + 4 * g);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = *(const half4 *)(S + (16 * a + r16) * ld + K32 + 4 * g);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    Ca[a][c] = __builtin_amdgcn_mfma_f32_16x16x16f16(av[a], ba[c], Ca[a][c], 0, 0, 0);
                    if (Wb) Cb[a][c] = __builtin_amdgcn_mfma_f32_16x16x16f16(av[a], bb[c], Cb[a][c], 0, 0, 0);
                }
        }
    };
    // H = SiLU(acc + bias) into the activation rows (lane: rows 4 g + i,
    // column r16 of each tile); acc is cleared for the next layer
    auto store_h = [&](const float *bias) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * a + 4 * g + i, cl = 32 * wave + 16 * c + r16;
                    const float z = acc[a][c][i] + bias[cl];
                    sh[row * kLdH + cl] = (_Float16)(z / (1.0f + expf(-z)));
                }
                acc[a][c] = float4v{0.f, 0.f, 0.f, 0.f};
            }
    };
    // layer 1 and the bypass of the last layer: one pass over the features
    mma(sf, kLdF, kMlpIn, wt.W[3], acc3, wt.W[0], acc);
    __syncthreads();   // every wave has read the features
    store_h(wt.bias[0]);
    __syncthreads();
    mma(sh, kLdH, kMlpHid, wt.W[1], acc, nullptr, acc);
    __syncthreads();   // every wave has read H1
    store_h(wt.bias[1]);
    __syncthreads();
    mma(sh, kLdH, kMlpHid, wt.W[2], acc3, nullptr, acc3);
    __syncthreads();   // every wave has read H2
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * a + 4 * g + i, cl = 32 * wave + 16 * c + r16;
                if (cl < kMlpNF) sy[row * (kMlpNF + 1) + cl] = acc3[a][c][i] + wt.bias[2][cl];
            }
    __syncthreads();

    // ---- resampling to the lattice levels (lane = column, the waves split the levels)
    if (lane >= nrow) return;
    const double sc = sscale[lane];
#pragma unroll 2
    for (int k = q; k < nz; k += NWV) {
        const long I = col0 + r + (long)k * nxy;
        const int lo = lg[k];
        const double t = tg[k];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float *yr = sy + lane * (kMlpNF + 1) + f * kMlpNC;
            double d = (1.0 - t) * yr[lo] + t * yr[lo + 1];
            if (!isfinite(d) || (f == 1 && (k == 0 || k == nz - 1))) d = 0.0;
            x0[f * U + I] = base[(base3 ? f : fld[f]) * U + I] + dg[f * nz + k] * sc * d;
        }
    }
}

// ---------------------------------------------------------------- backward (FP32 MFMA)
// C[Mo x No] = sum_k A(mo, k) B(k, no) over k in [z kslice, (z + 1) kslice),
// into C + z Mo No (split K; the slices are summed by sum_slices_kernel).
// A is FP32 with element strides (sam, sak), B FP16 or FP32 with strides
// (sbk, sbn).  FP32 products and accumulation on v_mfma_f32_16x16x4_f32
// (lane l: A row l % 16 and B column l % 16 at k = l / 16; result rows
// 4 (l / 16) + i, column l % 16).  Workgroup: a 64 x 64 tile, 4 waves of
// 2 x 2 MFMA tiles (wave w: rows 32 (w / 2) .., columns 32 (w % 2) ..); K
// staged through LDS in chunks of 32 as FP32, rows of kBkLd floats so that
// the four k rows a wave reads at once fall in distinct banks.  Staging
// walks whichever operand index has unit stride fastest (coalesced loads).
constexpr int kBkK = 32, kBkLd = 80, kBkPer = kBkK * 64 / 256;

template <typename TB>
__global__ void __launch_bounds__(256) gemm_mfma32_kernel(const float *__restrict__ A, long sam, long sak,
                                                          const TB *__restrict__ B, long sbk, long sbn, int Mo,
                                                          int No, int K, float *__restrict__ C, int kslice)
{
    __shared__ float As[kBkK][kBkLd];
    __shared__ float Bs[kBkK][kBkLd];
    const int t = threadIdx.x, wave = t / 64, lane = t % 64;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kb = blockIdx.z * kslice, ke = min(K, kb + kslice);
    C += (long)blockIdx.z * Mo * No;
    const int wm = 32 * (wave / 2), wn = 32 * (wave % 2);
    const int r16 = lane % 16, kq = lane / 16;
    // staging slots of this thread: (k, m) of A and (k, n) of B for each of
    // kBkPer values, the unit-stride index running fastest
    int ka[kBkPer], ma[kBkPer], kbs[kBkPer], nb[kBkPer];
#pragma unroll
    for (int r = 0; r < kBkPer; ++r) {
        const int i = t + r * 256;
        ka[r] = sak == 1 ? i % kBkK : i / 64;
        ma[r] = sak == 1 ? i / kBkK : i % 64;
        kbs[r] = sbk == 1 ? i % kBkK : i / 64;
        nb[r] = sbk == 1 ? i / kBkK : i % 64;
    }
    float ra[kBkPer], rb[kBkPer];
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < kBkPer; ++r) {
            const int gm = m0 + ma[r], gka = k0 + ka[r];
            ra[r] = (gm < Mo && gka < ke) ? A[gm * sam + gka * sak] : 0.f;
            const int gn = n0 + nb[r], gkb = k0 + kbs[r];
            rb[r] = (gn < No && gkb < ke) ? (float)B[gkb * sbk + gn * sbn] : 0.f;
        }
    };
    float4v acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = float4v{0.f, 0.f, 0.f, 0.f};
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += kBkK) {
        __syncthreads();   // the previous chunk has been read
#pragma unroll
        for (int r = 0; r < kBkPer; ++r) {
            As[ka[r]][ma[r]] = ra[r];
            Bs[kbs[r]][nb[r]] = rb[r];
        }
        __syncthreads();
        if (k0 + kBkK < ke) load(k0 + kBkK);   // next chunk in flight during the products
#pragma unroll
        for (int kk = 0; kk < kBkK; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = As[kk + kq][wm + 16 * x + r16];
                b[x] = Bs[kk + kq][wn + 16 * x + r16];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm + 16 * x + 4 * kq + i, col = n0 + wn + 16 * y + r16;
                if (row < Mo && col < No) C[(long)row * No + col] = acc[x][y][i];
            }
}

// out[i] = sum_z P[z][i], z = 0 .. slices-1 in order (deterministic)
__global__ void sum_slices_kernel(const float *__restrict__ P, int slices, long n, float *__restrict__ out)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        float t = 0.f;
        for (int z = 0; z < slices; ++z) t += P[z * n + i];
        out[i] = t;
    }
}

// column sums of X [M][N] over row chunks of kMlpColRows: part[c][n] = sum over
// rows m of chunk c of X[m][n].  Workgroup of 256 threads = 64 columns x 4
// row phases (coalesced 256-byte row segments); the 4 phase sums of a column
// are added in a fixed order, and sum_slices_kernel adds the chunks in
// order, so the result is deterministic.
__global__ void __launch_bounds__(256) colsum_part_kernel(const float *__restrict__ X, int M, int N,
                                                          float *__restrict__ part)
{
    __shared__ float ph[4][64];
    const int c = threadIdx.x % 64, r = threadIdx.x / 64;
    const int n = blockIdx.x * 64 + c;
    const int m0 = blockIdx.y * kMlpColRows, m1 = min(M, m0 + kMlpColRows);
    float s = 0.f;
    if (n < N)
        for (int m = m0 + r; m < m1; m += 4) s += X[(long)m * N + n];
    ph[r][c] = s;
    __syncthreads();
    if (r == 0 && n < N) part[(long)blockIdx.y * N + n] = ((ph[0][c] + ph[1][c]) + ph[2][c]) + ph[3][c];
}

// dY = 2 (Y - T) / (M N), loss partials per block
__global__ void mse_grad_kernel(const float *__restrict__ Y, const float *__restrict__ T, long n, float scale,
                                float *__restrict__ dY, float *__restrict__ part)
{
    __shared__ float sh[256];
    float a = 0.f;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        dY[i] = 2.f * d * scale;
        a += d * d;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// *out = scale * sum of part[0 .. n): one wave, lane l the entries l, l + 64,
// ... in order, then a fixed butterfly
__global__ void __launch_bounds__(64) sum_kernel(const float *__restrict__ part, int n, float scale,
                                                 float *__restrict__ out)
{
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 64) s += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x == 0) *out = s * scale;
}

// dZ = dH * SiLU'(Z),  SiLU'(z) = sig(z) (1 + z (1 - sig(z)))
__global__ void silu_back_kernel(const float *__restrict__ dH, const float *__restrict__ Z, long n,
                                 float *__restrict__ dZ)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float z = Z[i];
        const float sg = 1.f / (1.f + expf(-z));
        dZ[i] = dH[i] * sg * (1.f + z * (1.f - sg));
    }
}

// Adam on FP32 masters (Kingma & Ba), then FP16 copies.  The first ndecay
// parameters also take decoupled weight decay wd (Loshchilov & Hutter):
// w -= lr (m_hat / (sqrt(v_hat) + eps) + wd w).
__global__ void adam_kernel(long n, const float *__restrict__ g, float *__restrict__ w, float *__restrict__ m,
                            float *__restrict__ v, _Float16 *__restrict__ wh, float lr, float b1, float b2,
                            float eps, float c1, float c2, long ndecay, float wd)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float u = (mi / c1) / (sqrtf(vi / c2) + eps);
        if (i < ndecay) u += wd * w[i];
        const float wi = w[i] - lr * u;
        w[i] = wi;
        wh[i] = (_Float16)wi;
    }
}

__global__ void to_half_kernel(long n, const float *__restrict__ w, _Float16 *__restrict__ wh)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        wh[i] = (_Float16)w[i];
}

static int grid_for(long n, int block)
{
    long gsz = (n + block - 1) / block;
    if (gsz > 65535) gsz = 65535;
    if (gsz < 1) gsz = 1;
    return (int)gsz;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_mlp_features(const MlpColParams &p, const double *base, bool base3, const double *lb,
                               double rscale, const double *x, long col0, long ncol, void *feat, double *scale,
                               float *tgt, hipStream_t s)
{
    const int grid = (int)((ncol + 63) / 64);
    const size_t lds = sizeof(double) * 3 * (size_t)p.nz;
    hipLaunchKernelGGL(mlp_features_kernel, dim3(grid), dim3(512), lds, s, p, base, base3, lb, rscale, x, col0,
                       ncol, (_Float16 *)feat, scale, tgt);
    return hipGetLastError();
}

hipError_t launch_mlp_guess(const MlpColParams &p, const double *b, long col0, long ncol, const float *y,
                            const double *scale, double *x0, hipStream_t s)
{
    const int grid = (int)((ncol + 63) / 64);
    const size_t lds = (sizeof(double) * 4 + sizeof(int)) * (size_t)p.nz;
    hipLaunchKernelGGL(mlp_guess_kernel, dim3(grid), dim3(512), lds, s, p, b, col0, ncol, y, scale, x0);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpColParams &p, const HeviParams &hp, const MlpNet &net, const double *base,
                            bool base3, const double *b, const double *lb, double rscale, long col0, long ncol,
                            double *x0, hipStream_t s)
{
    MlpWeights wt;
    for (int i = 0; i < 4; ++i) wt.W[i] = (const _Float16 *)net.wh[i];
    for (int i = 0; i < 3; ++i) wt.bias[i] = net.b[i];
    const int grid = (int)((ncol + 63) / 64);
    const size_t lds = (sizeof(double) * 7 + sizeof(int)) * (size_t)p.nz;
    const int nv = lb ? 0 : hp.N;
    if (nv > 0 && p.nz > kMlpFusedNz) return hipErrorInvalidValue;
#define NH_INFER(NN)                                                                                           \
    hipLaunchKernelGGL(mlp_infer_kernel<NN>, dim3(grid), dim3(512), lds, s, p, hp, wt, base, base3, b, lb, rscale, \
                       col0, ncol, x0)
    switch (nv) {
    case 0: NH_INFER(0); break;
    case 1: NH_INFER(1); break;
    case 2: NH_INFER(2); break;
    case 3: NH_INFER(3); break;
    case 4: NH_INFER(4); break;
    case 5: NH_INFER(5); break;
    case 6: NH_INFER(6); break;
    default: return hipErrorInvalidValue;
    }
#undef NH_INFER
    return hipGetLastError();
}

int mlp_fused_max_nz() { return kMlpFusedNz; }

hipError_t mlp_forward(const MlpNet &net, int M, const void *X, hipStream_t s, bool keep_z)
{
    static_assert(kMlpHid == 256 && kMlpOut == 256, "gemm_rows_kernel computes 256 outputs");
    const dim3 blk(256), grid(M / 64);
    const _Float16 *none = nullptr;
    hipLaunchKernelGGL(gemm_rows_kernel, grid, blk, 0, s, (const _Float16 *)X, (const _Float16 *)net.wh[0], net.b[0],
                       kMlpIn, none, none, 0, keep_z ? net.Z1 : nullptr, (_Float16 *)net.H1, 1);
    hipLaunchKernelGGL(gemm_rows_kernel, grid, blk, 0, s, (const _Float16 *)net.H1, (const _Float16 *)net.wh[1],
                       net.b[1], kMlpHid, none, none, 0, keep_z ? net.Z2 : nullptr, (_Float16 *)net.H2, 1);
    hipLaunchKernelGGL(gemm_rows_kernel, grid, blk, 0, s, (const _Float16 *)net.H2, (const _Float16 *)net.wh[2],
                       net.b[2], kMlpHid, (const _Float16 *)X, (const _Float16 *)net.wh[3], kMlpIn, net.Y,
                       (_Float16 *)nullptr, 0);
    return hipGetLastError();
}

// Weight gradient G[Mo x No] = sum over the batch (K = M rows) of A^T B,
// split over the batch so that enough workgroups run (a 256 x 208 gradient
// is only 28 tiles), then the slices are summed in a fixed order.
template <typename TB>
static void weight_grad(const float *A, long lda, const TB *B, long ldb, int Mo, int No, int K, float *G,
                        float *part, hipStream_t s)
{
    int slices = K / 64;
    if (slices > kMlpSlices) slices = kMlpSlices;
    if (slices < 1) slices = 1;
    const int kslice = (K + slices - 1) / slices;
    hipLaunchKernelGGL((gemm_mfma32_kernel<TB>), dim3((No + 63) / 64, (Mo + 63) / 64, slices), dim3(256), 0, s,
                       A, 1L, lda, B, ldb, 1L, Mo, No, K, part, kslice);
    const long n = (long)Mo * No;
    hipLaunchKernelGGL(sum_slices_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, part, slices, n, G);
}

// out[n] = sum over the M rows of X[m][n], through row-chunk partials in part
static void column_sums(const float *X, int M, int N, float *out, float *part, hipStream_t s)
{
    const int chunks = (M + kMlpColRows - 1) / kMlpColRows;
    hipLaunchKernelGGL(colsum_part_kernel, dim3((N + 63) / 64, chunks), dim3(256), 0, s, X, M, N, part);
    const long n = N;
    hipLaunchKernelGGL(sum_slices_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, part, chunks, n, out);
}

hipError_t mlp_backward(const MlpNet &net, int M, const void *X, const float *dY, hipStream_t s)
{
    const dim3 blk(256);
    const _Float16 *Xh = (const _Float16 *)X, *H1 = (const _Float16 *)net.H1, *H2 = (const _Float16 *)net.H2;
    const _Float16 *W2 = (const _Float16 *)net.wh[1], *W3 = (const _Float16 *)net.wh[2];
    // linear bypass: dS = dY^T X [256 x 208]
    weight_grad(dY, (long)kMlpOut, Xh, (long)kMlpIn, kMlpOut, kMlpIn, M, net.gw[3], net.part_k, s);
    // layer 3: dW3 = dY^T H2 [256 x 256], db3 = sum dY, dH2 = dY W3 [M x 256]
    weight_grad(dY, (long)kMlpOut, H2, (long)kMlpHid, kMlpOut, kMlpHid, M, net.gw[2], net.part_k, s);
    column_sums(dY, M, kMlpOut, net.gb[2], net.part_k, s);
    hipLaunchKernelGGL((gemm_mfma32_kernel<_Float16>), dim3(kMlpHid / 64, M / 64, 1), blk, 0, s, dY,
                       (long)kMlpOut, 1L, W3, (long)kMlpHid, 1L, M, kMlpHid, kMlpOut, net.dH, kMlpOut);
    hipLaunchKernelGGL(silu_back_kernel, dim3(grid_for((long)M * kMlpHid, 256)), blk, 0, s, net.dH, net.Z2,
                       (long)M * kMlpHid, net.dZ);
    // layer 2
    weight_grad(net.dZ, (long)kMlpHid, H1, (long)kMlpHid, kMlpHid, kMlpHid, M, net.gw[1], net.part_k, s);
    column_sums(net.dZ, M, kMlpHid, net.gb[1], net.part_k, s);
    hipLaunchKernelGGL((gemm_mfma32_kernel<_Float16>), dim3(kMlpHid / 64, M / 64, 1), blk, 0, s, net.dZ,
                       (long)kMlpHid, 1L, W2, (long)kMlpHid, 1L, M, kMlpHid, kMlpHid, net.dH, kMlpHid);
    hipLaunchKernelGGL(silu_back_kernel, dim3(grid_for((long)M * kMlpHid, 256)), blk, 0, s, net.dH, net.Z1,
                       (long)M * kMlpHid, net.dZ);
    // layer 1: dW1 = dZ1^T X [256 x K0]
    weight_grad(net.dZ, (long)kMlpHid, Xh, (long)kMlpIn, kMlpHid, kMlpIn, M, net.gw[0], net.part_k, s);
    column_sums(net.dZ, M, kMlpHid, net.gb[0], net.part_k, s);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const MlpNet &net, int M, const float *T, float *loss, hipStream_t s)
{
    const long n = (long)M * kMlpOut;
    hipLaunchKernelGGL(mse_grad_kernel, dim3(kMlpLossBlocks), dim3(256), 0, s, net.Y, T, n, 1.0f / (float)n, net.dY,
                       net.part);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, s, net.part, kMlpLossBlocks, 1.0f / (float)n, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpNet &net, float lr, float b1, float b2, float eps, int step, float wd, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    // the hidden path (W1, b1, W2, b2, W3, b3) precedes the bypass S
    const long ndecay = wd > 0.f ? net.nparam - (long)kMlpOut * kMlpIn : 0;
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(net.nparam, 256)), dim3(256), 0, s, net.nparam, net.grad,
                       net.master, net.m, net.v, (_Float16 *)net.half, lr, b1, b2, eps, c1, c2, ndecay, wd);
    return hipGetLastError();
}

hipError_t mlp_sync_half(const MlpNet &net, hipStream_t s)
{
    hipLaunchKernelGGL(to_half_kernel, dim3(grid_for(net.nparam, 256)), dim3(256), 0, s, net.nparam, net.master,
                       (_Float16 *)net.half);
    return hipGetLastError();
}

}  // namespace nh
