// gfx950 kernels of libnhsem: the fused right-hand side / SSP-RK stage of the
// perturbation-form Euler equations on LGL hexahedral elements (Eq. governing,
// Eq. governing:matrix, Algorithms 1-3 of Kang, Giraldo & Camp), the
// element-based DSS gather and scatter, the diagonal mass and diagnostics.
//
// Design of the stage kernel (one launch per RK stage):
//   * The mesh is an axis-aligned tensor box, so the metric of element e is
//     diag(2/h_x, 2/h_y, 2/h_z) and its quadrature weight factorises,
//     w_i w_j w_k J^e = (w_i h_x/2)(w_j h_y/2)(w_k h_z/2).  Every term of S is
//     a pointwise coefficient times one first derivative, so
//       M_I^{-1} sum_{(i,e)->I} w J S  =  pointwise(I)
//         + sum_d coef_d(I) * [ sum_{e_d ∋ I_d} m_d(e_d) d_d^{(e_d)} f(I) ] / M_d(I_d)
//     -- the 3D direct stiffness summation collapses into one mass-weighted
//     average of one-sided element derivatives per direction.  This is the
//     same discrete operator as gather -> element contraction -> DSS -> M^{-1}
//     (up to rounding), evaluated without element-local copies in HBM, without
//     atomics, and with every unique node written exactly once.
//   * x/y: the averaged derivative is a (2N+1)-point stencil along the
//     lattice line with host-built coefficients (zero outside the one or two
//     elements that share the node).  z: element-local contractions on a
//     per-thread register column, with the lower element's contribution at a
//     shared level carried in registers.
//   * A workgroup owns a TX x TY tile of lattice columns (aligned to element
//     boundaries) and marches upward one level at a time.  Each level's
//     derived fields (p', u, v, w, theta', rho) for the tile and its halo
//     (N nodes before, 1 after, in x and y) are staged in LDS (double
//     buffered, one barrier per level); the EOS is evaluated once per staged
//     node.  HBM traffic per node and stage: read q^s (40 B), q^n (40 B, when
//     used), forcing (16 B), write q^{s+1} (40 B).
#include "nh_internal.h"

#include <math.h>

namespace nh {

// ---------------------------------------------------------------- EOS
// p' = p0 ((1+a)(1+b))^gamma - p0 with a = rho'/rho0, b = theta'/theta0: the
// equation of state p = p_a (rho R theta / p_a)^gamma (Sec. 2.1) relative to
// p0 = EOS(rho0, theta0), written without cancellation (a and b use the
// reciprocals 1/rho0, 1/theta0 of the level table).  s = a + b + ab is formed
// without FMA contraction.  For |s| < 1/16 the binomial series
// sum_{n=1}^{14} C(gamma, n) s^n (coefficients from the host; the first
// omitted term is below 1e-19 of the result) replaces expm1(gamma log1p(s)).
__device__ __noinline__ double pow_ratio_slow(double s, double gam)
{
    return expm1(gam * log1p(s));
}

__device__ __forceinline__ double pert_pressure(double rp, double tp, double inv_rho0, double inv_th0,
                                                double p0, double gam, const double *eosc)
{
    const double a = rp * inv_rho0;
    const double b = tp * inv_th0;
    const double s = __dadd_rn(__dadd_rn(a, b), __dmul_rn(a, b));
    double r;
    if (fabs(s) < 0.0625) {
        double acc = eosc[kEosTerms - 1];
#pragma unroll
        for (int n = kEosTerms - 2; n >= 0; --n) acc = fma(acc, s, eosc[n]);
        r = acc * s;
    } else {
        r = pow_ratio_slow(s, gam);
    }
    return p0 * r;
}

// ---------------------------------------------------------------- stage
// Workgroup shape of the stage kernel: tile of TX x TY lattice columns
// (AX x AY elements), one thread per owned node of a z-element slab
// (N levels x TX x TY, at most 1024).
// Two values of the stage kernel's arithmetic type in one LDS element.
template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

template <int N, int AX, int AY>
struct StageShape {
    static constexpr int N1 = N + 1;
    static constexpr int TX = AX * N, TY = AY * N, NCOL = TX * TY;
    static constexpr int NOWN = N * NCOL;
    static constexpr int NT = (NOWN + 63) / 64 * 64;
    static_assert(NT <= 1024, "one thread per owned node of a slab");
    static constexpr int PX = TX + N + 1, PY = TY + N + 1, PS = PX * PY;
    static constexpr int NSP = NCOL + (TX + TY) * N1;   // staged nodes per plane
    static constexpr int NC = 2 * N + 1;
    static_assert(NT >= NCOL, "bottom-level threads must own whole columns");
};

// One RK stage (or a bare RHS) over the whole lattice.
//
// A workgroup owns a TX x TY tile of lattice columns and walks up the
// z-elements.  For element ez it stages the N+1 levels ez*N .. ez*N+N of the
// tile and its x/y halo in LDS as (p', u, v, w, theta', rho')
// -- the bottom level is kept from the previous element -- then each thread
// evaluates one owned node: (2N+1)-point DSS'd derivative stencils along x
// and y on its level, the one-sided z derivative inside the element from the
// LDS column, sources, and the RK combination.  The element below's
// contribution at the shared bottom level is carried in registers by the
// threads that own the bottom level (same threads for every element).
template <int N, int AX, int AY, typename T>
__device__ __forceinline__ void stage_body(const StageParams &p, const int tile, const int tid)
{
    using S = StageShape<N, AX, AY>;
    constexpr int N1 = S::N1, TX = S::TX, TY = S::TY, NCOL = S::NCOL, NOWN = S::NOWN;
    constexpr int NT = S::NT, PX = S::PX, PS = S::PS, NSP = S::NSP, NC = S::NC;
    constexpr bool kF64 = sizeof(T) == 8;
    using T2 = typename Pair<T>::type;

    // Plane slots of field pairs (p', u), (v, w), (theta', rho'), one 16-byte
    // (FP32: 8-byte) LDS element per pair, so that a stencil tap reads the six
    // fields with three loads; plus N rows of padding: stencil taps past the
    // last row of a plane read finite padding or the next plane (always with
    // a zero coefficient), so tap addresses need no clamping.
    __shared__ T2 plbuf[N1 * 3 * PS + N * PX];
    T2(*pl)[3][PS] = reinterpret_cast<T2(*)[3][PS]>(plbuf);
    __shared__ T cx[TX * NC];
    __shared__ T cy[TY * NC];
    __shared__ T sD[N1 * N1];
    __shared__ double sE[kEosTerms];
    __shared__ uint32_t smap[NSP];
    __shared__ uint16_t sidx[NSP];
    // Level data of the current element's N+1 levels used by the compute
    // phase (rho0, dtheta0/dz, tau, w_lo, w_hi): LDS reads, so that no vector
    // load (and its wait on every outstanding vector-memory operation, the
    // prefetches included) sits in the middle of the compute phase.
    __shared__ double slev[N1 * 5];
    // EOS level data (1/rho0, 1/theta0, p0) of the levels being staged:
    // slot 0 the bottom level, slots 1..N the element's new levels.
    __shared__ double stlev[N1 * 3];
    __shared__ T scarry[6 * NCOL];
    // FP32 form: the tile's own nodes in FP64 (ring of N+1 levels, as the
    // planes), kept at staging for the RK combination a q^n + b q^s + c R,
    // which stays FP64
    __shared__ double qown[kF64 ? 1 : N1 * 5 * NCOL];

    const int bx = tile % p.ntx, by = tile / p.ntx;
    const int x0 = bx * TX, y0 = by * TY;
    const uint32_t nx = p.nx, ny = p.ny;
    const uint32_t plane_bytes = nx * ny * 8u;
    const uint64_t field_bytes = (uint64_t)plane_bytes * (uint32_t)p.nz;

    for (int i = tid; i < TX * NC; i += NT) {
        const int xg = x0 + i / NC;
        if constexpr (kF64)
            cx[i] = (xg < p.nx) ? p.gx[(long)xg * NC + i % NC] : 0.0;
        else
            cx[i] = (xg < p.nx) ? p.gxf[(long)xg * NC + i % NC] : 0.0f;
    }
    for (int i = tid; i < TY * NC; i += NT) {
        const int yg = y0 + i / NC;
        if constexpr (kF64)
            cy[i] = (yg < p.ny) ? p.gy[(long)yg * NC + i % NC] : 0.0;
        else
            cy[i] = (yg < p.ny) ? p.gyf[(long)yg * NC + i % NC] : 0.0f;
    }
    for (int i = tid; i < N1 * N1; i += NT) sD[i] = T(p.cst[kCstD + i]);
    for (int i = tid; i < kEosTerms; i += NT) sE[i] = p.cst[kCstEos + i];
    // slots that are never staged (plane corners, padding) stay zero
    for (int i = tid; i < N1 * 3 * PS + N * PX; i += NT) plbuf[i] = T2{T(0), T(0)};
    __syncthreads();

    // Staging map, the same for every level: staged node s (0 <= s < NSP)
    // -> byte offset of its column in a level (0xffffffff: outside the
    // lattice, staged as zeros) and its slot index in a plane.
    for (int sn = tid; sn < NSP; sn += NT) {
        int px, py;
        if (sn < NCOL) {
            px = N + sn % TX;
            py = N + sn / TX;
        } else if (sn < NCOL + TY * N1) {
            const int s1 = sn - NCOL, c = s1 % N1;
            px = (c < N) ? c : N + TX;
            py = N + s1 / N1;
        } else {
            const int s2 = sn - NCOL - TY * N1, r = s2 / TX;
            px = N + s2 % TX;
            py = (r < N) ? r : N + TY;
        }
        // Periodic wrap by one period (no integer division): staged columns
        // lie in [-N, n + TX), and every column a valid node reads with a
        // nonzero coefficient lies in [-N, n - 1 + N], which one period maps
        // into the lattice (n >= N).  Columns further out are only read with
        // zero coefficients and are staged as zeros.
        int xg = x0 + px - N, yg = y0 + py - N;
        bool ok = true;
        if (xg < 0 || xg >= p.nx) {
            if (p.perx) {
                xg += (xg < 0) ? p.nx : -p.nx;
                ok = xg < p.nx;
            } else {
                ok = false;
            }
        }
        if (yg < 0 || yg >= p.ny) {
            if (p.pery) {
                yg += (yg < 0) ? p.ny : -p.ny;
                ok = ok && yg < p.ny;
            } else {
                ok = false;
            }
        }
        smap[sn] = ok ? ((uint32_t)xg + nx * (uint32_t)yg) * 8u : 0xffffffffu;
        sidx[sn] = (uint16_t)(py * PX + px);
    }
    for (int i = tid; i < N1 * 3; i += NT) {
        const int c = i % 3;
        stlev[i] = p.lev[(long)(i / 3) * kLevW + (c == 0 ? 7 : c == 1 ? 8 : 2)];
    }
    __syncthreads();

    // Stage node s (0 <= s < NSP) of level k into plane slot k mod (N+1).
    // Fill stlev with the EOS data of levels k0 .. k0 + N (the first
    // element's are filled with the staging map above).
    auto fill_stlev = [&](int k0) {
        for (int i = tid; i < N1 * 3; i += NT) {
            const int c = i % 3;
            stlev[i] = p.lev[(long)(k0 + i / 3) * kLevW + (c == 0 ? 7 : c == 1 ? 8 : 2)];
        }
    };

    // Stage node s of level k (stlev slot j) into plane slot k mod (N+1).
    auto stage = [&](int k, int j, int s) {
        const uint32_t off = smap[s];
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0, v4 = 0.0, pp = 0.0;
        if (off != 0xffffffffu) {
            const double *L = stlev + j * 3;
            const char *b = (const char *)p.qs + (off + plane_bytes * (uint32_t)k);
            v0 = *(const double *)(b);
            v1 = *(const double *)(b + field_bytes);
            v2 = *(const double *)(b + 2 * field_bytes);
            v3 = *(const double *)(b + 3 * field_bytes);
            v4 = *(const double *)(b + 4 * field_bytes);
            pp = pert_pressure(v0, v4, L[0], L[1], L[2], p.gamma, sE);
        }
        T2(*P)[PS] = pl[k % N1];
        const int idx = sidx[s];
        if constexpr (!kF64) {
            if (s < NCOL) {
                double *Q = qown + (k % N1) * 5 * NCOL + s;
                Q[0] = v0; Q[NCOL] = v1; Q[2 * NCOL] = v2; Q[3 * NCOL] = v3; Q[4 * NCOL] = v4;
            }
        }
        P[0][idx] = T2{T(pp), T(v1)};
        P[1][idx] = T2{T(v2), T(v3)};
        P[2][idx] = T2{T(v4), T(v0)};
    };

    // x/y part of the tendency at (tx, ty) of plane slot `sl` (reference
    // density r0 of that level) and 1/rho there.
    // NH_FENCE: compiler-only memory fence between phases.  It stops the
    // scheduler from front-loading every LDS read of the x, y and z
    // contractions at once (which spills at the 1024-thread register budget).
#define NH_FENCE() __builtin_amdgcn_sched_barrier(0)
    // NH_PIN: ties the accumulators to an ordered point so instruction
    // selection cannot defer the FMAs of a tap past the loads of later taps.
#define NH_PIN(a)                                                                        \
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]))
    auto horizontal = [&](int sl, T r0, int tx, int ty, T *XY, T &inv) {
        NH_FENCE();
        const T2(*P)[PS] = pl[sl];
        T dx[6], dy[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) { dx[f] = T(0); dy[f] = T(0); }
        const int rowx = (N + ty) * PX;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const T c = cx[tx * NC + m];
            const int j = rowx + tx + m;
            const T2 a = P[0][j], b = P[1][j], e = P[2][j];
            dx[0] += c * a.x;
            dx[1] += c * a.y;
            dx[2] += c * b.x;
            dx[3] += c * b.y;
            dx[4] += c * e.x;
            dx[5] += c * ((r0 + e.y) * a.y);
            NH_PIN(dx);
        }
        NH_FENCE();
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const T c = cy[ty * NC + m];
            const int j = (ty + m) * PX + N + tx;
            const T2 a = P[0][j], b = P[1][j], e = P[2][j];
            dy[0] += c * a.x;
            dy[1] += c * a.y;
            dy[2] += c * b.x;
            dy[3] += c * b.y;
            dy[4] += c * e.x;
            dy[5] += c * ((r0 + e.y) * b.x);
            NH_PIN(dy);
        }
        NH_FENCE();
        const int jo = rowx + N + tx;
        const T u = P[0][jo].y, v = P[1][jo].x;
        inv = T(1) / (r0 + P[2][jo].y);
        XY[0] = -(dx[5] + dy[5]);
        XY[1] = -(u * dx[1] + v * dy[1]) - dx[0] * inv;
        XY[2] = -(u * dx[2] + v * dy[2]) - dy[0] * inv;
        XY[3] = -(u * dx[3] + v * dy[3]);
        XY[4] = -(u * dx[4] + v * dy[4]);
    };

    // one-sided z derivative at local level r of element ez (column (tx,ty))
    auto zderiv = [&](int ez, int r, int tx, int ty, T h2, T *dz) {
        NH_FENCE();
        const int jo = (N + ty) * PX + N + tx;
#pragma unroll
        for (int f = 0; f < 6; ++f) dz[f] = T(0);
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            const T2(*P)[PS] = pl[(ez * N + m) % N1];
            const T d = sD[r * N1 + m];
            const T2 a = P[0][jo], b = P[1][jo], e = P[2][jo];
            const T w = b.y;
            const T r0 = T(slev[m * 5]);
            dz[0] += d * a.x;
            dz[1] += d * a.y;
            dz[2] += d * b.x;
            dz[3] += d * w;
            dz[4] += d * e.x;
            dz[5] += d * ((r0 + e.y) * w);
            NH_PIN(dz);
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) dz[f] *= h2;
    };

    // Loads of the node's own global data (q^n, heating) issued before the
    // contractions so their latency overlaps them.  Every thread runs the
    // arithmetic (coordinates clamped into the lattice) and only the stores
    // are predicated: a conditional use would let the compiler sink the
    // contractions into the branch and keep every loaded LDS value alive.
    //
    // With p.stream (set by the host for states of at least twice the
    // 256 MB last-level cache) these loads and the result stores are
    // non-temporal: each is touched once per launch, and the caches are
    // left to the staged q^s halos that neighbouring tiles re-read
    // (0.3-2.6 % faster per launch on the 512 x 512 x 81 lattice).  On
    // states that fit the last-level cache the next stage re-reads the
    // result from it, and streaming measured 6-11 % slower.
    struct NodeIn {
        uint32_t o;
        bool valid;
        double qn[5], h0, h1;
    };
    auto ld_own = [&](const double *a) -> double {
        if (p.stream) return __builtin_nontemporal_load(a);
        return *a;
    };
    auto prefetch = [&](int k, int gx0, int gy0, NodeIn &nd) {
        nd.valid = gx0 < p.nx && gy0 < p.ny;
        const int gx = nd.valid ? gx0 : 0, gy = nd.valid ? gy0 : 0;
        nd.o = ((uint32_t)gx + nx * (uint32_t)gy) * 8u + plane_bytes * (uint32_t)k;
#pragma unroll
        for (int f = 0; f < 5; ++f)
            nd.qn[f] = (p.a != 0.0) ? ld_own((const double *)((const char *)p.qn + nd.o + f * field_bytes)) : 0.0;
        nd.h0 = p.hq0 ? ld_own((const double *)((const char *)p.hq0 + nd.o)) : 0.0;
        nd.h1 = p.hq0 ? ld_own((const double *)((const char *)p.hq1 + nd.o)) : 0.0;
    };

    // Complete the tendency at level k and write a q^n + b q^s + c R.
    auto finish = [&](int k, int li, int gx0, int gy0, const NodeIn &nd, int tx, int ty, const T *XY, const T *dz,
                      const T inv) {
        NH_FENCE();
        // the node's own fields, re-read from its plane rather than kept in
        // registers through the contractions
        T own[6];
        {
            const T2(*P)[PS] = pl[k % N1];
            const int jo = (N + ty) * PX + N + tx;
            const T2 a = P[0][jo], b = P[1][jo], e = P[2][jo];
            own[1] = a.y;
            own[2] = b.x;
            own[3] = b.y;
            own[4] = e.x;
            own[5] = e.y;
        }
        const bool valid = nd.valid;
        const int gx = valid ? gx0 : 0, gy = valid ? gy0 : 0;
        const double *L = slev + li * 5;
        const uint32_t o = nd.o;
        const T u = own[1], v = own[2], w = own[3];
        const T rp = own[5];
        const T tau = T(L[2]);
        double qs[5];
        if constexpr (kF64) {
            qs[0] = own[5]; qs[1] = own[1]; qs[2] = own[2]; qs[3] = own[3]; qs[4] = own[4];
        } else {
            const double *Q = qown + (k % N1) * 5 * NCOL + (ty * TX + tx);
#pragma unroll
            for (int f = 0; f < 5; ++f) qs[f] = Q[f * NCOL];
        }
        T R[5];
        R[0] = XY[0] - dz[5];
        R[1] = XY[1] - w * dz[1] + T(p.fcor) * v - tau * u;
        R[2] = XY[2] - w * dz[2] - T(p.fcor) * u - tau * v;
        R[3] = XY[3] - w * dz[3] - dz[0] * inv - T(p.g) * rp * inv - tau * w;
        R[4] = XY[4] - w * (dz[4] + T(L[1])) - tau * own[4];
        double Rd[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) Rd[f] = double(R[f]);
        if (p.hq0) Rd[4] += (1.0 - p.hlam) * nd.h0 + p.hlam * nd.h1;
        if (!p.perx && (gx == 0 || gx == p.nx - 1)) Rd[1] = 0.0;
        if (!p.pery && (gy == 0 || gy == p.ny - 1)) Rd[2] = 0.0;
        if (k == 0 || k == p.nz - 1) Rd[3] = 0.0;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const double r = p.a * nd.qn[f] + p.b * qs[f] + p.c * Rd[f];
            double *dst = (double *)((char *)p.out + o + f * field_bytes);
            if (valid) {
                if (p.stream) __builtin_nontemporal_store(r, dst);
                else *dst = r;
            }
        }
    };

    // The lower element's weighted z-derivative at the shared level, per
    // column: written and read only by the thread that owns the column's
    // bottom level (thread col), so it needs no barrier; kept in LDS rather
    // than in registers, which the compute phase needs.
    if (tid < NCOL)
#pragma unroll
        for (int f = 0; f < 6; ++f) scarry[f * NCOL + tid] = T(0);

    for (int s = tid; s < NSP; s += NT) stage(0, 0, s);
    for (int ez = 0; ez < p.nelz; ++ez) {
        for (int i = tid; i < N * NSP; i += NT) stage(ez * N + 1 + i / NSP, 1 + i / NSP, i % NSP);
        for (int i = tid; i < N1 * 5; i += NT) {
            const int c = i % 5;
            slev[i] = p.lev[(long)(ez * N + i / 5) * kLevW + (c == 0 ? 0 : c + 2)];
        }
        __syncthreads();
        const T h2 = T(p.hz2[ez]);
        for (int idx = tid; idx < NOWN; idx += NT) {
            const int l = idx / NCOL, col = idx % NCOL;
            const int tx = col % TX, ty = col / TX;
            const int gx = x0 + tx, gy = y0 + ty;
            const int k = ez * N + l;
            T XY[5], dz[6], inv;
            NodeIn nd;
            prefetch(k, gx, gy, nd);
            horizontal(k % N1, T(slev[l * 5]), tx, ty, XY, inv);
            zderiv(ez, l, tx, ty, h2, dz);
            if (l == 0) {
                const T whi = T(slev[4]);
#pragma unroll
                for (int f = 0; f < 6; ++f) dz[f] = whi * dz[f] + scarry[f * NCOL + col];
                T dt[6];
                zderiv(ez, N, tx, ty, h2, dt);
                const T wlo = T(slev[N * 5 + 3]);
#pragma unroll
                for (int f = 0; f < 6; ++f) scarry[f * NCOL + col] = wlo * dt[f];
            }
            finish(k, l, gx, gy, nd, tx, ty, XY, dz, inv);
        }
        // EOS level data for the next element's staging (its reads of this
        // element's data finished before the barrier above)
        if (ez + 1 < p.nelz) fill_stlev((ez + 1) * N);
        __syncthreads();
    }
    // top level: only the contribution of the element below
    const int ktop = p.nz - 1;
    for (int col = tid; col < NCOL; col += NT) {
        const int tx = col % TX, ty = col / TX;
        const int gx = x0 + tx, gy = y0 + ty;
        T XY[5], inv, carry[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) carry[f] = scarry[f * NCOL + col];
        NodeIn nd;
        prefetch(ktop, gx, gy, nd);
        horizontal(ktop % N1, T(slev[N * 5]), tx, ty, XY, inv);
        finish(ktop, N, gx, gy, nd, tx, ty, XY, carry, inv);
    }
#undef NH_FENCE
#undef NH_PIN
}

// Workgroups are handed to the 8 XCDs round robin (b mod 8), and each XCD has
// its own L2.  Give XCD x the contiguous tile range [x q + min(x, r), ...)
// (q = n / 8, r = n mod 8): tiles that run at the same time on one XCD are
// row neighbours whose x/y halos overlap, so halo re-reads hit that L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

template <int N, int AX, int AY, typename T>
__global__ void __launch_bounds__((StageShape<N, AX, AY>::NT)) stage_kernel(const StageParams p)
{
    stage_body<N, AX, AY, T>(p, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x);
}

// Batched form: the (instance, tile) items of an order group sit in one list
// per XCD, each a contiguous run of tiles of the cost-sorted sequence (so the
// workgroups one XCD runs at a time are neighbours that share halos through
// its L2); workgroup b runs on XCD x = b mod 8 and takes item b / 8 of list x
// (none past its end), and reads the instance's parameters from a device
// descriptor table.
__device__ __forceinline__ int xcd_item(const XcdLists &xl, int b)
{
    const int x = b & (kXcds - 1), it = xl.off[x] + b / kXcds;
    return it < xl.off[x + 1] ? it : -1;
}

template <int N, int AX, int AY, typename T>
__global__ void __launch_bounds__((StageShape<N, AX, AY>::NT))
stage_kernel_batched(const StageParams *__restrict__ P, const int2 *__restrict__ work, const XcdLists xl)
{
    const int i = xcd_item(xl, blockIdx.x);
    if (i < 0) return;
    const int2 it = work[i];
    stage_body<N, AX, AY, T>(P[it.x], it.y, threadIdx.x);
}

// Next item of a persistent workgroup whose home XCD list is `home`: from the
// list of the first XCD (home, home + 1, ...) that is not exhausted, through
// that list's device counter (one vector atomic per attempt, thread 0
// only); `tried` counts the lists found exhausted and only grows, so every
// workgroup reaches -1 (all lists exhausted) after at most one more attempt
// per list.
__device__ __forceinline__ int next_item(const XcdLists &xl, int *counter, int home, int &tried)
{
    while (tried < kXcds) {
        const int x = (home + tried) & (kXcds - 1);
        const int j = __hip_atomic_fetch_add(counter + x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (xl.off[x] + j < xl.off[x + 1]) return xl.off[x] + j;
        ++tried;
    }
    return -1;
}

// ---------------------------------------------------------------- stage, node-class form
// The same fused stage as stage_body, with nodes assigned to threads by
// node class: wave (i, j) of the workgroup takes every node whose local x
// index is i and local y index is j, over all AX x AY elements of the tile
// and all N levels of the slab (lane = element + AX AY level).  Within a
// wave the x and y derivative rules are then uniform: a node inside its
// element (i != 0) uses the element-local (N+1)-tap contraction with the
// LGL derivative row D[i] and one per-node factor 2/h; a node on an element
// face (i = 0) uses the left element's row D[N] and the right element's row
// D[0], each with its factor of the mass-weighted average -- the same
// discrete operator as the (2N+1)-tap stencil of stage_body, with about a
// third fewer taps and the tap weights wave-uniform (scalar registers)
// instead of per-lane LDS reads.
//
// LDS: the N+1 levels of the current element in five plane slots (fields
// p', u, v, w, theta', rho'); slots 0 and 4 alternate as the element's
// bottom and top level (the top of one element is the bottom of the next,
// so no level is copied or staged twice) and slots 1..N-1 hold the local
// levels between.  Plane address of (px, py): py RP + (py / N) PADY + px,
// the skew PADY per element row and the slot bases chosen (residues 0, 1,
// 0, 1, 0 mod 4 doubles) so that the 32 lanes of a half-wave -- 8 elements
// along x, 2 element rows, 2 levels -- read 64 distinct banks.  The lower
// element's weighted z-derivative at the shared level (the carry) is
// computed for every column and field by all threads at the end of each
// element, double-buffered in LDS.
template <int N, int AX, int AY>
struct ClsShape {
    static_assert(N == 4 && AX == 8 && AY == 2, "bank layout worked out for 8 x 2 elements of order 4");
    static constexpr int N1 = N + 1, NE = AX * AY;
    static constexpr int TX = AX * N, TY = AY * N, NCOL = TX * TY;
    static constexpr int NT = N * N * 64;
    static constexpr int PX = TX + N + 1, PY = TY + N + 1;
    static constexpr int RP = PX, PADY = 2;
    static constexpr int PSZ = (PY - 1) * RP + ((PY - 1) / N) * PADY + PX;
    static constexpr int FS = PSZ, SLOT = 6 * PSZ;
    static constexpr int NSP = NCOL + (TX + TY) * N1;
    static constexpr int up4(int v, int r) { return v + (((r - v % 4) % 4) + 4) % 4; }
    static constexpr int B0 = 0;
    static constexpr int B1 = up4(B0 + SLOT, 1);
    static constexpr int B2 = up4(B1 + SLOT, 0);
    static constexpr int B3 = up4(B2 + SLOT, 1);
    static constexpr int B4 = up4(B3 + SLOT, 0);
    static constexpr int TOTAL = B4 + SLOT;
    static __host__ __device__ constexpr int addr(int px, int py) { return py * RP + (py / N) * PADY + px; }
};

__device__ __forceinline__ double wave_uniform(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float wave_uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// One LDS read that the compiler may not merge with a neighbouring one:
// merged pairs (ds_read2_b64 with adjacent or row-strided offsets) took eight
// bank-conflict cycles each in the node-class layout, where single reads of
// the same addresses take none (measured on gfx950).
template <typename T>
__device__ __forceinline__ T lds_one(const T *p)
{
    typedef __attribute__((address_space(3))) const volatile T lds_t;
    return *(lds_t *)p;
}

template <int N, int AX, int AY, typename T>
__device__ __forceinline__ void stage_body_cls(const StageParams &p, const int tile, const int tid)
{
    using S = ClsShape<N, AX, AY>;
    constexpr int N1 = S::N1, NE = S::NE, TX = S::TX, TY = S::TY, NCOL = S::NCOL, NT = S::NT;
    constexpr int PX = S::PX, RP = S::RP, PADY = S::PADY, FS = S::FS, NSP = S::NSP;
    constexpr bool kF64 = sizeof(T) == 8;

    __shared__ T planes[S::TOTAL + N * RP];
    __shared__ T sD[N1 * N1];
    __shared__ double sE[kEosTerms];
    __shared__ uint32_t smap[NSP];
    __shared__ uint16_t sidx[NSP];
    __shared__ double slev[N1 * 5];
    __shared__ double stlev[N1 * 3];
    __shared__ T scarry[2][6 * NCOL];
    // per tile column / row: the two factors of the x (y) average (cfx, cfy)
    __shared__ T scx[2 * TX], scy[2 * TY];

    const int bx = tile % p.ntx, by = tile / p.ntx;
    const int x0 = bx * TX, y0 = by * TY;
    const uint32_t nx = p.nx, ny = p.ny;
    const uint32_t plane_bytes = nx * ny * 8u;
    const uint64_t field_bytes = (uint64_t)plane_bytes * (uint32_t)p.nz;

    for (int i = tid; i < N1 * N1; i += NT) sD[i] = T(p.cst[kCstD + i]);
    for (int i = tid; i < kEosTerms; i += NT) sE[i] = p.cst[kCstEos + i];
    for (int i = tid; i < S::TOTAL + N * RP; i += NT) planes[i] = T(0);
    for (int i = tid; i < 6 * NCOL; i += NT) scarry[0][i] = T(0);   // no element below the bottom
    for (int i = tid; i < 2 * TX; i += NT) {
        const int xg = x0 + i / 2;
        scx[i] = T(p.cfx[2 * (xg < p.nx ? xg : p.nx - 1) + i % 2]);
    }
    for (int i = tid; i < 2 * TY; i += NT) {
        const int yg = y0 + i / 2;
        scy[i] = T(p.cfy[2 * (yg < p.ny ? yg : p.ny - 1) + i % 2]);
    }
    for (int sn = tid; sn < NSP; sn += NT) {
        int px, py;
        if (sn < NCOL) {
            px = N + sn % TX;
            py = N + sn / TX;
        } else if (sn < NCOL + TY * N1) {
            const int s1 = sn - NCOL, c = s1 % N1;
            px = (c < N) ? c : N + TX;
            py = N + s1 / N1;
        } else {
            const int s2 = sn - NCOL - TY * N1, r = s2 / TX;
            px = N + s2 % TX;
            py = (r < N) ? r : N + TY;
        }
        int xg = x0 + px - N, yg = y0 + py - N;
        bool ok = true;
        if (xg < 0 || xg >= p.nx) {
            if (p.perx) {
                xg += (xg < 0) ? p.nx : -p.nx;
                ok = xg < p.nx;
            } else {
                ok = false;
            }
        }
        if (yg < 0 || yg >= p.ny) {
            if (p.pery) {
                yg += (yg < 0) ? p.ny : -p.ny;
                ok = ok && yg < p.ny;
            } else {
                ok = false;
            }
        }
        smap[sn] = ok ? ((uint32_t)xg + nx * (uint32_t)yg) * 8u : 0xffffffffu;
        sidx[sn] = (uint16_t)S::addr(px, py);
    }
    for (int i = tid; i < N1 * 3; i += NT) {
        const int c = i % 3;
        stlev[i] = p.lev[(long)(i / 3) * kLevW + (c == 0 ? 7 : c == 1 ? 8 : 2)];
    }
    __syncthreads();

    auto fill_stlev = [&](int k0) {
        for (int i = tid; i < N1 * 3; i += NT) {
            const int c = i % 3;
            stlev[i] = p.lev[(long)(k0 + i / 3) * kLevW + (c == 0 ? 7 : c == 1 ? 8 : 2)];
        }
    };
    // Stage node s of level k (EOS level data in stlev slot j) into the
    // plane slot starting at `base`.  The loads are unconditional (a node
    // outside the lattice reads column 0 and is zeroed after): a load under a
    // branch makes the compiler wait for it where the branch joins.
    auto stage = [&](int k, int j, int s, int base) {
        const uint32_t off = smap[s];
        const bool in = off != 0xffffffffu;
        const double *L = stlev + j * 3;
        const char *b = (const char *)p.qs + ((in ? off : 0u) + plane_bytes * (uint32_t)k);
        double v0 = *(const double *)(b);
        double v1 = *(const double *)(b + field_bytes);
        double v2 = *(const double *)(b + 2 * field_bytes);
        double v3 = *(const double *)(b + 3 * field_bytes);
        double v4 = *(const double *)(b + 4 * field_bytes);
        v0 = in ? v0 : 0.0; v1 = in ? v1 : 0.0; v2 = in ? v2 : 0.0; v3 = in ? v3 : 0.0; v4 = in ? v4 : 0.0;
        const double pp = pert_pressure(v0, v4, L[0], L[1], L[2], p.gamma, sE);
        T *P = planes + base + sidx[s];
        P[0] = T(pp);
        P[FS] = T(v1);
        P[2 * FS] = T(v2);
        P[3 * FS] = T(v3);
        P[4 * FS] = T(v4);
        P[5 * FS] = T(v0);
    };

    // this thread's node class and node.  Waves w, w + 4, w + 8, w + 12 share
    // a SIMD: class (k, (k + w) mod 4) for wave w + 4k gives every SIMD one
    // face class in x and one in y (the face rules take 2N+2 taps, the
    // interior ones N+1), so the SIMDs finish together.
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ci = wv / N, cj = (wv / N + wv % N) % N;
    const int lane = tid & 63;
    const int el = lane % NE;
    const int ex = el % AX, ey = el / AX;
    // per-lane values, laundered at every element (below) so that the
    // compiler does not hoist address arithmetic derived from them out of
    // the element loop (it would hold it in registers it does not have)
    int l = lane / NE;
    int tx = ex * N + ci, ty = ey * N + cj, col = ty * TX + tx;
    int gx0 = x0 + tx, gy0 = y0 + ty;
    int noff = S::addr(N + ex * N, N + ey * N) + cj * RP + ci;
    // wave-uniform derivative rows D[i], D[j] (scalar registers) and this
    // lane's row D[l] for the z contraction
    T dxr[N1], dyr[N1];
#pragma unroll
    for (int m = 0; m < N1; ++m) {
        dxr[m] = wave_uniform(sD[ci * N1 + m]);
        dyr[m] = wave_uniform(sD[cj * N1 + m]);
    }
    // plane slot of local level 1..N-1 (level 0 and N: the bottom and top
    // slots, which alternate between elements)
    auto mid_slot = [](int m) { return m == 1 ? S::B1 : (m == 2 ? S::B2 : S::B3); };

// NH_FENCE: a compiler memory barrier (no loads moved or merged across it at
// the IR level) plus a scheduling barrier: it keeps the loads of one field's
// taps from being hoisted together with every other field's, which would need
// more registers than a 1024-thread workgroup has.
#define NH_FENCE()                        \
    do {                                  \
        asm volatile("" ::: "memory");    \
        __builtin_amdgcn_sched_barrier(0); \
    } while (0)
#define NH_PIN(a) \
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]))

    struct NodeIn {
        uint32_t o;
        bool valid;
        double qn[5], h0, h1;
    };
    // (unconditional loads, as in `stage`; q^n and the heating snapshots are
    // read from q^s when absent and weighted by zero)
    auto prefetch = [&](int k, NodeIn &nd) {
        nd.valid = gx0 < p.nx && gy0 < p.ny;
        const int gx = nd.valid ? gx0 : 0, gy = nd.valid ? gy0 : 0;
        nd.o = ((uint32_t)gx + nx * (uint32_t)gy) * 8u + plane_bytes * (uint32_t)k;
        const char *qnb = (const char *)(p.a != 0.0 ? p.qn : p.qs);
        const char *h0b = (const char *)(p.hq0 ? p.hq0 : p.qs), *h1b = (const char *)(p.hq0 ? p.hq1 : p.qs);
#pragma unroll
        for (int f = 0; f < 5; ++f) nd.qn[f] = *(const double *)(qnb + nd.o + f * field_bytes);
        nd.h0 = *(const double *)(h0b + nd.o);
        nd.h1 = *(const double *)(h1b + nd.o);
    };

    // Derivatives of the staged fields along x or y at the node `nd` of
    // class c, in the element-average form: S_R = sum_k D[c][k] f(P + R(k))
    // over the element starting at P = node - c (the node itself on a face)
    // and, on a face, the mirrored left element S_L = sum_k D[0][k]
    // f(node - L(k)); with D[N][N-k] = -D[0][k] the average is c1 S_R - c0 S_L
    // (x: R(k) = L(k) = k; y: R(k) = k RP + PADY at k = N, L(k) = k RP +
    // PADY for k >= 1).  Field by field, all taps of a field loaded before its
    // multiply-adds; the momentum component (u along x, v along y) and the
    // mass flux (rho0 + rho') u share one pass.  Each derivative is folded
    // into the tendency XY as it is formed: with a the advecting velocity
    // component (u or v), XY[0] -= d(mass flux), XY[f] -= a d f (f = u, v, w,
    // theta'), and the pressure gradient -d p' / rho into XY[1] (x) or
    // XY[2] (y).
    auto deriv = [&](auto ydir_c, const T *nd, int c, const T (&cr)[N1], T c0, T c1, T r0, T a, T inv, T (&XY)[5]) {
        constexpr bool ydir = decltype(ydir_c)::value;
        const T *P = nd - c * (ydir ? RP : 1);
        const bool face = c == 0;
        auto offR = [&](int k) { return ydir ? k * RP + (k == N ? PADY : 0) : k; };
        auto offL = [&](int k) { return ydir ? -(k * RP + (k >= 1 ? PADY : 0)) : -k; };
        constexpr int FM = ydir ? 2 : 1;
        T dm, dfl;
        {
            T m[N1], v[N1], sr = T(0), sf = T(0);
#pragma unroll
            for (int k = 0; k < N1; ++k) m[k] = lds_one(P + FM * FS + offR(k));
#pragma unroll
            for (int k = 0; k < N1; ++k) v[k] = lds_one(P + 5 * FS + offR(k));
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                sr += cr[k] * m[k];
                sf += cr[k] * ((r0 + v[k]) * m[k]);
            }
            dm = c1 * sr;
            dfl = c1 * sf;
        }
        if (face) {
            NH_FENCE();
            T m[N1], v[N1], sl = T(0), sf = T(0);
#pragma unroll
            for (int k = 0; k < N1; ++k) m[k] = lds_one(nd + FM * FS + offL(k));
#pragma unroll
            for (int k = 0; k < N1; ++k) v[k] = lds_one(nd + 5 * FS + offL(k));
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                sl += cr[k] * m[k];
                sf += cr[k] * ((r0 + v[k]) * m[k]);
            }
            dm -= c0 * sl;
            dfl -= c0 * sf;
        }
        XY[0] -= dfl;
        XY[FM] -= a * dm;
        constexpr int rest[4] = {0, 3 - FM, 3, 4};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            NH_FENCE();
            const int fo = rest[q] * FS;
            T v[N1], sr = T(0), sl = T(0);
#pragma unroll
            for (int k = 0; k < N1; ++k) v[k] = lds_one(P + fo + offR(k));
#pragma unroll
            for (int k = 0; k < N1; ++k) sr += cr[k] * v[k];
            T dd = c1 * sr;
            if (face) {
#pragma unroll
                for (int k = 0; k < N1; ++k) v[k] = lds_one(nd + fo + offL(k));
#pragma unroll
                for (int k = 0; k < N1; ++k) sl += cr[k] * v[k];
                dd -= c0 * sl;
            }
            if (q == 0) XY[FM] -= dd * inv;   // pressure gradient
            else XY[rest[q]] -= a * dd;
        }
    };

    // Complete the tendency at level k (level-data row li of slev) and write
    // a q^n + b q^s + c R: R holds the x, y and z derivative terms, the
    // pointwise terms (Coriolis, sponge, buoyancy, heating) are added here.
    auto finish = [&](int k, int li, const NodeIn &nd, const T *own, const T (&R)[5], const T inv) {
        NH_FENCE();
        const bool valid = nd.valid;
        const int gx = valid ? gx0 : 0, gy = valid ? gy0 : 0;
        const double *L = slev + li * 5;
        const uint32_t o = nd.o;
        const T u = own[FS], v = own[2 * FS], w = own[3 * FS], th = own[4 * FS], rp = own[5 * FS];
        const T tau = T(L[2]);
        double qs[5];
        if constexpr (kF64) {
            qs[0] = rp; qs[1] = u; qs[2] = v; qs[3] = w; qs[4] = th;
        } else {
            const char *qb = (const char *)p.qs + o;
#pragma unroll
            for (int f = 0; f < 5; ++f) qs[f] = *(const double *)(qb + f * field_bytes);
        }
        double Rd[5];
        Rd[0] = double(R[0]);
        Rd[1] = double(R[1] + T(p.fcor) * v - tau * u);
        Rd[2] = double(R[2] - T(p.fcor) * u - tau * v);
        Rd[3] = double(R[3] - T(p.g) * rp * inv - tau * w);
        Rd[4] = double(R[4] - w * T(L[1]) - tau * th);
        if (p.hq0) Rd[4] += (1.0 - p.hlam) * nd.h0 + p.hlam * nd.h1;
        if (!p.perx && (gx == 0 || gx == p.nx - 1)) Rd[1] = 0.0;
        if (!p.pery && (gy == 0 || gy == p.ny - 1)) Rd[2] = 0.0;
        if (k == 0 || k == p.nz - 1) Rd[3] = 0.0;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const double r = (p.a != 0.0 ? p.a * nd.qn[f] : 0.0) + p.b * qs[f] + p.c * Rd[f];
            if (valid) *(double *)((char *)p.out + o + f * field_bytes) = r;
        }
    };

    // x and y part of the tendency at `own` (reference density r0 of its
    // level) into R, and 1/rho
    auto horizontal = [&](const T *own, T r0, T (&R)[5], T &inv) {
        NH_FENCE();
        inv = T(1) / (r0 + own[5 * FS]);
#pragma unroll
        for (int f = 0; f < 5; ++f) R[f] = T(0);
        deriv(std::integral_constant<bool, false>{}, own, ci, dxr, ci == 0 ? scx[2 * tx] : T(0), scx[2 * tx + 1], r0,
              own[FS], inv, R);
        NH_FENCE();
        deriv(std::integral_constant<bool, true>{}, own, cj, dyr, cj == 0 ? scy[2 * ty] : T(0), scy[2 * ty + 1], r0,
              own[2 * FS], inv, R);
    };

    for (int s = tid; s < NSP; s += NT) stage(0, 0, s, S::B0);
    for (int ez = 0; ez < p.nelz; ++ez) {
        asm volatile("" : "+v"(l), "+v"(tx), "+v"(ty), "+v"(col), "+v"(gx0), "+v"(gy0), "+v"(noff));
        const int sbot = (ez & 1) ? S::B4 : S::B0, stop = (ez & 1) ? S::B0 : S::B4;
        for (int i = tid; i < N * NSP; i += NT) {
            const int lv = 1 + i / NSP;
            stage(ez * N + lv, lv, i % NSP, lv < N ? mid_slot(lv) : stop);
        }
        for (int i = tid; i < N1 * 5; i += NT) {
            const int c = i % 5;
            slev[i] = p.lev[(long)(ez * N + i / 5) * kLevW + (c == 0 ? 0 : c + 2)];
        }
        __syncthreads();
        const T h2 = T(p.hz2[ez]);
        {
            const int k = ez * N + l;
            const int myslot = (l == 0) ? sbot : mid_slot(l);
            const T *own = planes + myslot + noff;
            const T r0 = T(slev[l * 5]);
            T R[5], inv;
            horizontal(own, r0, R, inv);
            NH_FENCE();
            NodeIn nd;
            prefetch(k, nd);
            // z: element-local contraction with this lane's row D[l], tap by
            // tap (the six accumulators pinned after each tap, so the
            // scheduler cannot hoist every tap's loads at once); on level 0
            // the lower element's weighted contribution (the carry) is added.
            // Folded into R.
            {
                NH_FENCE();
                T dz[6];
#pragma unroll
                for (int f = 0; f < 6; ++f) dz[f] = T(0);
#pragma unroll
                for (int m = 0; m < N1; ++m) {
                    const int sm = (m == 0) ? sbot : (m == N ? stop : mid_slot(m));
                    const T *q = planes + sm + noff;
                    const T d = sD[l * N1 + m];
                    const T w = lds_one(q + 3 * FS);
                    const T r0m = T(slev[m * 5]);
                    dz[0] += d * lds_one(q);
                    dz[1] += d * lds_one(q + FS);
                    dz[2] += d * lds_one(q + 2 * FS);
                    dz[3] += d * w;
                    dz[4] += d * lds_one(q + 4 * FS);
                    dz[5] += d * ((r0m + lds_one(q + 5 * FS)) * w);
                    NH_PIN(dz);
                }
                const bool bot = l == 0;
                const T sc = bot ? h2 * T(slev[4]) : h2;
                const T *cry = scarry[ez & 1] + col;
#pragma unroll
                for (int f = 0; f < 6; ++f) dz[f] = sc * dz[f] + (bot ? cry[f * NCOL] : T(0));
                const T w = own[3 * FS];
                R[0] -= dz[5];
                R[1] -= w * dz[1];
                R[2] -= w * dz[2];
                R[3] -= w * dz[3] + dz[0] * inv;
                R[4] -= w * dz[4];
            }
            finish(k, l, nd, own, R, inv);
        }
        // carry for the element above (or the top level): the weighted
        // one-sided z derivative of this element at its top level (row D[N]),
        // per column and field
        NH_FENCE();
        {
            const T wlo = T(slev[N * 5 + 3]);
            for (int t = tid; t < 6 * NCOL; t += NT) {
                const int c = t % NCOL, f = t / NCOL;
                const int off = S::addr(N + c % TX, N + c / TX);
                T v[N1], acc = T(0);
#pragma unroll
                for (int m = 0; m < N1; ++m) {
                    const int sm = (m == 0) ? sbot : (m == N ? stop : mid_slot(m));
                    v[m] = (f == 5) ? (T(slev[m * 5]) + planes[sm + off + 5 * FS]) * planes[sm + off + 3 * FS]
                                    : planes[sm + off + f * FS];
                }
#pragma unroll
                for (int m = 0; m < N1; ++m) acc += sD[N * N1 + m] * v[m];
                scarry[(ez + 1) & 1][t] = wlo * (h2 * acc);
            }
        }
        if (ez + 1 < p.nelz) fill_stlev((ez + 1) * N);
        __syncthreads();
    }
    // top level: only the contribution of the element below (lanes of level
    // 0 take it; level data of the last element's top row)
    if (l == 0) {
        const int ktop = p.nz - 1;
        const int stop = (p.nelz & 1) ? S::B4 : S::B0;
        NodeIn nd;
        prefetch(ktop, nd);
        const T *own = planes + stop + noff;
        T R[5], inv;
        horizontal(own, T(slev[N * 5]), R, inv);
        const T *cry = scarry[p.nelz & 1] + col;
        const T w = own[3 * FS];
        R[0] -= cry[5 * NCOL];
        R[1] -= w * cry[NCOL];
        R[2] -= w * cry[2 * NCOL];
        R[3] -= w * cry[3 * NCOL] + cry[0] * inv;
        R[4] -= w * cry[4 * NCOL];
        finish(ktop, N, nd, own, R, inv);
    }
#undef NH_FENCE
#undef NH_PIN
}

template <int N, int AX, int AY, typename T>
__global__ void __launch_bounds__((ClsShape<N, AX, AY>::NT)) stage_kernel_cls(const StageParams p)
{
    stage_body_cls<N, AX, AY, T>(p, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x);
}

template <int N, int AX, int AY, typename T>
__global__ void __launch_bounds__((ClsShape<N, AX, AY>::NT))
stage_kernel_cls_batched(const StageParams *__restrict__ P, const int2 *__restrict__ work, const XcdLists xl)
{
    const int i = xcd_item(xl, blockIdx.x);
    if (i < 0) return;
    const int2 it = work[i];
    stage_body_cls<N, AX, AY, T>(P[it.x], it.y, threadIdx.x);
}

// Persistent batched forms: a grid of at most one workgroup per CU, each
// workgroup taking (instance, tile) items in order from its own XCD's list,
// then from the other lists once its own is exhausted (next_item), until
// every list is exhausted -- every workgroup reaches the exit.  The counters
// are zeroed by a fill kernel before the launch (inside the captured graph).
template <int N, int AX, int AY, typename T>
__global__ void __launch_bounds__((StageShape<N, AX, AY>::NT))
stage_kernel_persist(const StageParams *__restrict__ P, const int2 *__restrict__ work, const XcdLists xl,
                     int *counter)
{
    __shared__ int item;
    int tried = 0;
    const int home = blockIdx.x & (kXcds - 1);
    for (;;) {
        if (threadIdx.x == 0) item = next_item(xl, counter, home, tried);
        __syncthreads();
        // uniform across the workgroup: readfirstlane lets the compiler keep
        // the item's descriptor in scalar registers
        const int it = __builtin_amdgcn_readfirstlane(item);
        __syncthreads();
        if (it < 0) break;
        // the thread index is passed laundered, so that per-thread arithmetic
        // of the body is not hoisted out of the item loop (and held in
        // registers across items)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int2 w = work[it];
        stage_body<N, AX, AY, T>(P[w.x], w.y, tid);
        __syncthreads();
    }
}

template <int N, int AX, int AY, typename T>
__global__ void __launch_bounds__((ClsShape<N, AX, AY>::NT))
stage_kernel_cls_persist(const StageParams *__restrict__ P, const int2 *__restrict__ work, const XcdLists xl,
                         int *counter)
{
    __shared__ int item;
    int tried = 0;
    const int home = blockIdx.x & (kXcds - 1);
    for (;;) {
        if (threadIdx.x == 0) item = next_item(xl, counter, home, tried);
        __syncthreads();
        // uniform across the workgroup: readfirstlane lets the compiler keep
        // the item's descriptor in scalar registers
        const int it = __builtin_amdgcn_readfirstlane(item);
        __syncthreads();
        if (it < 0) break;
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int2 w = work[it];
        stage_body_cls<N, AX, AY, T>(P[w.x], w.y, tid);
        __syncthreads();
    }
}

__global__ void zero_ints_kernel(int *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// Tile shapes per order (AX x AY elements), three per order.  Variant 0 uses
// rows of 32 (or 30) lattice columns so that each half-wave's stencil reads
// cover one contiguous 256-byte LDS row (bank-conflict free); variant 1 is a
// squarer ~16 x 16 tile with a smaller halo; variant 2 a third shape (order 4:
// variant 0's tile in the node-class form).
#define NH_TILE_CASES(X)    \
    X(2, 16, 4, 8, 8, 16, 8) \
    X(3, 10, 3, 5, 5, 8, 4)  \
    X(4, 8, 2, 4, 4, 8, 2)   \
    X(5, 6, 1, 3, 2, 4, 2)   \
    X(6, 4, 1, 2, 2, 3, 1)

void stage_tile(int N, int variant, int *tx, int *ty)
{
    switch (N) {
#define NH_TILE(NN, AX0, AY0, AX1, AY1, AX2, AY2)                          \
    case NN:                                                               \
        *tx = (variant == 1 ? AX1 : (variant == 2 ? AX2 : AX0)) * NN;      \
        *ty = (variant == 1 ? AY1 : (variant == 2 ? AY2 : AY0)) * NN;      \
        return;
        NH_TILE_CASES(NH_TILE)
#undef NH_TILE
    default: *tx = *ty = 0;
    }
}

template <int N, int AX, int AY>
static void launch_cls(int precision, const StageParams &p, hipStream_t s)
{
    const dim3 grid(p.ntx * p.nty), block(ClsShape<N, AX, AY>::NT);
    if (precision == 0)
        hipLaunchKernelGGL((stage_kernel_cls<N, AX, AY, double>), grid, block, 0, s, p);
    else
        hipLaunchKernelGGL((stage_kernel_cls<N, AX, AY, float>), grid, block, 0, s, p);
}

template <int N, int AX, int AY>
static void launch_cls_batched(int precision, const StageParams *P, const int2 *work, const XcdLists &xl,
                               int maxlen, hipStream_t s)
{
    const dim3 grid(kXcds * maxlen), block(ClsShape<N, AX, AY>::NT);
    if (precision == 0)
        hipLaunchKernelGGL((stage_kernel_cls_batched<N, AX, AY, double>), grid, block, 0, s, P, work, xl);
    else
        hipLaunchKernelGGL((stage_kernel_cls_batched<N, AX, AY, float>), grid, block, 0, s, P, work, xl);
}

template <int N, int AX, int AY>
static void launch_one(int precision, const StageParams &p, hipStream_t s)
{
    const dim3 grid(p.ntx * p.nty), block(StageShape<N, AX, AY>::NT);
    if (precision == 0)
        hipLaunchKernelGGL((stage_kernel<N, AX, AY, double>), grid, block, 0, s, p);
    else
        hipLaunchKernelGGL((stage_kernel<N, AX, AY, float>), grid, block, 0, s, p);
}

template <int N, int AX, int AY>
static void launch_batched_one(int precision, const StageParams *P, const int2 *work, const XcdLists &xl, int maxlen,
                               int *counter, int persist_grid, hipStream_t s)
{
    const dim3 block(StageShape<N, AX, AY>::NT);
    const int nitems = xl.off[kXcds];
    if (counter) {
        const dim3 grid(nitems < persist_grid ? nitems : persist_grid);
        if (precision == 0)
            hipLaunchKernelGGL((stage_kernel_persist<N, AX, AY, double>), grid, block, 0, s, P, work, xl, counter);
        else
            hipLaunchKernelGGL((stage_kernel_persist<N, AX, AY, float>), grid, block, 0, s, P, work, xl, counter);
        return;
    }
    const dim3 grid(kXcds * maxlen);
    if (precision == 0)
        hipLaunchKernelGGL((stage_kernel_batched<N, AX, AY, double>), grid, block, 0, s, P, work, xl);
    else
        hipLaunchKernelGGL((stage_kernel_batched<N, AX, AY, float>), grid, block, 0, s, P, work, xl);
}

template <int N, int AX, int AY>
static void launch_cls_batched_any(int precision, const StageParams *P, const int2 *work, const XcdLists &xl,
                                   int maxlen, int *counter, int persist_grid, hipStream_t s)
{
    const dim3 block(ClsShape<N, AX, AY>::NT);
    const int nitems = xl.off[kXcds];
    if (counter) {
        const dim3 grid(nitems < persist_grid ? nitems : persist_grid);
        if (precision == 0)
            hipLaunchKernelGGL((stage_kernel_cls_persist<N, AX, AY, double>), grid, block, 0, s, P, work, xl, counter);
        else
            hipLaunchKernelGGL((stage_kernel_cls_persist<N, AX, AY, float>), grid, block, 0, s, P, work, xl, counter);
        return;
    }
    launch_cls_batched<N, AX, AY>(precision, P, work, xl, maxlen, s);
}

hipError_t launch_stage_batched(int N, int precision, int variant, const StageParams *P, const int2 *work,
                                const XcdLists &xl, int maxlen, int *counter, int persist_grid, hipStream_t s)
{
    if (xl.off[0] != 0 || maxlen < 1) return hipErrorInvalidValue;
    for (int x = 0; x < kXcds; ++x)
        if (xl.off[x + 1] < xl.off[x] || xl.off[x + 1] - xl.off[x] > maxlen) return hipErrorInvalidValue;
    switch (N) {
#define NH_LAUNCHB(NN, AX0, AY0, AX1, AY1, AX2, AY2)                                                          \
    case NN:                                                                                                  \
        if (variant == 1)                                                                                     \
            launch_batched_one<NN, AX1, AY1>(precision, P, work, xl, maxlen, counter, persist_grid, s);       \
        else if (variant == 2 && NN == 4)                                                                     \
            launch_cls_batched_any<4, 8, 2>(precision, P, work, xl, maxlen, counter, persist_grid, s);        \
        else if (variant == 2)                                                                                \
            launch_batched_one<NN, AX2, AY2>(precision, P, work, xl, maxlen, counter, persist_grid, s);       \
        else launch_batched_one<NN, AX0, AY0>(precision, P, work, xl, maxlen, counter, persist_grid, s);      \
        break;
        NH_TILE_CASES(NH_LAUNCHB)
#undef NH_LAUNCHB
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stage(int N, int precision, int variant, const StageParams &p, hipStream_t s)
{
    switch (N) {
#define NH_LAUNCH(NN, AX0, AY0, AX1, AY1, AX2, AY2)                    \
    case NN:                                                           \
        if (variant == 1) launch_one<NN, AX1, AY1>(precision, p, s);   \
        else if (variant == 2 && NN == 4) launch_cls<4, 8, 2>(precision, p, s); \
        else if (variant == 2) launch_one<NN, AX2, AY2>(precision, p, s); \
        else launch_one<NN, AX0, AY0>(precision, p, s);                \
        break;
        NH_TILE_CASES(NH_LAUNCH)
#undef NH_LAUNCH
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Forcing of fields other than theta' (manufactured solutions):
// out += c ((1 - lam) f0 + lam f1), elementwise, except where the no-flux
// condition fixes the tendency of that field (u on x-walls, v on y-walls,
// w at z = 0 and z = H).
__global__ void add_forcing_kernel(WallParams wp, int field, double c, const double *__restrict__ f0,
                                   const double *__restrict__ f1, double lam, double *__restrict__ out)
{
    const long n = (long)wp.nx * wp.ny * wp.nz;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(i % wp.nx), iy = (int)((i / wp.nx) % wp.ny), iz = (int)(i / ((long)wp.nx * wp.ny));
        bool wall = false;
        if (field == 1) wall = !wp.perx && (ix == 0 || ix == wp.nx - 1);
        if (field == 2) wall = !wp.pery && (iy == 0 || iy == wp.ny - 1);
        if (field == 3) wall = (iz == 0 || iz == wp.nz - 1);
        if (!wall) out[i] += c * ((1.0 - lam) * f0[i] + lam * f1[i]);
    }
}

// ---------------------------------------------------------------- DSS / scatter
// Elements sharing lattice index `i` along one direction, ascending element
// index: up to two (element, local position) pairs.
__device__ __forceinline__ int owners(int i, int N, int nel, int n, int per, int *e, int *loc)
{
    const int eq = i / N, r = i % N;
    if (r != 0) { e[0] = eq; loc[0] = r; return 1; }
    int c = 0;
    int el = eq - 1, er = eq;
    if (el < 0) el = per ? nel - 1 : -1;
    if (er >= nel) er = per ? 0 : -1;
    (void)n;
    if (el >= 0 && er >= 0 && el > er) {
        e[c] = er; loc[c] = 0; ++c;
        e[c] = el; loc[c] = N; ++c;
    } else {
        if (el >= 0) { e[c] = el; loc[c] = N; ++c; }
        if (er >= 0) { e[c] = er; loc[c] = 0; ++c; }
    }
    return c;
}

__global__ void dss_kernel(GeomParams g, int nfields, int mode, const double *__restrict__ E,
                           double *__restrict__ out)
{
    const long U = (long)g.nx * g.ny * g.nz;
    const int N1 = g.N + 1;
    const long np = (long)N1 * N1 * N1;
    const long L = (long)g.nelx * g.nely * g.nelz * np;
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < U; I += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(I % g.nx), iy = (int)((I / g.nx) % g.ny), iz = (int)(I / ((long)g.nx * g.ny));
        int ex[2], lx[2], ey[2], ly[2], ez[2], lz[2];
        const int cxn = owners(ix, g.N, g.nelx, g.nx, g.perx, ex, lx);
        const int cyn = owners(iy, g.N, g.nely, g.ny, g.pery, ey, ly);
        const int czn = owners(iz, g.N, g.nelz, g.nz, 0, ez, lz);
        for (int f = 0; f < nfields; ++f) {
            double acc = 0.0;
            for (int c = 0; c < czn; ++c)
                for (int b = 0; b < cyn; ++b)
                    for (int a = 0; a < cxn; ++a) {
                        const long e = ex[a] + (long)g.nelx * (ey[b] + (long)g.nely * ez[c]);
                        double v = E[f * L + e * np + lx[a] + N1 * (ly[b] + N1 * lz[c])];
                        if (mode == 1) {
                            const double J = g.hx[ex[a]] * g.hy[ey[b]] * g.hz[ez[c]] / 8.0;
                            v = g.wlgl[lx[a]] * g.wlgl[ly[b]] * g.wlgl[lz[c]] * J * v;
                        }
                        acc += v;
                    }
            if (mode == 1) acc /= g.mx[ix] * g.my[iy] * g.mz[iz];
            out[f * U + I] = acc;
        }
    }
}

__global__ void scatter_kernel(GeomParams g, int nfields, const double *__restrict__ Uv,
                               double *__restrict__ E)
{
    const long U = (long)g.nx * g.ny * g.nz;
    const int N1 = g.N + 1;
    const long np = (long)N1 * N1 * N1;
    const long L = (long)g.nelx * g.nely * g.nelz * np;
    for (long m = blockIdx.x * (long)blockDim.x + threadIdx.x; m < L; m += (long)gridDim.x * blockDim.x) {
        const long e = m / np;
        const int loc = (int)(m % np);
        const int i = loc % N1, j = (loc / N1) % N1, k = loc / (N1 * N1);
        const int ex = (int)(e % g.nelx), ey = (int)((e / g.nelx) % g.nely), ez = (int)(e / ((long)g.nelx * g.nely));
        int ix = ex * g.N + i, iy = ey * g.N + j;
        const int iz = ez * g.N + k;
        if (g.perx && ix == g.nx) ix = 0;
        if (g.pery && iy == g.ny) iy = 0;
        const long I = ix + (long)g.nx * (iy + (long)g.ny * iz);
        for (int f = 0; f < nfields; ++f) E[f * L + m] = Uv[f * U + I];
    }
}

__global__ void mass_kernel(GeomParams g, double *__restrict__ M)
{
    const long U = (long)g.nx * g.ny * g.nz;
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < U; I += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(I % g.nx), iy = (int)((I / g.nx) % g.ny), iz = (int)(I / ((long)g.nx * g.ny));
        M[I] = g.mx[ix] * g.my[iy] * g.mz[iz];
    }
}

// Diagnostics: block partials [kDiagBlocks][8] then one block folds them in a
// fixed order (deterministic).
__global__ void __launch_bounds__(256) diag_partial_kernel(GeomParams g, const double *__restrict__ q,
                                                           double *__restrict__ part)
{
    const long U = (long)g.nx * g.ny * g.nz;
    double s_m = 0, mu = 0, mv = 0, mw = 0, tmin = INFINITY, tmax = -INFINITY, s_t = 0, bad = 0;
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < U; I += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(I % g.nx), iy = (int)((I / g.nx) % g.ny), iz = (int)(I / ((long)g.nx * g.ny));
        const double M = g.mx[ix] * g.my[iy] * g.mz[iz];
        const double r = q[I], u = q[U + I], v = q[2 * U + I], w = q[3 * U + I], t = q[4 * U + I];
        s_m += M * r;
        s_t += M * t;
        mu = fmax(mu, fabs(u));
        mv = fmax(mv, fabs(v));
        mw = fmax(mw, fabs(w));
        tmin = fmin(tmin, t);
        tmax = fmax(tmax, t);
        bad += (double)(!isfinite(r)) + !isfinite(u) + !isfinite(v) + !isfinite(w) + !isfinite(t);
    }
    __shared__ double sh[8][256];
    const int t = threadIdx.x;
    sh[0][t] = s_m; sh[1][t] = mu; sh[2][t] = mv; sh[3][t] = mw;
    sh[4][t] = tmin; sh[5][t] = tmax; sh[6][t] = s_t; sh[7][t] = bad;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sh[0][t] += sh[0][t + h];
            sh[1][t] = fmax(sh[1][t], sh[1][t + h]);
            sh[2][t] = fmax(sh[2][t], sh[2][t + h]);
            sh[3][t] = fmax(sh[3][t], sh[3][t + h]);
            sh[4][t] = fmin(sh[4][t], sh[4][t + h]);
            sh[5][t] = fmax(sh[5][t], sh[5][t + h]);
            sh[6][t] += sh[6][t + h];
            sh[7][t] += sh[7][t + h];
        }
        __syncthreads();
    }
    if (t < 8) part[blockIdx.x * 8 + t] = sh[t][0];
}

__global__ void __launch_bounds__(64) diag_final_kernel(const double *__restrict__ part, int nb,
                                                        double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double r[8] = {0, 0, 0, 0, INFINITY, -INFINITY, 0, 0};
    for (int b = 0; b < nb; ++b) {
        const double *pp = part + b * 8;
        r[0] += pp[0];
        r[1] = fmax(r[1], pp[1]);
        r[2] = fmax(r[2], pp[2]);
        r[3] = fmax(r[3], pp[3]);
        r[4] = fmin(r[4], pp[4]);
        r[5] = fmax(r[5], pp[5]);
        r[6] += pp[6];
        r[7] += pp[7];
    }
    for (int i = 0; i < 8; ++i) out[i] = r[i];
}

static int grid_for(long n, int block)
{
    long g = (n + block - 1) / block;
    if (g > 65535) g = 65535;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_add_forcing(const WallParams &wp, int field, double c, const double *f0, const double *f1,
                              double lam, double *out, hipStream_t s)
{
    const long n = (long)wp.nx * wp.ny * wp.nz;
    hipLaunchKernelGGL(add_forcing_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, wp, field, c, f0, f1, lam,
                       out);
    return hipGetLastError();
}

hipError_t launch_dss(const GeomParams &g, int nfields, int mode, const double *E, double *out,
                      hipStream_t s)
{
    const long U = (long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(dss_kernel, dim3(grid_for(U, 256)), dim3(256), 0, s, g, nfields, mode, E, out);
    return hipGetLastError();
}

hipError_t launch_scatter(const GeomParams &g, int nfields, const double *Uv, double *E, hipStream_t s)
{
    const long N1 = g.N + 1;
    const long L = (long)g.nelx * g.nely * g.nelz * N1 * N1 * N1;
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(L, 256)), dim3(256), 0, s, g, nfields, Uv, E);
    return hipGetLastError();
}

hipError_t launch_mass(const GeomParams &g, double *M, hipStream_t s)
{
    const long U = (long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(mass_kernel, dim3(grid_for(U, 256)), dim3(256), 0, s, g, M);
    return hipGetLastError();
}

hipError_t launch_diag(const GeomParams &g, const double *q, double *partials, double *out8, hipStream_t s)
{
    hipLaunchKernelGGL(diag_partial_kernel, dim3(kDiagBlocks), dim3(256), 0, s, g, q, partials);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, partials, kDiagBlocks, out8);
    return hipGetLastError();
}

}  // namespace nh
