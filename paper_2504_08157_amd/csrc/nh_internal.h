// Internal declarations shared by the host layer and the gfx950 kernels of
// libnhsem.  Not part of the public ABI (see include/nhsem.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nh {

constexpr int kMaxN = 6;
constexpr int kMaxN1 = kMaxN + 1;
// per-level table row: rho0 theta0 p0 dtheta0/dz tau wlo whi 1/rho0 1/theta0 pad
constexpr int kLevW = 10;
constexpr int kNF = 5;     // prognostic fields rho', u, v, w, theta'
constexpr int kDiagBlocks = 512;
constexpr int kEosTerms = 14;  // binomial-series terms of the EOS perturbation

// Arguments of one fused RHS / SSP-RK stage launch.
//   out = a * qn + b * qs + c * R(qs)
// (a = b = 0, c = 1 evaluates the right-hand side alone).
struct StageParams {
    const double *qs;      // [5][U] state the tendency is evaluated at
    const double *qn;      // [5][U] state at the start of the step (read iff a != 0)
    double *out;           // [5][U]
    double a, b, c;
    const double *gx;      // [n_x][2N+1] DSS'd first-derivative stencil along x
    const double *gy;      // [n_y][2N+1]
    const float *gxf;      // FP32 copies for the mixed-precision path
    const float *gyf;
    const double *cfx;     // [n_x][2] the x average written per element: weight of the
                           // element the node ends (local index N), of the one it starts or
                           // lies inside
    const double *cfy;     // [n_y][2]
    const double *lev;     // [n_z][kLevW]
    const double *hz2;     // [nel_z] 2 / h_z of each element layer
    const double *cst;     // [kCst]: D (row-major, (N+1)^2) then the EOS series
    const double *hq0;     // theta' forcing snapshot below t (or null)
    const double *hq1;     // theta' forcing snapshot above t
    double hlam;           // interpolation weight of hq1
    int nx, ny, nz, nelz;
    int perx, pery;
    int ntx, nty;
    double fcor, g, gamma;
    int stream;            // stream q^n, the heating and the result past the caches
};

// States of at least this many bytes per array are streamed past the
// caches by the stage and hyper-diffusion kernels (twice the 256 MB
// last-level cache: below it the next launch re-reads what this one wrote
// from that cache).
constexpr size_t kStreamBytes = size_t(512) << 20;

// Layout of the constant table StageParams::cst.
constexpr int kCstD = 0;                          // D[i][j] = h_j'(xi_i), (N+1)^2 entries
constexpr int kCstEos = kMaxN1 * kMaxN1;          // C(gamma, n+1), n = 0..kEosTerms-1
constexpr int kCst = kCstEos + kEosTerms;

struct GeomParams {
    int N, nelx, nely, nelz, nx, ny, nz, perx, pery;
    const double *mx, *my, *mz;   // 1D assembled masses per lattice index
    const double *wlgl;           // [N+1] LGL weights
    const double *hx, *hy, *hz;   // element sizes
};

hipError_t launch_stage(int N, int precision, int variant, const StageParams &p, hipStream_t s);
// Work items of one order group, split into one list per XCD: list x is
// work[off[x] .. off[x + 1]), x = 0 .. kXcds - 1 (workgroup b of a launch
// runs on XCD b mod kXcds).
constexpr int kXcds = 8;
struct XcdLists {
    int off[kXcds + 1];
};
// Grouped stage launch over the (instance, tile) items of `xl`; with device
// counters (kXcds, zeroed beforehand) the persistent form with at most
// persist_grid workgroups, else one workgroup per item (kXcds * maxlen
// workgroups, maxlen the longest list).
hipError_t launch_stage_batched(int N, int precision, int variant, const StageParams *P, const int2 *work,
                                const XcdLists &xl, int maxlen, int *counter, int persist_grid, hipStream_t s);
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
struct WallParams {
    int nx, ny, nz, perx, pery;
};

// ---- 1D-IMEX (HEVI)
struct HeviParams {
    int nx, ny, nz, N;
    const double *lev;   // [n_z][kLevW]
    const double *gz;    // [n_z][2N+1] DSS'd vertical derivative stencil
    double gamma, g;
};

// L_v x on levels k0 .. k1-1 of lattice column col (the vertical operator
// of the HEVI step, Sec. 2.3): a walk up the column that keeps the
// (2N+1)-level window of the stencil inputs rho0 w and
// p'_L = gamma p0 (rho'/rho0 + theta'/theta0) in registers, so every value of
// x is loaded once per walk.  x holds rho' at element offset 0, w at xw and
// theta' at xt; levels outside the column count as zero.  For each level k
// the callback out(k, l0, l3, l4, r, w, t) receives the rho', w and theta'
// rows of L_v x (the w row zero at z = 0 and z = H) and x's own values.
template <int N, typename Out>
__device__ __forceinline__ void lv_walk(const HeviParams &h, long col, int k0, int k1, const double *x, long xw,
                                        long xt, Out &&out)
{
    constexpr int NC = 2 * N + 1;
    const long nxy = (long)h.nx * h.ny;
    const int nz = h.nz;
    double ta[NC], tb[NC], rr[N + 1], ww[N + 1], th[N + 1];
    auto load = [&](int kk, double &a, double &bb, double &r, double &w, double &t) {
        a = bb = r = w = t = 0.0;
        if (kk >= 0 && kk < nz) {
            const double *L = h.lev + (long)kk * kLevW;
            const long J = col + (long)kk * nxy;
            r = x[J];
            w = x[xw + J];
            t = x[xt + J];
            a = L[0] * w;
            bb = h.gamma * L[2] * (r * L[7] + t * L[8]);
        }
    };
    // window slots 0 .. 2N-1: levels k0-N .. k0+N-1; rr/ww/th slots 0 .. N-1: levels k0 .. k0+N-1
    double u0, u1, u2;
#pragma unroll
    for (int o = 0; o < N; ++o) load(k0 - N + o, ta[o], tb[o], u0, u1, u2);
#pragma unroll
    for (int j = 0; j < N; ++j) load(k0 + j, ta[N + j], tb[N + j], rr[j], ww[j], th[j]);
    for (int k = k0; k < k1; ++k) {
        load(k + N, ta[2 * N], tb[2 * N], rr[N], ww[N], th[N]);
        const double *L = h.lev + (long)k * kLevW;
        const double *G = h.gz + (long)k * NC;
        double d_rw = 0.0, d_pl = 0.0;
#pragma unroll
        for (int o = 0; o < NC; ++o) {
            d_rw += G[o] * ta[o];
            d_pl += G[o] * tb[o];
        }
        const double l3 = (k == 0 || k == nz - 1) ? 0.0 : -d_pl * L[7] - h.g * rr[0] * L[7];
        out(k, -d_rw, l3, -ww[0] * L[3], rr[0], ww[0], th[0]);
#pragma unroll
        for (int o = 0; o < 2 * N; ++o) { ta[o] = ta[o + 1]; tb[o] = tb[o + 1]; }
#pragma unroll
        for (int j = 0; j < N; ++j) { rr[j] = rr[j + 1]; ww[j] = ww[j + 1]; th[j] = th[j + 1]; }
    }
}

struct GmresArgs {
    const double *b;     // [5][U] right-hand sides
    const double *x0;    // [3][U] initial guess of (rho', w, theta') or null (x0 = b)
    double *x;           // [5][U] solution
    double alpha;        // A = I - alpha L_v
    double rtol;
    int restart, max_restarts;
    int *iters;          // [n_x n_y] Arnoldi steps per column (negative: not converged), or null
    int schur;           // 1: solve the Schur complement in w (restart kGmresRegM only)
    int pick;            // with x0: per column, start from x0 or from b, whichever has the smaller residual
    const int *gate;     // device flag: the launch does nothing while it is 0 (null: always runs)
};

constexpr int kMaxComb = 6;
struct LinComb {
    const double *src[kMaxComb];
    double c[kMaxComb];
};

size_t gmres_lds_bytes(int nz, int N, int restart);
// y = L_v x on [5][U]; with uv false the u and v rows of y are left untouched
hipError_t launch_lv_apply(const HeviParams &h, const double *x, double *y, hipStream_t s, bool uv = true);
// y (fields 0, 3, 4 of [5][U]) = b - x3 + alpha L_v x3: the residual of
// (I - alpha L_v) x = b at x3 = (rho', w, theta') as [3][U].
hipError_t launch_lv_resid(const HeviParams &h, double alpha, const double *b, const double *x3, double *y,
                           hipStream_t s);
hipError_t launch_axpy_multi(long n, const double *base, int nsrc, const LinComb &lc, double *out,
                             hipStream_t s);
hipError_t launch_gmres(const HeviParams &h, const GmresArgs &g, hipStream_t s);

// ---- tensor hyper-diffusion (box elements: one assembled 1D operator per direction)
struct HyperParams {
    int nx, ny, nz, N, perx, pery;
    int stream;                   // stream the output column past the caches
    const double *sx, *sy, *sz;   // [n_d][2N+1] operator rows per lattice position of each direction
};
// out = scale * (div tau grad) q on [5][U] (out += ... with accumulate); with
// wallmask the wall-normal velocity rows get no contribution
hipError_t launch_hd_laplace(const HyperParams &h, const double *q, double *out, double scale, bool accumulate,
                             bool wallmask, hipStream_t s);

// ---- 3D-IMEX: linear operator over all directions and the global GMRES
constexpr int kG3MaxRestart = 32;
struct L3Params {
    int nx, ny, nz, N, perx, pery;
    const double *gx, *gy;   // DSS'd x/y first-derivative stencils [n][2N+1]
    const double *lev;       // level table [n_z][kLevW]
    double gamma;
    HeviParams hv;           // the vertical part (L_v)
};
// Device-resident state of one global GMRES solve: the Hessenberg problem,
// the coefficients of the next vector combination and the control flags
// that gate the launches queued ahead of them.
struct G3State {
    double H[(kG3MaxRestart + 1) * kG3MaxRestart];   // rotated Hessenberg, H[i kG3MaxRestart + j]
    double cs[kG3MaxRestart], sn[kG3MaxRestart], gv[kG3MaxRestart + 1];
    double hc[kG3MaxRestart + 1];     // current column after the first Gram-Schmidt pass
    double coef[kG3MaxRestart + 1];   // coefficients of the next combination
    double scale, one, zero, bn, relres;
    int go;      // the current cycle's Arnoldi process continues
    int pass2;   // the current column takes a second Gram-Schmidt pass
    int open;    // rtol not met yet
    int bzero;   // b = 0
    int ncols;   // columns of the current cycle
    int iters;   // Arnoldi steps so far
};
// What the host reads of the solve: written by the kernels into host-mapped
// memory, read once an event recorded after them has completed.
struct G3Status {
    int go, open, iters, pad;
    double relres;
};
struct G3Work {
    double *V;      // (restart + 1) Krylov vectors of 5U
    double *Z;      // restart preconditioned vectors (flexible GMRES)
    double *t;      // one 5U vector
    double *part;   // [35][1024] block partial sums, quantity-major
    G3State *state;                 // device
    G3Status *status_dev;           // host-mapped status, device address
    const volatile G3Status *status;  // the same, host address
    hipEvent_t ev[2];               // marks of the host's look-ahead
};
// out = a x + c L x on [5][U] (out may not alias x); with a gate (device
// flag) nothing is done while it is 0
hipError_t launch_l3(const L3Params &h, const double *x, double *out, double a, double c, hipStream_t s,
                     const int *gate = nullptr);
// (I - alpha L) x = b by restarted GMRES(m); iters = Arnoldi steps, relres =
// final ||b - A x|| / ||b||
// precond: right-precondition with the column systems (I - alpha L_v)
hipError_t gmres3d(const L3Params &h, const G3Work &w, double alpha, const double *b, const double *x0, double *x,
                   int m, int max_restarts, double rtol, bool precond, hipStream_t s, int *iters, double *relres);

// ---- RI-velocity diagnostic
constexpr int kRiMaxStrips = 4096;
struct RiParams {
    int nx, ny, nz, nstrips, nb;   // nb: chunks (workgroups) per level
    long U;
    const double *x, *y;           // lattice coordinates [n_x], [n_y]
    const double *mx, *my;         // assembled 1D masses
    double eps, xmid, ymid;        // strip width; centre of a level at rest
};
struct RiWork {
    double *cpart;   // [n_z][nb][3] centroid partial sums
    double *ssum;    // [n_z][nb][n_strips] strip partial sums
    int *scnt;       // [n_z][nb][n_strips] strip partial counts
    double *umax;    // [n_z][nb] partial maxima of the horizontal speed
};
size_t ri_lds_bytes(int nstrips);
hipError_t launch_ri(const RiParams &p, const double *q, bool center_given, double *center, double *ubar,
                     int *count, double *result, const double *z, const RiWork &w, hipStream_t s);

constexpr int kGmresRegM = 10;        // restart length of the register-basis GMRES
constexpr int kGmresRegSlots = 4;     // unknowns per lane it supports (3 n_z <= 256)
constexpr int kGmresSchurSlots = 2;   // Schur form: interior w levels up to 128

// ---- column MLP
constexpr int kMlpIn = 208;    // 198 features (195 residual values, 3 scalars) padded to a multiple of 16
constexpr int kMlpHid = 256;
constexpr int kMlpOut = 256;   // 3 fields x 65 canonical levels, padded to a multiple of 64
constexpr int kMlpMaxPasses = 4;   // network applications per initial guess, at most
constexpr int kMlpSlices = 16;  // batch slices of the weight-gradient GEMMs
constexpr int kMlpNC = 65;     // canonical levels: LGL nodes of 16 order-4 elements
constexpr int kMlpNF = 3 * kMlpNC;
constexpr int kMlpLossBlocks = 256;
constexpr int kMlpColRows = 64;    // rows per partial of the bias-gradient column sums

struct MlpColParams {
    int nx, ny, nz;
    const double *z;     // [n_z] lattice levels
    const double *lev;   // level table [n_z][kLevW] (rho0, theta0, p0, ...)
    double alpha, gamma;
    double zc[kMlpNC];   // canonical normalised heights in [0, 1]
};

struct MlpNet {
    long nparam;
    float *master, *grad, *m, *v;  // FP32 [nparam]
    void *half;                    // FP16 [nparam]
    const void *wh[4];             // FP16 weights inside `half` (W1, W2, W3, linear bypass S)
    float *b[3];                   // FP32 biases inside `master`
    float *gw[4], *gb[3];          // gradients inside `grad`
    float *Z1, *Z2, *Y, *dY, *dH, *dZ, *part, *loss;
    float *part_k;                 // [kMlpSlices][kMlpOut][kMlpIn] split-K partials
    void *H1, *H2;                 // FP16 activations
    void *feat;                    // FP16 [max_batch][kMlpIn]
    double *scale;                 // [max_batch] column scales
};

// FP16 weights and FP32 biases of the network, by value for kernels
struct MlpWeights {
    const _Float16 *W[4];   // W1 [256][208], W2 [256][256], W3 [256][256], bypass S [256][208]
    const float *bias[3];
};

// x0 = base + the network's correction for the residual of the start base,
// columns col0 .. col0 + ncol - 1, in one kernel: base = b ([5][U]) for the
// first pass, or the previous guess ([3][U], base3; x0 may be base) for a
// refinement pass.  With lb the residual is rscale * lb (lb = L_v b,
// rscale = alpha; or lb = the residual, rscale = 1); with lb null it is
// computed in the kernel from base and b (n_z <= mlp_fused_max_nz()).
hipError_t launch_mlp_infer(const MlpColParams &p, const HeviParams &hp, const MlpNet &net, const double *base,
                            bool base3, const double *b, const double *lb, double rscale, long col0, long ncol,
                            double *x0, hipStream_t s);
int mlp_fused_max_nz();
// features (and, with x, targets x - base) of the residual rscale * lb of
// the start base: b ([5][U]) with lb = L_v b, rscale = alpha, or a previous
// guess ([3][U], base3) with lb its residual, rscale = 1
hipError_t launch_mlp_features(const MlpColParams &p, const double *base, bool base3, const double *lb,
                               double rscale, const double *x, long col0, long ncol, void *feat, double *scale,
                               float *tgt, hipStream_t s);
hipError_t launch_mlp_guess(const MlpColParams &p, const double *b, long col0, long ncol, const float *y,
                            const double *scale, double *x0, hipStream_t s);
hipError_t mlp_forward(const MlpNet &net, int M, const void *X, hipStream_t s, bool keep_z = true);
hipError_t mlp_backward(const MlpNet &net, int M, const void *X, const float *dY, hipStream_t s);
hipError_t mlp_loss_grad(const MlpNet &net, int M, const float *T, float *loss, hipStream_t s);
// Adam step; wd > 0 adds decoupled weight decay on the hidden path's
// parameters (W1, b1, W2, b2, W3, b3), not on the bypass S
hipError_t mlp_adam(const MlpNet &net, float lr, float b1, float b2, float eps, int step, float wd, hipStream_t s);
hipError_t mlp_sync_half(const MlpNet &net, hipStream_t s);

hipError_t launch_add_forcing(const WallParams &wp, int field, double c, const double *f0, const double *f1,
                              double lam, double *out, hipStream_t s);
hipError_t launch_dss(const GeomParams &g, int nfields, int mode, const double *E, double *out,
                      hipStream_t s);
hipError_t launch_scatter(const GeomParams &g, int nfields, const double *Uv, double *E,
                          hipStream_t s);
hipError_t launch_mass(const GeomParams &g, double *M, hipStream_t s);
hipError_t launch_diag(const GeomParams &g, const double *q, double *partials, double *out8,
                       hipStream_t s);
void stage_tile(int N, int variant, int *tx, int *ty);
constexpr int kTileVariants = 3;

}  // namespace nh
