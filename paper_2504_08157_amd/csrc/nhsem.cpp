// Host layer of libnhsem: the C ABI declared in include/nhsem.h.
//
// Set-up work (basis, lattice numbering, per-direction DSS weights and
// derivative stencils, reference-state tables) runs once on the host, as in
// the paper's workflow where the grid and initial conditions are prepared on
// the CPU before the time loop moves to the GPU (Sec. 3.2).  Every step of
// the time loop runs in the gfx950 kernels of nh_kernels.hip.
#include "nh_internal.h"
#include "nhsem.h"

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

using namespace nh;

struct nh_ctx {
    int N, nel[3], per[2], n[3], precision, tile;
    int64_t U, L;
    std::vector<double> xe, ye, ze;
    std::vector<double> xi, w, D;       // LGL basis
    std::vector<double> lx, ly, lz;     // lattice coordinates
    std::vector<double> m1[3];          // assembled 1D masses
    std::vector<double> G[3];           // [n][2N+1] DSS'd derivative stencils
    std::vector<double> levtab;         // [n_z][kLevW]
    nh_physics phys;
    bool have_ref;
    hipStream_t stream;
    // workspace carve
    char *ws;
    size_t ws_bytes;
    double *q[3];
    double *gx, *gy, *lev, *hz2, *mx, *my, *mz, *hx, *hy, *hz, *wl, *cst, *diag_part, *diag_out;
    float *gxf, *gyf;
    // forcing
    int nsnap[kNF];
    std::vector<double> tsnap[kNF];
    const double *snap[kNF];
    // error state
    bool sticky;
    std::string err;
};

namespace {

thread_local std::string g_last_global_error;

nh_status fail(nh_ctx *c, nh_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (code == NH_EHIP) c->sticky = true;
    } else {
        g_last_global_error = buf;
    }
    return code;
}

#define HIPCHK(c, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail((c), NH_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---- LGL basis, computed here independently of any other component.
// Nodes: Newton iteration on q(x) = x P_N(x) - P_{N-1}(x), whose zeros in
// (-1, 1) are the roots of P_N' (since (1-x^2) P_N' = N (P_{N-1} - x P_N)),
// started from Chebyshev-Gauss-Lobatto points.  Weights 2/(N(N+1) P_N^2).
// Derivative matrix from barycentric weights: D_ij = (lam_j/lam_i)/(x_i-x_j),
// D_ii = -sum_{j != i} D_ij.
void legendre_pair(int N, double x, double *pn, double *pnm1)
{
    double a = 1.0, b = x;  // P_0, P_1
    if (N == 0) { *pn = 1.0; *pnm1 = 0.0; return; }
    for (int k = 2; k <= N; ++k) {
        const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    *pn = b;
    *pnm1 = a;
}

void lgl_basis(int N, std::vector<double> &xi, std::vector<double> &w, std::vector<double> &D)
{
    const int n1 = N + 1;
    xi.assign(n1, 0.0);
    w.assign(n1, 0.0);
    D.assign(n1 * n1, 0.0);
    for (int j = 0; j < n1; ++j) {
        double x = -cos(M_PI * j / N);
        if (j > 0 && j < N) {
            for (int it = 0; it < 60; ++it) {
                double pn, pm;
                legendre_pair(N, x, &pn, &pm);
                // q = x P_N - P_{N-1};  q' = (N+1) P_N  (Legendre identity)
                const double dx = (x * pn - pm) / ((N + 1) * pn);
                x -= dx;
                if (fabs(dx) < 1e-16) break;
            }
        }
        xi[j] = x;
    }
    for (int j = 0; j < n1 / 2; ++j) {  // exact symmetry
        const double s = 0.5 * (xi[N - j] - xi[j]);
        xi[j] = -s;
        xi[N - j] = s;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int j = 0; j < n1; ++j) {
        double pn, pm;
        legendre_pair(N, xi[j], &pn, &pm);
        w[j] = 2.0 / (N * (N + 1.0) * pn * pn);
    }
    std::vector<double> lam(n1, 1.0);
    for (int j = 0; j < n1; ++j)
        for (int k = 0; k < n1; ++k)
            if (k != j) lam[j] *= (xi[j] - xi[k]);
    for (int i = 0; i < n1; ++i) {
        double s = 0.0;
        for (int j = 0; j < n1; ++j) {
            if (j == i) continue;
            D[i * n1 + j] = (lam[i] / lam[j]) / (xi[i] - xi[j]);
            s += D[i * n1 + j];
        }
        D[i * n1 + i] = -s;
    }
}

// Per-direction tables along one lattice line: coordinates, assembled 1D
// mass m(I) = sum_{e ∋ I} w_i h_e / 2, and the DSS'd first-derivative
// stencil G[I][N + o] (offset o in -N..N): the m-weighted average of the
// one-sided element derivatives (2/h_e) sum_l D_il f(e, l) of the elements
// sharing I.
void line_tables(int N, int nel, int periodic, const double *edges, const std::vector<double> &xi,
                 const std::vector<double> &w, const std::vector<double> &D, std::vector<double> &coord,
                 std::vector<double> &m1, std::vector<double> &G)
{
    const int n = nel * N + (periodic ? 0 : 1);
    const int nc = 2 * N + 1, n1 = N + 1;
    coord.assign(n, 0.0);
    m1.assign(n, 0.0);
    G.assign((size_t)n * nc, 0.0);
    for (int e = 0; e < nel; ++e) {
        const double h = edges[e + 1] - edges[e];
        for (int i = 0; i < n1; ++i) {
            int I = e * N + i;
            if (periodic) I %= n;
            m1[I] += w[i] * h / 2;
            if (i < N || (!periodic && e == nel - 1))
                coord[I] = (i == 0) ? edges[e] : (i == N ? edges[e + 1] : edges[e] + 0.5 * h * (xi[i] + 1.0));
        }
    }
    for (int e = 0; e < nel; ++e) {
        const double h = edges[e + 1] - edges[e];
        for (int i = 0; i < n1; ++i) {
            int I = e * N + i;
            if (periodic) I %= n;
            const double wt = (w[i] * h / 2) / m1[I];
            for (int l = 0; l < n1; ++l) {
                const int off = l - i;  // lattice offset of node l relative to node i
                G[(size_t)I * nc + N + off] += wt * (2.0 / h) * D[i * n1 + l];
            }
        }
    }
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t q[3], gx, gy, gxf, gyf, lev, hz2, mx, my, mz, hx, hy, hz, wl, cst, dpart, dout, total;
};

bool valid_desc(const nh_mesh_desc *m, std::string *why)
{
    if (!m) { *why = "null mesh descriptor"; return false; }
    if (m->order < 2 || m->order > kMaxN) { *why = "order must be in 2..6"; return false; }
    for (int d = 0; d < 3; ++d)
        if (m->nel[d] < 1 || m->nel[d] > (1 << 20)) { *why = "element counts must be >= 1"; return false; }
    if (m->precision != NH_FP64 && m->precision != NH_FP32_MIXED) { *why = "bad precision"; return false; }
    const double *e[3] = {m->xe, m->ye, m->ze};
    for (int d = 0; d < 3; ++d) {
        if (!e[d]) { *why = "null edge array"; return false; }
        for (int i = 0; i < m->nel[d]; ++i)
            if (!(e[d][i + 1] > e[d][i]) || !isfinite(e[d][i]) || !isfinite(e[d][i + 1])) {
                *why = "edges must be finite and strictly increasing";
                return false;
            }
    }
    if ((m->periodic[0] != 0 && m->periodic[0] != 1) || (m->periodic[1] != 0 && m->periodic[1] != 1)) {
        *why = "periodic flags must be 0 or 1";
        return false;
    }
    // kernels address one field with 32-bit byte offsets
    const int64_t nx = (int64_t)m->nel[0] * m->order + (m->periodic[0] ? 0 : 1);
    const int64_t ny = (int64_t)m->nel[1] * m->order + (m->periodic[1] ? 0 : 1);
    const int64_t nz = (int64_t)m->nel[2] * m->order + 1;
    if (nx * ny * nz * 8 >= ((int64_t)1 << 32)) { *why = "more than 2^29 unique nodes"; return false; }
    return true;
}

Layout layout_for(const nh_mesh_desc *m)
{
    const int N = m->order;
    const int64_t nx = (int64_t)m->nel[0] * N + (m->periodic[0] ? 0 : 1);
    const int64_t ny = (int64_t)m->nel[1] * N + (m->periodic[1] ? 0 : 1);
    const int64_t nz = (int64_t)m->nel[2] * N + 1;
    const int64_t U = nx * ny * nz;
    const int nc = 2 * N + 1;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    for (int i = 0; i < 3; ++i) L.q[i] = take(sizeof(double) * kNF * U);
    L.gx = take(sizeof(double) * nx * nc);
    L.gy = take(sizeof(double) * ny * nc);
    L.gxf = take(sizeof(float) * nx * nc);
    L.gyf = take(sizeof(float) * ny * nc);
    L.lev = take(sizeof(double) * nz * kLevW);
    L.hz2 = take(sizeof(double) * m->nel[2]);
    L.mx = take(sizeof(double) * nx);
    L.my = take(sizeof(double) * ny);
    L.mz = take(sizeof(double) * nz);
    L.hx = take(sizeof(double) * m->nel[0]);
    L.hy = take(sizeof(double) * m->nel[1]);
    L.hz = take(sizeof(double) * m->nel[2]);
    L.wl = take(sizeof(double) * (N + 1));
    L.cst = take(sizeof(double) * kCst);
    L.dpart = take(sizeof(double) * kDiagBlocks * 8);
    L.dout = take(sizeof(double) * 8);
    L.total = off;
    return L;
}

GeomParams geom(const nh_ctx *c)
{
    GeomParams g{};
    g.N = c->N;
    g.nelx = c->nel[0]; g.nely = c->nel[1]; g.nelz = c->nel[2];
    g.nx = c->n[0]; g.ny = c->n[1]; g.nz = c->n[2];
    g.perx = c->per[0]; g.pery = c->per[1];
    g.mx = c->mx; g.my = c->my; g.mz = c->mz;
    g.wlgl = c->wl;
    g.hx = c->hx; g.hy = c->hy; g.hz = c->hz;
    return g;
}

nh_status guard(const nh_ctx *c)
{
    if (!c) return fail(nullptr, NH_EINVAL, "null context");
    if (c->sticky) return NH_ESTATE;
    return NH_OK;
}

// Forcing snapshot pair and weight at time t (linear in time, clamped).
void forcing_at(const nh_ctx *c, int f, double t, const double **a, const double **b, double *lam)
{
    *a = *b = nullptr;
    *lam = 0.0;
    const int ns = c->nsnap[f];
    if (ns <= 0) return;
    const std::vector<double> &ts = c->tsnap[f];
    const double *base = c->snap[f];
    if (ns == 1 || t <= ts[0]) { *a = *b = base; return; }
    if (t >= ts[ns - 1]) { *a = *b = base + (size_t)(ns - 1) * c->U; return; }
    int k = 0;
    while (k + 1 < ns - 1 && t >= ts[k + 1]) ++k;
    *a = base + (size_t)k * c->U;
    *b = base + (size_t)(k + 1) * c->U;
    *lam = (t - ts[k]) / (ts[k + 1] - ts[k]);
}

StageParams stage_params(const nh_ctx *c, double t, const double *qs, const double *qn, double *out,
                         double a, double b, double cc)
{
    StageParams p{};
    p.qs = qs; p.qn = qn; p.out = out;
    p.a = a; p.b = b; p.c = cc;
    p.gx = c->gx; p.gy = c->gy; p.gxf = c->gxf; p.gyf = c->gyf;
    p.lev = c->lev; p.hz2 = c->hz2; p.cst = c->cst;
    forcing_at(c, 4, t, &p.hq0, &p.hq1, &p.hlam);
    p.nx = c->n[0]; p.ny = c->n[1]; p.nz = c->n[2]; p.nelz = c->nel[2];
    p.perx = c->per[0]; p.pery = c->per[1];
    int tx, ty;
    stage_tile(c->N, c->tile, &tx, &ty);
    p.ntx = (c->n[0] + tx - 1) / tx;
    p.nty = (c->n[1] + ty - 1) / ty;
    p.fcor = c->phys.f; p.g = c->phys.g; p.gamma = c->phys.cp / c->phys.cv;
    return p;
}

// One fused stage launch, then the forcing of fields 0..3 (used by
// manufactured solutions; the heating of field 4 is fused in the kernel).
hipError_t run_stage(nh_ctx *c, double t, const double *qs, const double *qn, double *out, double a,
                     double b, double cc)
{
    const StageParams p = stage_params(c, t, qs, qn, out, a, b, cc);
    hipError_t e = launch_stage(c->N, c->precision, c->tile, p, c->stream);
    for (int f = 0; f < 4 && e == hipSuccess; ++f) {
        if (c->nsnap[f] == 0) continue;
        const double *f0, *f1;
        double lam;
        forcing_at(c, f, t, &f0, &f1, &lam);
        const WallParams wp{c->n[0], c->n[1], c->n[2], c->per[0], c->per[1]};
        e = launch_add_forcing(wp, f, cc, f0, f1, lam, out + (size_t)f * c->U, c->stream);
    }
    return e;
}

}  // namespace

extern "C" {

const char *nh_version(void) { return "nhsem 0.1 (gfx950)"; }

nh_status nh_workspace_bytes(const nh_mesh_desc *mesh, size_t *bytes)
{
    std::string why;
    if (!bytes) return fail(nullptr, NH_EINVAL, "null output");
    if (!valid_desc(mesh, &why)) return fail(nullptr, NH_EINVAL, "%s", why.c_str());
    *bytes = layout_for(mesh).total;
    return NH_OK;
}

nh_status nh_init_mesh(const nh_mesh_desc *mesh, const nh_physics *phys, void *dev_ws, size_t ws_bytes,
                       void *hip_stream, nh_ctx **out)
{
    std::string why;
    if (!out) return fail(nullptr, NH_EINVAL, "null output");
    *out = nullptr;
    if (!valid_desc(mesh, &why)) return fail(nullptr, NH_EINVAL, "%s", why.c_str());
    if (!phys) return fail(nullptr, NH_EINVAL, "null physics");
    if (!(phys->cv > 0) || !(phys->cp > phys->cv) || !(phys->R > 0) || !(phys->p_a > 0) ||
        !isfinite(phys->g) || !isfinite(phys->f) || !(phys->sponge_tau >= 0))
        return fail(nullptr, NH_EINVAL, "invalid physical constants");
    const Layout L = layout_for(mesh);
    if (!dev_ws) return fail(nullptr, NH_EINVAL, "null workspace");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(nullptr, NH_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(nullptr, NH_ESPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);

    nh_ctx *c = new nh_ctx();
    c->N = mesh->order;
    for (int d = 0; d < 3; ++d) c->nel[d] = mesh->nel[d];
    c->per[0] = mesh->periodic[0];
    c->per[1] = mesh->periodic[1];
    c->n[0] = mesh->nel[0] * c->N + (c->per[0] ? 0 : 1);
    c->n[1] = mesh->nel[1] * c->N + (c->per[1] ? 0 : 1);
    c->n[2] = mesh->nel[2] * c->N + 1;
    c->U = (int64_t)c->n[0] * c->n[1] * c->n[2];
    c->L = (int64_t)mesh->nel[0] * mesh->nel[1] * mesh->nel[2] * (c->N + 1) * (c->N + 1) * (c->N + 1);
    c->precision = mesh->precision;
    c->tile = 0;
    c->xe.assign(mesh->xe, mesh->xe + mesh->nel[0] + 1);
    c->ye.assign(mesh->ye, mesh->ye + mesh->nel[1] + 1);
    c->ze.assign(mesh->ze, mesh->ze + mesh->nel[2] + 1);
    c->phys = *phys;
    c->have_ref = false;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char *)dev_ws;
    c->ws_bytes = ws_bytes;
    c->sticky = false;
    for (int f = 0; f < kNF; ++f) { c->nsnap[f] = 0; c->snap[f] = nullptr; }
    for (int i = 0; i < 3; ++i) c->q[i] = (double *)(c->ws + L.q[i]);
    c->gx = (double *)(c->ws + L.gx); c->gy = (double *)(c->ws + L.gy);
    c->gxf = (float *)(c->ws + L.gxf); c->gyf = (float *)(c->ws + L.gyf);
    c->lev = (double *)(c->ws + L.lev); c->hz2 = (double *)(c->ws + L.hz2);
    c->mx = (double *)(c->ws + L.mx); c->my = (double *)(c->ws + L.my); c->mz = (double *)(c->ws + L.mz);
    c->hx = (double *)(c->ws + L.hx); c->hy = (double *)(c->ws + L.hy); c->hz = (double *)(c->ws + L.hz);
    c->wl = (double *)(c->ws + L.wl);
    c->cst = (double *)(c->ws + L.cst);
    c->diag_part = (double *)(c->ws + L.dpart);
    c->diag_out = (double *)(c->ws + L.dout);

    lgl_basis(c->N, c->xi, c->w, c->D);
    line_tables(c->N, c->nel[0], c->per[0], c->xe.data(), c->xi, c->w, c->D, c->lx, c->m1[0], c->G[0]);
    line_tables(c->N, c->nel[1], c->per[1], c->ye.data(), c->xi, c->w, c->D, c->ly, c->m1[1], c->G[1]);
    line_tables(c->N, c->nel[2], 0, c->ze.data(), c->xi, c->w, c->D, c->lz, c->m1[2], c->G[2]);

    std::vector<float> gxf(c->G[0].begin(), c->G[0].end()), gyf(c->G[1].begin(), c->G[1].end());
    std::vector<double> hz2(c->nel[2]), hx(c->nel[0]), hy(c->nel[1]), hz(c->nel[2]);
    for (int e = 0; e < c->nel[0]; ++e) hx[e] = c->xe[e + 1] - c->xe[e];
    for (int e = 0; e < c->nel[1]; ++e) hy[e] = c->ye[e + 1] - c->ye[e];
    for (int e = 0; e < c->nel[2]; ++e) { hz[e] = c->ze[e + 1] - c->ze[e]; hz2[e] = 2.0 / hz[e]; }
    c->levtab.assign((size_t)c->n[2] * kLevW, 0.0);
    // constant table: D, then C(gamma, n+1) for the EOS series
    std::vector<double> cst(kCst, 0.0);
    {
        const int n1 = c->N + 1;
        for (int i = 0; i < n1 * n1; ++i) cst[kCstD + i] = c->D[i];
        const double gam = phys->cp / phys->cv;
        double cb = gam;  // C(gamma, 1)
        for (int n = 0; n < kEosTerms; ++n) {
            cst[kCstEos + n] = cb;
            cb = cb * (gam - (n + 1)) / (n + 2);
        }
    }

    hipStream_t s = c->stream;
    auto up = [&](void *dst, const void *src, size_t n) { return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s); };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(c->gx, c->G[0].data(), sizeof(double) * c->G[0].size());
    if (e == hipSuccess) e = up(c->gy, c->G[1].data(), sizeof(double) * c->G[1].size());
    if (e == hipSuccess) e = up(c->gxf, gxf.data(), sizeof(float) * gxf.size());
    if (e == hipSuccess) e = up(c->gyf, gyf.data(), sizeof(float) * gyf.size());
    if (e == hipSuccess) e = up(c->hz2, hz2.data(), sizeof(double) * hz2.size());
    if (e == hipSuccess) e = up(c->mx, c->m1[0].data(), sizeof(double) * c->n[0]);
    if (e == hipSuccess) e = up(c->my, c->m1[1].data(), sizeof(double) * c->n[1]);
    if (e == hipSuccess) e = up(c->mz, c->m1[2].data(), sizeof(double) * c->n[2]);
    if (e == hipSuccess) e = up(c->hx, hx.data(), sizeof(double) * hx.size());
    if (e == hipSuccess) e = up(c->hy, hy.data(), sizeof(double) * hy.size());
    if (e == hipSuccess) e = up(c->hz, hz.data(), sizeof(double) * hz.size());
    if (e == hipSuccess) e = up(c->wl, c->w.data(), sizeof(double) * c->w.size());
    if (e == hipSuccess) e = up(c->cst, cst.data(), sizeof(double) * cst.size());
    if (e == hipSuccess) e = up(c->lev, c->levtab.data(), sizeof(double) * c->levtab.size());
    if (e == hipSuccess) e = hipMemsetAsync(c->q[0], 0, sizeof(double) * kNF * c->U, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        g_last_global_error = std::string("nh_init_mesh: ") + hipGetErrorString(e);
        delete c;
        return NH_EHIP;
    }
    *out = c;
    return NH_OK;
}

nh_status nh_set_stream(nh_ctx *c, void *hip_stream)
{
    nh_status st = guard(c);
    if (st) return st;
    c->stream = (hipStream_t)hip_stream;
    return NH_OK;
}

nh_status nh_set_precision(nh_ctx *c, int32_t precision)
{
    nh_status st = guard(c);
    if (st) return st;
    if (precision != NH_FP64 && precision != NH_FP32_MIXED) return fail(c, NH_EINVAL, "bad precision");
    c->precision = precision;
    return NH_OK;
}

nh_status nh_set_tile(nh_ctx *c, int32_t variant)
{
    nh_status st = guard(c);
    if (st) return st;
    if (variant < 0 || variant >= kTileVariants) return fail(c, NH_EINVAL, "tile variant must be 0 or 1");
    c->tile = variant;
    return NH_OK;
}

nh_status nh_tile_shape(int32_t order, int32_t variant, int32_t *tx, int32_t *ty)
{
    if (order < 2 || order > kMaxN || variant < 0 || variant >= kTileVariants || !tx || !ty)
        return fail(nullptr, NH_EINVAL, "bad order or tile variant");
    int a, b;
    stage_tile(order, variant, &a, &b);
    *tx = a;
    *ty = b;
    return NH_OK;
}

nh_status nh_sizes(const nh_ctx *c, int64_t *U, int64_t *L, int32_t n[3])
{
    if (!c) return fail(nullptr, NH_EINVAL, "null context");
    if (U) *U = c->U;
    if (L) *L = c->L;
    if (n) for (int d = 0; d < 3; ++d) n[d] = c->n[d];
    return NH_OK;
}

nh_status nh_lattice_coords(const nh_ctx *c, double *x, double *y, double *z)
{
    if (!c) return fail(nullptr, NH_EINVAL, "null context");
    if (x) memcpy(x, c->lx.data(), sizeof(double) * c->n[0]);
    if (y) memcpy(y, c->ly.data(), sizeof(double) * c->n[1]);
    if (z) memcpy(z, c->lz.data(), sizeof(double) * c->n[2]);
    return NH_OK;
}

nh_status nh_set_reference(nh_ctx *c, const double *rho0, const double *theta0)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!rho0 || !theta0) return fail(c, NH_EINVAL, "null reference arrays");
    const int nz = c->n[2], N = c->N, nc = 2 * N + 1;
    for (int k = 0; k < nz; ++k)
        if (!(rho0[k] > 0) || !(theta0[k] > 0) || !isfinite(rho0[k]) || !isfinite(theta0[k]))
            return fail(c, NH_EINVAL, "reference state must be positive and finite (level %d)", k);
    const nh_physics &ph = c->phys;
    const double gam = ph.cp / ph.cv;
    const double H = c->ze[c->nel[2]];
    for (int k = 0; k < nz; ++k) {
        double *r = &c->levtab[(size_t)k * kLevW];
        r[0] = rho0[k];
        r[1] = theta0[k];
        r[2] = ph.p_a * pow(rho0[k] * ph.R * theta0[k] / ph.p_a, gam);
        // discrete vertical derivative of theta0 (same DSS'd stencil as the state)
        double d = 0.0;
        for (int o = -N; o <= N; ++o) {
            const int kk = k + o;
            if (kk < 0 || kk >= nz) continue;
            d += c->G[2][(size_t)k * nc + N + o] * theta0[kk];
        }
        r[3] = d;
        const double z = c->lz[k];
        double tau = 0.0;
        if (ph.sponge_tau > 0 && z >= ph.sponge_z0 && H > ph.sponge_z0) {
            const double sn = sin(0.5 * M_PI * (z - ph.sponge_z0) / (H - ph.sponge_z0));
            tau = ph.sponge_tau * sn * sn;
        }
        r[4] = tau;
        // weights of the element below (top node) and above (bottom node) at
        // a shared level
        double wlo = 0.0, whi = 1.0;
        if (k % N == 0) {
            const int ez = k / N;
            const double mlo = (ez > 0) ? c->w[N] * (c->ze[ez] - c->ze[ez - 1]) / 2 : 0.0;
            const double mhi = (ez < c->nel[2]) ? c->w[0] * (c->ze[ez + 1] - c->ze[ez]) / 2 : 0.0;
            wlo = mlo / c->m1[2][k];
            whi = mhi / c->m1[2][k];
        }
        r[5] = wlo;
        r[6] = whi;
        r[7] = 1.0 / rho0[k];
        r[8] = 1.0 / theta0[k];
        r[9] = 0.0;
    }
    HIPCHK(c, hipMemcpyAsync(c->lev, c->levtab.data(), sizeof(double) * c->levtab.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_ref = true;
    return NH_OK;
}

nh_status nh_set_forcing(nh_ctx *c, int32_t field, int32_t nsnap, const double *t_snap, const double *dev_snap)
{
    nh_status st = guard(c);
    if (st) return st;
    if (field < 0 || field >= kNF) return fail(c, NH_EINVAL, "field must be in 0..4");
    if (nsnap < 0) return fail(c, NH_EINVAL, "nsnap must be >= 0");
    if (nsnap == 0) {
        c->nsnap[field] = 0;
        c->snap[field] = nullptr;
        c->tsnap[field].clear();
        return NH_OK;
    }
    if (!t_snap || !dev_snap) return fail(c, NH_EINVAL, "null forcing arrays");
    for (int i = 0; i + 1 < nsnap; ++i)
        if (!(t_snap[i + 1] > t_snap[i])) return fail(c, NH_EINVAL, "snapshot times must increase");
    c->nsnap[field] = nsnap;
    c->tsnap[field].assign(t_snap, t_snap + nsnap);
    c->snap[field] = dev_snap;
    return NH_OK;
}

nh_status nh_set_state(nh_ctx *c, const double *dev_q)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_q) return fail(c, NH_EINVAL, "null state");
    HIPCHK(c, hipMemcpyAsync(c->q[0], dev_q, sizeof(double) * kNF * c->U, hipMemcpyDeviceToDevice, c->stream));
    return NH_OK;
}

nh_status nh_get_state(const nh_ctx *cc, double *dev_q)
{
    nh_ctx *c = const_cast<nh_ctx *>(cc);
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_q) return fail(c, NH_EINVAL, "null state");
    HIPCHK(c, hipMemcpyAsync(dev_q, c->q[0], sizeof(double) * kNF * c->U, hipMemcpyDeviceToDevice, c->stream));
    return NH_OK;
}

nh_status nh_state_ptr(nh_ctx *c, double **dev_q)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_q) return fail(c, NH_EINVAL, "null output");
    *dev_q = c->q[0];
    return NH_OK;
}

nh_status nh_rhs(nh_ctx *c, double t, const double *dev_q, double *dev_dqdt)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_q || !dev_dqdt) return fail(c, NH_EINVAL, "null state or output");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    const size_t n = sizeof(double) * kNF * c->U;
    if ((const char *)dev_q < (const char *)dev_dqdt + n && (const char *)dev_dqdt < (const char *)dev_q + n)
        return fail(c, NH_EINVAL, "input and output overlap");
    HIPCHK(c, run_stage(c, t, dev_q, nullptr, dev_dqdt, 0.0, 0.0, 1.0));
    return NH_OK;
}

nh_status nh_rk_step(nh_ctx *c, double t, double dt, int32_t nsteps)
{
    nh_status st = guard(c);
    if (st) return st;
    if (nsteps < 0 || !isfinite(dt) || !isfinite(t)) return fail(c, NH_EINVAL, "bad step arguments");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    double *q0 = c->q[0], *q1 = c->q[1], *q2 = c->q[2];
    for (int s = 0; s < nsteps; ++s) {
        const double ts = t + s * dt;
        HIPCHK(c, run_stage(c, ts, q0, nullptr, q1, 0.0, 1.0, dt));
        HIPCHK(c, run_stage(c, ts + dt, q1, q0, q2, 0.75, 0.25, 0.25 * dt));
        // in place on q0: each node's q^n is read by the thread that overwrites it
        HIPCHK(c, run_stage(c, ts + 0.5 * dt, q2, q0, q0, 1.0 / 3.0, 2.0 / 3.0, 2.0 * dt / 3.0));
    }
    return NH_OK;
}

nh_status nh_dss(nh_ctx *c, int32_t nfields, int32_t mode, const double *dev_E, double *dev_out)
{
    nh_status st = guard(c);
    if (st) return st;
    if (nfields < 1 || nfields > 64) return fail(c, NH_EINVAL, "nfields must be in 1..64");
    if (mode != NH_DSS_SUM && mode != NH_DSS_MASS_AVG) return fail(c, NH_EINVAL, "bad DSS mode");
    if (!dev_E || !dev_out) return fail(c, NH_EINVAL, "null arrays");
    HIPCHK(c, launch_dss(geom(c), nfields, mode, dev_E, dev_out, c->stream));
    return NH_OK;
}

nh_status nh_scatter(nh_ctx *c, int32_t nfields, const double *dev_U, double *dev_E)
{
    nh_status st = guard(c);
    if (st) return st;
    if (nfields < 1 || nfields > 64) return fail(c, NH_EINVAL, "nfields must be in 1..64");
    if (!dev_U || !dev_E) return fail(c, NH_EINVAL, "null arrays");
    HIPCHK(c, launch_scatter(geom(c), nfields, dev_U, dev_E, c->stream));
    return NH_OK;
}

nh_status nh_mass(nh_ctx *c, double *dev_M)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_M) return fail(c, NH_EINVAL, "null output");
    HIPCHK(c, launch_mass(geom(c), dev_M, c->stream));
    return NH_OK;
}

nh_status nh_diagnostics(nh_ctx *c, double out[8])
{
    nh_status st = guard(c);
    if (st) return st;
    if (!out) return fail(c, NH_EINVAL, "null output");
    HIPCHK(c, launch_diag(geom(c), c->q[0], c->diag_part, c->diag_out, c->stream));
    HIPCHK(c, hipMemcpyAsync(out, c->diag_out, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NH_OK;
}

nh_status nh_check_finite(nh_ctx *c)
{
    double d[8];
    nh_status st = nh_diagnostics(c, d);
    if (st) return st;
    if (d[7] != 0.0) return fail(c, NH_ENONFINITE, "state holds %.0f non-finite values", d[7]);
    return NH_OK;
}

nh_status nh_last_error(const nh_ctx *c, char *buf, size_t n)
{
    if (!buf || n == 0) return NH_EINVAL;
    const std::string &s = c ? c->err : g_last_global_error;
    snprintf(buf, n, "%s", s.c_str());
    return NH_OK;
}

nh_status nh_destroy(nh_ctx *c)
{
    if (!c) return NH_EINVAL;
    delete c;
    return NH_OK;
}

}  // extern "C"
