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
#include <algorithm>
#include <mutex>
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
    std::vector<double> CF[3];          // [n][2] per-element factors of the same average
    std::vector<double> levtab;         // [n_z][kLevW]
    nh_physics phys;
    bool have_ref;
    hipStream_t stream;
    // workspace carve
    char *ws;
    size_t ws_bytes;
    double *q[3];
    double *gx, *gy, *gz, *xl, *yl, *zl, *lev, *hz2, *mx, *my, *mz, *hx, *hy, *hz, *wl, *cst, *diag_part, *diag_out;
    double *cfx, *cfy;
    // HEVI workspace (caller-provided, see nh_hevi_attach)
    char *hws;
    size_t hws_bytes;
    int *hiters;
    float *gxf, *gyf;
    // tensor hyper-diffusion (caller-provided workspace, see nh_set_hyperdiffusion)
    bool hd_on;
    double *hd_tmp, *hd_s[3];
    // forcing
    int nsnap[kNF];
    std::vector<double> tsnap[kNF];
    const double *snap[kNF];
    // device of the context and the address of that device's copy of the
    // allocation-free scratch array (see nh_ri_velocity_noalloc)
    int device;
    void *scratch_dev;
    // host-mapped status and look-ahead events of the global GMRES (made by
    // the first 3D-IMEX solve, released by nh_destroy)
    G3Status *g3s_host, *g3s_dev;
    hipEvent_t g3ev[2];
    // error state
    bool sticky;
    std::string err;
};

// Scratch of the allocation-free entry point nh_ri_velocity_noalloc: a fixed
// array in device memory, one copy per GPU, held until the process ends.  On
// the host `scratch` is only a stand-in symbol, never a device address: the
// address of each GPU's copy is resolved once per device, with that device
// current, by resolve_scratch() (called from nh_init_mesh), and only that
// resolved address is handed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_global_error;

// Per-device address of `scratch`, resolved on first use of each device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

// Address of the current device's copy of `scratch` (null on error).
hipError_t resolve_scratch(int *device, void **addr)
{
    *addr = nullptr;
    hipError_t e = hipGetDevice(device);
    if (e != hipSuccess) return e;
    if (*device < 0 || *device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[*device]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[*device] = ptr;
    }
    *addr = g_scratch_addr[*device];
    return hipSuccess;
}

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
    // exact antisymmetry under the reflection of the nodes,
    // D[N-i][N-j] = -D[i][j] (the first half of the rows is kept)
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j)
            if (i > N - i || (i == N - i && j > N - j)) D[i * n1 + j] = -D[(N - i) * n1 + (N - j)];
    if (N % 2 == 0) D[(N / 2) * n1 + N / 2] = 0.0;
}

// Per-direction tables along one lattice line: coordinates, assembled 1D
// mass m(I) = sum_{e ∋ I} w_i h_e / 2, the DSS'd first-derivative stencil
// G[I][N + o] (offset o in -N..N): the m-weighted average of the one-sided
// element derivatives (2/h_e) sum_l D_il f(e, l) of the elements sharing I,
// and the two factors of the same average written per element, CF [n][2]:
// CF[I][0] weights the one-sided derivative of the element in which I is the
// last node (local index N; 0 if there is none), CF[I][1] that of the
// element in which I has local index 0..N-1 (0 if there is none), each
// (w_i h/2) / m(I) * 2/h.
void line_tables(int N, int nel, int periodic, const double *edges, const std::vector<double> &xi,
                 const std::vector<double> &w, const std::vector<double> &D, std::vector<double> &coord,
                 std::vector<double> &m1, std::vector<double> &G, std::vector<double> &CF)
{
    const int n = nel * N + (periodic ? 0 : 1);
    const int nc = 2 * N + 1, n1 = N + 1;
    coord.assign(n, 0.0);
    m1.assign(n, 0.0);
    G.assign((size_t)n * nc, 0.0);
    CF.assign((size_t)n * 2, 0.0);
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
            CF[(size_t)I * 2 + (i == N ? 0 : 1)] += wt * (2.0 / h);
            for (int l = 0; l < n1; ++l) {
                const int off = l - i;  // lattice offset of node l relative to node i
                G[(size_t)I * nc + N + off] += wt * (2.0 / h) * D[i * n1 + l];
            }
        }
    }
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t q[3], gx, gy, gz, xl, yl, zl, gxf, gyf, lev, hz2, mx, my, mz, hx, hy, hz, wl, cst, dpart, dout, cfx, cfy,
        total;
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
    L.gz = take(sizeof(double) * nz * nc);
    L.xl = take(sizeof(double) * nx);
    L.yl = take(sizeof(double) * ny);
    L.zl = take(sizeof(double) * nz);
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
    L.cfx = take(sizeof(double) * nx * 2);
    L.cfy = take(sizeof(double) * ny * 2);
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

// Stage parameters of context c; the tile counts follow tile variant
// `variant` (the context's own unless a batch launches it with another).
StageParams stage_params(const nh_ctx *c, double t, const double *qs, const double *qn, double *out,
                         double a, double b, double cc, int variant = -1)
{
    StageParams p{};
    p.qs = qs; p.qn = qn; p.out = out;
    p.a = a; p.b = b; p.c = cc;
    p.gx = c->gx; p.gy = c->gy; p.gxf = c->gxf; p.gyf = c->gyf;
    p.cfx = c->cfx; p.cfy = c->cfy;
    p.lev = c->lev; p.hz2 = c->hz2; p.cst = c->cst;
    forcing_at(c, 4, t, &p.hq0, &p.hq1, &p.hlam);
    p.nx = c->n[0]; p.ny = c->n[1]; p.nz = c->n[2]; p.nelz = c->nel[2];
    p.perx = c->per[0]; p.pery = c->per[1];
    int tx, ty;
    stage_tile(c->N, variant < 0 ? c->tile : variant, &tx, &ty);
    p.ntx = (c->n[0] + tx - 1) / tx;
    p.nty = (c->n[1] + ty - 1) / ty;
    p.fcor = c->phys.f; p.g = c->phys.g; p.gamma = c->phys.cp / c->phys.cv;
    p.stream = sizeof(double) * kNF * (size_t)c->U >= kStreamBytes;
    return p;
}

// One fused stage launch, then the forcing of fields 0..3 (used by
// manufactured solutions; the heating of field 4 is fused in the kernel).
HyperParams hyper_params(const nh_ctx *c)
{
    HyperParams h{};
    h.nx = c->n[0]; h.ny = c->n[1]; h.nz = c->n[2]; h.N = c->N;
    h.perx = c->per[0]; h.pery = c->per[1];
    h.sx = c->hd_s[0]; h.sy = c->hd_s[1]; h.sz = c->hd_s[2];
    h.stream = sizeof(double) * kNF * (size_t)c->U >= kStreamBytes;
    return h;
}

size_t hyper_bytes(const nh_ctx *c)
{
    const size_t nc = 2 * (size_t)c->N + 1;
    return align_up(sizeof(double) * kNF * (size_t)c->U) +
           align_up(sizeof(double) * nc * ((size_t)c->n[0] + c->n[1] + c->n[2]));
}

// Rows of -m^-1 K along one direction: K = sum_e (tau_e / a_e) D^T W D and
// m = sum_e a_e W assembled over the elements of the line (a_e the half
// length of element e), periodic lines wrapped; row p holds the taps of the
// nodes p - N .. p + N.
void hyper_rows(const nh_ctx *c, int nel, const double *edges, int periodic, const std::vector<double> &tau,
                std::vector<double> &rows)
{
    const int N = c->N, n1 = N + 1, nc = 2 * N + 1;
    const int n = nel * N + (periodic ? 0 : 1);
    rows.assign((size_t)n * nc, 0.0);
    std::vector<double> m(n, 0.0);
    for (int e = 0; e < nel; ++e) {
        const double a = 0.5 * (edges[e + 1] - edges[e]);
        for (int i = 0; i < n1; ++i) {
            const int P = (e * N + i) % n;
            m[P] += a * c->w[i];
            for (int j = 0; j < n1; ++j) {
                double k = 0.0;
                for (int q = 0; q < n1; ++q) k += c->D[q * n1 + i] * c->w[q] * c->D[q * n1 + j];
                rows[(size_t)P * nc + (j - i + N)] += tau[e] / a * k;
            }
        }
    }
    for (int P = 0; P < n; ++P)
        for (int o = 0; o < nc; ++o) rows[(size_t)P * nc + o] = -rows[(size_t)P * nc + o] / m[P];
}

hipError_t run_stage(nh_ctx *c, double t, const double *qs, const double *qn, double *out, double a,
                     double b, double cc)
{
    const StageParams p = stage_params(c, t, qs, qn, out, a, b, cc);
    hipError_t e = launch_stage(c->N, c->precision, c->tile, p, c->stream);
    if (e == hipSuccess && c->hd_on) {
        // out += cc H(qs), H = -(div tau grad)^2 qs
        const HyperParams hp = hyper_params(c);
        e = launch_hd_laplace(hp, qs, c->hd_tmp, 1.0, false, false, c->stream);
        if (e == hipSuccess) e = launch_hd_laplace(hp, c->hd_tmp, out, -cc, true, true, c->stream);
    }
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

    int device = -1;
    void *scratch_dev = nullptr;
    {
        const hipError_t e = resolve_scratch(&device, &scratch_dev);
        if (e != hipSuccess) return fail(nullptr, NH_EHIP, "scratch address: %s", hipGetErrorString(e));
    }
    nh_ctx *c = new nh_ctx();
    c->device = device;
    c->scratch_dev = scratch_dev;
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
    c->gx = (double *)(c->ws + L.gx); c->gy = (double *)(c->ws + L.gy); c->gz = (double *)(c->ws + L.gz);
    c->xl = (double *)(c->ws + L.xl);
    c->yl = (double *)(c->ws + L.yl);
    c->zl = (double *)(c->ws + L.zl);
    c->hws = nullptr; c->hws_bytes = 0; c->hiters = nullptr;
    c->gxf = (float *)(c->ws + L.gxf); c->gyf = (float *)(c->ws + L.gyf);
    c->lev = (double *)(c->ws + L.lev); c->hz2 = (double *)(c->ws + L.hz2);
    c->mx = (double *)(c->ws + L.mx); c->my = (double *)(c->ws + L.my); c->mz = (double *)(c->ws + L.mz);
    c->hx = (double *)(c->ws + L.hx); c->hy = (double *)(c->ws + L.hy); c->hz = (double *)(c->ws + L.hz);
    c->wl = (double *)(c->ws + L.wl);
    c->cst = (double *)(c->ws + L.cst);
    c->diag_part = (double *)(c->ws + L.dpart);
    c->diag_out = (double *)(c->ws + L.dout);
    c->cfx = (double *)(c->ws + L.cfx);
    c->cfy = (double *)(c->ws + L.cfy);

    lgl_basis(c->N, c->xi, c->w, c->D);
    line_tables(c->N, c->nel[0], c->per[0], c->xe.data(), c->xi, c->w, c->D, c->lx, c->m1[0], c->G[0], c->CF[0]);
    line_tables(c->N, c->nel[1], c->per[1], c->ye.data(), c->xi, c->w, c->D, c->ly, c->m1[1], c->G[1], c->CF[1]);
    line_tables(c->N, c->nel[2], 0, c->ze.data(), c->xi, c->w, c->D, c->lz, c->m1[2], c->G[2], c->CF[2]);

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
    if (e == hipSuccess) e = up(c->cfx, c->CF[0].data(), sizeof(double) * c->CF[0].size());
    if (e == hipSuccess) e = up(c->cfy, c->CF[1].data(), sizeof(double) * c->CF[1].size());
    if (e == hipSuccess) e = up(c->gz, c->G[2].data(), sizeof(double) * c->G[2].size());
    if (e == hipSuccess) e = up(c->xl, c->lx.data(), sizeof(double) * c->lx.size());
    if (e == hipSuccess) e = up(c->yl, c->ly.data(), sizeof(double) * c->ly.size());
    if (e == hipSuccess) e = up(c->zl, c->lz.data(), sizeof(double) * c->lz.size());
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
    if (variant < 0 || variant >= kTileVariants) return fail(c, NH_EINVAL, "tile variant must be 0, 1 or 2");
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


}  // extern "C"

// ------------------------------------------------------------------ HEVI
nh_status mlp_guess(nh_mlp *m, nh_ctx *c, double alpha, const double *b, double *lb, double *x0);

namespace {

// ARK2 of Giraldo, Kelly & Constantinescu (2013) ("ARK(2,3,2)b", Sec. 2.3):
// explicit A, implicit At (singly diagonally implicit), b = bt, c.
struct Ark2 {
    double A[3][3], At[3][3], b[3], c[3];
    Ark2()
    {
        const double g = 1.0 - 1.0 / sqrt(2.0), d = 1.0 / (2.0 * sqrt(2.0)), a = (3.0 + 2.0 * sqrt(2.0)) / 6.0;
        const double A0[3][3] = {{0, 0, 0}, {2 * g, 0, 0}, {1 - a, a, 0}};
        const double T0[3][3] = {{0, 0, 0}, {g, g, 0}, {d, d, g}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) { A[i][j] = A0[i][j]; At[i][j] = T0[i][j]; }
        b[0] = d; b[1] = d; b[2] = g;
        c[0] = 0.0; c[1] = 2 * g; c[2] = 1.0;
    }
};

constexpr int kHeviArrays = 11;  // S1 S2 S3 L1 L2 Q2 Q3 R2 R3, L_v R and the MLP guess

size_t hevi_bytes(const nh_ctx *c)
{
    const size_t fb = align_up(sizeof(double) * kNF * (size_t)c->U);
    const size_t ib = align_up(sizeof(int) * 2 * (size_t)c->n[0] * c->n[1]);
    return kHeviArrays * fb + ib;
}

double *hevi_arr(const nh_ctx *c, int i)
{
    const size_t fb = align_up(sizeof(double) * kNF * (size_t)c->U);
    return (double *)(c->hws + fb * i);
}

HeviParams hevi_params(const nh_ctx *c)
{
    HeviParams h{};
    h.nx = c->n[0]; h.ny = c->n[1]; h.nz = c->n[2]; h.N = c->N;
    h.lev = c->lev; h.gz = c->gz;
    h.gamma = c->phys.cp / c->phys.cv; h.g = c->phys.g;
    return h;
}

nh_status check_gmres_opts(nh_ctx *c, const nh_gmres_opts *o)
{
    if (!o) return fail(c, NH_EINVAL, "null GMRES options");
    if (o->restart < 1 || o->restart > 40) return fail(c, NH_EINVAL, "restart must be in 1..40");
    if (o->max_restarts < 0 || o->max_restarts > 1000) return fail(c, NH_EINVAL, "max_restarts out of range");
    if (!(o->rtol > 0.0) || !(o->rtol < 1.0)) return fail(c, NH_EINVAL, "rtol must be in (0, 1)");
    if (o->schur != 0 && o->schur != 1) return fail(c, NH_EINVAL, "schur must be 0 or 1");
    if (o->schur) {
        if (o->restart != kGmresRegM) return fail(c, NH_EUNSUPPORTED, "the Schur form runs with restart %d", kGmresRegM);
        if (c->n[2] - 2 > 64 * kGmresSchurSlots)
            return fail(c, NH_EUNSUPPORTED, "the Schur form supports up to %d interior levels", 64 * kGmresSchurSlots);
        return NH_OK;
    }
    if (gmres_lds_bytes(c->n[2], c->N, o->restart) > 160 * 1024)
        return fail(c, NH_EUNSUPPORTED, "column too tall for an LDS-resident Krylov basis of this restart length");
    return NH_OK;
}

hipError_t run_gmres(nh_ctx *c, double alpha, const double *b, const double *x0, double *x,
                     const nh_gmres_opts *o, int *iters)
{
    GmresArgs g{};
    g.b = b; g.x0 = x0; g.x = x; g.alpha = alpha; g.rtol = o->rtol;
    g.restart = o->restart; g.max_restarts = o->max_restarts; g.iters = iters; g.schur = o->schur;
    g.pick = o->guess_pick;
    return launch_gmres(hevi_params(c), g, c->stream);
}

nh_status gather_stats(nh_ctx *c, const int *dev_iters, int nsolves, nh_solve_stats *st)
{
    if (!st) return NH_OK;
    const size_t ncol = (size_t)c->n[0] * c->n[1];
    std::vector<int> h(ncol * nsolves);
    HIPCHK(c, hipMemcpyAsync(h.data(), dev_iters, sizeof(int) * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    st->columns = (int64_t)ncol;
    st->solves = nsolves;
    st->iters_total = 0; st->iters_max = 0; st->not_converged = 0;
    for (int v : h) {
        const int it = v >= 0 ? v : -v - 1;
        st->iters_total += it;
        if (it > st->iters_max) st->iters_max = it;
        if (v < 0) ++st->not_converged;
    }
    return st->not_converged ? fail(c, NH_ENOCONV, "%lld column solves did not converge",
                                    (long long)st->not_converged)
                             : NH_OK;
}

}  // namespace

extern "C" {

nh_status nh_hyperdiffusion_workspace_bytes(const nh_ctx *c, size_t *bytes)
{
    if (!c) return fail(nullptr, NH_EINVAL, "null context");
    if (!bytes) return fail(nullptr, NH_EINVAL, "null output");
    *bytes = hyper_bytes(c);
    return NH_OK;
}

nh_status nh_set_hyperdiffusion(nh_ctx *c, const double *coef, double dt, void *dev_ws, size_t bytes)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!coef) {
        c->hd_on = false;
        return NH_OK;
    }
    for (int i = 0; i < 3; ++i)
        if (!(coef[i] >= 0.0) || !isfinite(coef[i])) return fail(c, NH_EINVAL, "coefficients must be finite and >= 0");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, NH_EINVAL, "dt must be finite and > 0");
    if (!dev_ws) return fail(c, NH_EINVAL, "null hyper-diffusion workspace");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(c, NH_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < hyper_bytes(c)) return fail(c, NH_ESPACE, "hyper-diffusion workspace %zu < %zu bytes", bytes,
                                            hyper_bytes(c));
    // principal-axis rank of each direction in every element: the metric
    // tensor of a box is diag(4 / h^2); ascending eigenvalues = descending
    // extents, values equal to 1e-10 (relative) taken in x, y, z order
    const std::vector<double> *edges[3] = {&c->xe, &c->ye, &c->ze};
    int rank[3] = {-1, -1, -1};
    for (int ez = 0; ez < c->nel[2]; ++ez)
        for (int ey = 0; ey < c->nel[1]; ++ey)
            for (int ex = 0; ex < c->nel[0]; ++ex) {
                const int el[3] = {ex, ey, ez};
                double g[3], gmax = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const double h = (*edges[d])[el[d] + 1] - (*edges[d])[el[d]];
                    g[d] = 4.0 / (h * h);
                    gmax = std::max(gmax, g[d]);
                }
                const double tol = 1e-10 * gmax;
                for (int d = 0; d < 3; ++d) {
                    int r = 0;
                    for (int o = 0; o < 3; ++o) {
                        if (o == d) continue;
                        const bool before = g[o] < g[d] - tol || (std::fabs(g[o] - g[d]) <= tol && o < d);
                        r += before ? 1 : 0;
                    }
                    if (rank[d] < 0) rank[d] = r;
                    else if (rank[d] != r)
                        return fail(c, NH_EUNSUPPORTED,
                                    "the order of element extents changes across the mesh (tau not separable)");
                }
            }
    // tau of direction d in element e: nu_rank = c_rank^(1/2) h^2 / dt^(1/2)
    char *w = (char *)dev_ws;
    c->hd_tmp = (double *)w;
    double *tab = (double *)(w + align_up(sizeof(double) * kNF * (size_t)c->U));
    std::vector<double> all;
    for (int d = 0; d < 3; ++d) {
        const int nel = c->nel[d];
        std::vector<double> tau(nel), rows;
        for (int e = 0; e < nel; ++e) {
            const double h = (*edges[d])[e + 1] - (*edges[d])[e];
            tau[e] = std::sqrt(coef[rank[d]]) * h * h / std::sqrt(dt);
        }
        hyper_rows(c, nel, edges[d]->data(), d < 2 ? c->per[d] : 0, tau, rows);
        c->hd_s[d] = tab + all.size();
        all.insert(all.end(), rows.begin(), rows.end());
    }
    HIPCHK(c, hipMemcpyAsync(tab, all.data(), sizeof(double) * all.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->hd_on = true;
    return NH_OK;
}

nh_status nh_hyperdiffusion(nh_ctx *c, const double *dev_q, double *dev_H)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!c->hd_on) return fail(c, NH_EINVAL, "hyper-diffusion not set");
    if (!dev_q || !dev_H) return fail(c, NH_EINVAL, "null arrays");
    if (dev_q == dev_H) return fail(c, NH_EINVAL, "dev_q and dev_H must differ");
    const HyperParams hp = hyper_params(c);
    HIPCHK(c, launch_hd_laplace(hp, dev_q, c->hd_tmp, 1.0, false, false, c->stream));
    HIPCHK(c, launch_hd_laplace(hp, c->hd_tmp, dev_H, -1.0, false, true, c->stream));
    return NH_OK;
}

// ---- RI-velocity diagnostic: workspace carve (per-workgroup partials); nb
// workgroups per level of ~4096 columns each
static int ri_chunks(const nh_ctx *c)
{
    const int64_t nxy = (int64_t)c->n[0] * c->n[1];
    return (int)std::min<int64_t>(256, std::max<int64_t>(1, (nxy + 4095) / 4096));
}

static size_t ri_bytes(const nh_ctx *c, int ns, RiWork *w, char *base)
{
    const size_t nb = ri_chunks(c), nz = c->n[2];
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return base ? base + o : nullptr; };
    double *cpart = (double *)take(sizeof(double) * nz * nb * 3);
    double *ssum = (double *)take(sizeof(double) * nz * nb * ns);
    int *scnt = (int *)take(sizeof(int) * nz * nb * ns);
    double *umax = (double *)take(sizeof(double) * nz * nb);
    if (w) *w = RiWork{cpart, ssum, scnt, umax};
    return off;
}

nh_status nh_ri_workspace_bytes(const nh_ctx *c, int32_t nstrips, size_t *bytes)
{
    if (!c || !bytes) return fail(nullptr, NH_EINVAL, "null argument");
    if (nstrips < 1 || nstrips > kRiMaxStrips) return fail(nullptr, NH_EINVAL, "nstrips must be in [1, %d]", kRiMaxStrips);
    *bytes = ri_bytes(c, nstrips, nullptr, nullptr);
    return NH_OK;
}

static nh_status ri_check(nh_ctx *c, const double *dev_q, int32_t nstrips, double rmax, double *dev_center,
                          double *dev_ubar, int32_t *dev_count, double *dev_result)
{
    nh_status st = guard(c);
    if (st) return st;
    if (nstrips < 1 || nstrips > kRiMaxStrips) return fail(c, NH_EINVAL, "nstrips must be in [1, %d]", kRiMaxStrips);
    if (!(rmax > 0.0) || !isfinite(rmax)) return fail(c, NH_EINVAL, "rmax must be finite and > 0");
    if (!dev_q || !dev_center || !dev_ubar || !dev_count || !dev_result) return fail(c, NH_EINVAL, "null arrays");
    return NH_OK;
}

static nh_status ri_run(nh_ctx *c, const double *dev_q, int32_t nstrips, double rmax, int32_t center_given,
                        double *dev_center, double *dev_ubar, int32_t *dev_count, double *dev_result, void *dev_ws);

nh_status nh_ri_velocity(nh_ctx *c, const double *dev_q, int32_t nstrips, double rmax, int32_t center_given,
                         double *dev_center, double *dev_ubar, int32_t *dev_count, double *dev_result, void *dev_ws,
                         size_t bytes)
{
    nh_status st = ri_check(c, dev_q, nstrips, rmax, dev_center, dev_ubar, dev_count, dev_result);
    if (st) return st;
    if (!dev_ws) return fail(c, NH_EINVAL, "null arrays");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(c, NH_EINVAL, "RI workspace must be 256-byte aligned");
    const size_t need = ri_bytes(c, nstrips, nullptr, nullptr);
    if (bytes < need) return fail(c, NH_ESPACE, "RI workspace %zu < %zu bytes", bytes, need);
    return ri_run(c, dev_q, nstrips, rmax, center_given, dev_center, dev_ubar, dev_count, dev_result, dev_ws);
}

nh_status nh_ri_velocity_noalloc(nh_ctx *c, const double *dev_q, int32_t nstrips, double rmax, int32_t center_given,
                                 double *dev_center, double *dev_ubar, int32_t *dev_count, double *dev_result)
{
    nh_status st = ri_check(c, dev_q, nstrips, rmax, dev_center, dev_ubar, dev_count, dev_result);
    if (st) return st;
    const size_t need = ri_bytes(c, nstrips, nullptr, nullptr);
    if (need > kNoAllocScratchBytes)
        return fail(c, NH_ESPACE,
                    "the diagnostic needs %zu bytes of partial sums here; the allocation-free form holds at most %zu "
                    "(fewer strips, or nh_ri_velocity with a workspace)", need, kNoAllocScratchBytes);
    if (!c->scratch_dev) return fail(c, NH_ESTATE, "scratch address of the context's device not resolved");
    // every partial the kernels read is written first in the same call: the
    // scratch needs no clearing
    return ri_run(c, dev_q, nstrips, rmax, center_given, dev_center, dev_ubar, dev_count, dev_result,
                  c->scratch_dev);
}

static nh_status ri_run(nh_ctx *c, const double *dev_q, int32_t nstrips, double rmax, int32_t center_given,
                        double *dev_center, double *dev_ubar, int32_t *dev_count, double *dev_result, void *dev_ws)
{
    RiWork w;
    ri_bytes(c, nstrips, &w, (char *)dev_ws);
    RiParams p{};
    p.nx = c->n[0]; p.ny = c->n[1]; p.nz = c->n[2];
    p.nstrips = nstrips;
    p.nb = ri_chunks(c);
    p.U = c->U;
    p.x = c->xl; p.y = c->yl; p.mx = c->mx; p.my = c->my;
    p.eps = rmax / nstrips;
    p.xmid = 0.5 * (c->xe.front() + c->xe.back());
    p.ymid = 0.5 * (c->ye.front() + c->ye.back());
    HIPCHK(c, launch_ri(p, dev_q, center_given != 0, dev_center, dev_ubar, dev_count, dev_result, c->zl, w,
                        c->stream));
    return NH_OK;
}

nh_status nh_hevi_workspace_bytes(const nh_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(nullptr, NH_EINVAL, "null argument");
    *bytes = hevi_bytes(c);
    return NH_OK;
}

nh_status nh_hevi_attach(nh_ctx *c, void *dev_ws, size_t bytes)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_ws) return fail(c, NH_EINVAL, "null HEVI workspace");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(c, NH_EINVAL, "HEVI workspace must be 256-byte aligned");
    if (bytes < hevi_bytes(c)) return fail(c, NH_ESPACE, "HEVI workspace %zu < %zu bytes", bytes, hevi_bytes(c));
    c->hws = (char *)dev_ws;
    c->hws_bytes = bytes;
    c->hiters = (int *)(c->hws + kHeviArrays * align_up(sizeof(double) * kNF * (size_t)c->U));
    return NH_OK;
}

nh_status nh_hevi_last_solves(nh_ctx *c, const double **R2, const double **X2, const double **R3,
                              const double **X3, double *alpha, double *scratch_ptr_unused)
{
    (void)scratch_ptr_unused;
    nh_status st = guard(c);
    if (st) return st;
    if (!c->hws) return fail(c, NH_EINVAL, "no HEVI workspace attached");
    static const Ark2 ark;
    if (R2) *R2 = hevi_arr(c, 7);
    if (X2) *X2 = hevi_arr(c, 5);
    if (R3) *R3 = hevi_arr(c, 8);
    if (X3) *X3 = hevi_arr(c, 6);
    if (alpha) *alpha = ark.At[1][1];
    return NH_OK;
}

nh_status nh_lv_apply(nh_ctx *c, const double *dev_x, double *dev_y)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_x || !dev_y) return fail(c, NH_EINVAL, "null arrays");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    HIPCHK(c, launch_lv_apply(hevi_params(c), dev_x, dev_y, c->stream));
    return NH_OK;
}

nh_status nh_column_solve(nh_ctx *c, double alpha, const double *dev_b, const double *dev_x0, double *dev_x,
                          const nh_gmres_opts *opts, nh_solve_stats *stats, int32_t *dev_iters)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!dev_b || !dev_x) return fail(c, NH_EINVAL, "null arrays");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    if (!(alpha >= 0.0) || !isfinite(alpha)) return fail(c, NH_EINVAL, "alpha must be finite and >= 0");
    if ((st = check_gmres_opts(c, opts))) return st;
    int *it = dev_iters ? dev_iters : c->hiters;
    if (!it && stats) return fail(c, NH_EINVAL, "stats need dev_iters or an attached HEVI workspace");
    HIPCHK(c, run_gmres(c, alpha, dev_b, dev_x0, dev_x, opts, it));
    return gather_stats(c, it, 1, stats);
}

nh_status nh_hevi_step(nh_ctx *c, double t, double dt, const nh_gmres_opts *opts, nh_mlp *guess,
                       nh_solve_stats *stats)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!c->hws) return fail(c, NH_EINVAL, "no HEVI workspace attached");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    if (!isfinite(t) || !(dt > 0.0) || !isfinite(dt)) return fail(c, NH_EINVAL, "bad time step");
    if ((st = check_gmres_opts(c, opts))) return st;
    static const Ark2 ark;
    const long n = kNF * (long)c->U;
    double *Q1 = c->q[0];
    double *S[3] = {hevi_arr(c, 0), hevi_arr(c, 1), hevi_arr(c, 2)};
    double *Lv[2] = {hevi_arr(c, 3), hevi_arr(c, 4)};
    double *Q[3] = {Q1, hevi_arr(c, 5), hevi_arr(c, 6)};
    double *Rs[3] = {nullptr, hevi_arr(c, 7), hevi_arr(c, 8)};
    const size_t ncol = (size_t)c->n[0] * c->n[1];
    for (int i = 0; i < 3; ++i) {
        if (i > 0) {
            // R = q^n + dt sum_{j<i} [A_ij S_j + (At_ij - A_ij) L_j]
            LinComb lc{};
            int ns = 0;
            for (int j = 0; j < i; ++j) {
                lc.src[ns] = S[j]; lc.c[ns++] = dt * ark.A[i][j];
                lc.src[ns] = Lv[j]; lc.c[ns++] = dt * (ark.At[i][j] - ark.A[i][j]);
            }
            double *R = Rs[i];
            HIPCHK(c, launch_axpy_multi(n, Q1, ns, lc, R, c->stream));
            const double *x0 = nullptr;
            if (guess) {
                st = mlp_guess(guess, c, dt * ark.At[i][i], R, hevi_arr(c, 9), hevi_arr(c, 10));
                if (st) return st;
                x0 = hevi_arr(c, 10);
            }
            HIPCHK(c, run_gmres(c, dt * ark.At[i][i], R, x0, Q[i], opts, c->hiters + (i - 1) * ncol));
        }
        HIPCHK(c, run_stage(c, t + ark.c[i] * dt, Q[i], nullptr, S[i], 0.0, 0.0, 1.0));
        if (i < 2) HIPCHK(c, launch_lv_apply(hevi_params(c), Q[i], Lv[i], c->stream));
    }
    LinComb lc{};
    for (int j = 0; j < 3; ++j) { lc.src[j] = S[j]; lc.c[j] = dt * ark.b[j]; }
    HIPCHK(c, launch_axpy_multi(n, Q1, 3, lc, Q1, c->stream));
    return gather_stats(c, c->hiters, 2, stats);
}

// ---- 3D-IMEX (linear operator over all directions, global GMRES)
static L3Params l3_params(const nh_ctx *c)
{
    L3Params h{};
    h.nx = c->n[0]; h.ny = c->n[1]; h.nz = c->n[2]; h.N = c->N;
    h.perx = c->per[0]; h.pery = c->per[1];
    h.gx = c->gx; h.gy = c->gy; h.lev = c->lev;
    h.gamma = c->phys.cp / c->phys.cv;
    h.hv = hevi_params(c);
    return h;
}

// workspace: restart + 1 Krylov vectors, restart preconditioned vectors, one
// scratch vector, partial sums, then (step only) the ARK2 arrays S_0..2,
// L_0..1, Q_1..2, R
static size_t g3_bytes(const nh_ctx *c, int restart, bool step, G3Work *w, double **ark, char *base)
{
    const size_t nv = align_up(sizeof(double) * kNF * (size_t)c->U);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return base ? base + o : nullptr; };
    G3Work g{};
    g.V = (double *)take(nv * (restart + 1));
    g.Z = (double *)take(nv * restart);
    g.t = (double *)take(nv);
    g.part = (double *)take(sizeof(double) * 1024 * 35);
    g.state = (G3State *)take(sizeof(G3State));
    if (step)
        for (int i = 0; i < 8; ++i) {
            double *a = (double *)take(nv);
            if (ark) ark[i] = a;
        }
    if (w) *w = g;
    return off;
}

// The context's host-mapped status block and events, made on first use
static nh_status g3_host(nh_ctx *c, G3Work *w)
{
    if (!c->g3s_host) {
        void *p = nullptr;
        HIPCHK(c, hipHostMalloc(&p, sizeof(G3Status), hipHostMallocMapped | hipHostMallocCoherent));
        void *d = nullptr;
        hipError_t e = hipHostGetDevicePointer(&d, p, 0);
        hipEvent_t ev[2] = {nullptr, nullptr};
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            (void)hipHostFree(p);
            HIPCHK(c, e);
        }
        c->g3s_host = (G3Status *)p;
        c->g3s_dev = (G3Status *)d;
        c->g3ev[0] = ev[0];
        c->g3ev[1] = ev[1];
    }
    w->status = c->g3s_host;
    w->status_dev = c->g3s_dev;
    w->ev[0] = c->g3ev[0];
    w->ev[1] = c->g3ev[1];
    return NH_OK;
}

static nh_status check_g3_opts(nh_ctx *c, const nh_gmres_opts *o)
{
    if (!o) return fail(c, NH_EINVAL, "null GMRES options");
    if (o->restart < 1 || o->restart > kG3MaxRestart)
        return fail(c, NH_EINVAL, "restart must be in [1, %d]", kG3MaxRestart);
    if (o->max_restarts < 0) return fail(c, NH_EINVAL, "max_restarts must be >= 0");
    if (!(o->rtol > 0.0) || !(o->rtol < 1.0)) return fail(c, NH_EINVAL, "rtol must be in (0, 1)");
    if (o->schur) return fail(c, NH_EUNSUPPORTED, "no Schur form of the global solve");
    if (o->precondition != 0 && o->precondition != 1) return fail(c, NH_EINVAL, "precondition must be 0 or 1");
    if (o->precondition && 3 * c->n[2] > 256 && c->n[2] - 2 > 64 * kGmresSchurSlots)
        return fail(c, NH_EUNSUPPORTED, "column preconditioner needs n_z <= 130");
    return NH_OK;
}

static nh_status check_g3_ws(nh_ctx *c, const nh_gmres_opts *o, bool step, void *ws, size_t bytes)
{
    if (!ws) return fail(c, NH_EINVAL, "null 3D-IMEX workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(c, NH_EINVAL, "3D-IMEX workspace must be 256-byte aligned");
    const size_t need = g3_bytes(c, o->restart, step, nullptr, nullptr, nullptr);
    if (bytes < need) return fail(c, NH_ESPACE, "3D-IMEX workspace %zu < %zu bytes", bytes, need);
    return NH_OK;
}

static void g3_count(nh_solve_stats *st, int it, double relres, double rtol)
{
    if (!st) return;
    st->columns = 1;
    st->solves += 1;
    st->iters_total += it;
    st->iters_max = std::max<int64_t>(st->iters_max, it);
    if (!(relres <= rtol)) st->not_converged += 1;
}

nh_status nh_l3_apply(nh_ctx *c, const double *dev_x, double *dev_y)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    if (!dev_x || !dev_y) return fail(c, NH_EINVAL, "null arrays");
    if (dev_x == dev_y) return fail(c, NH_EINVAL, "dev_x and dev_y must differ");
    HIPCHK(c, launch_l3(l3_params(c), dev_x, dev_y, 0.0, 1.0, c->stream));
    return NH_OK;
}

nh_status nh_imex3d_workspace_bytes(const nh_ctx *c, int32_t restart, size_t *bytes)
{
    if (!c || !bytes) return fail(nullptr, NH_EINVAL, "null argument");
    if (restart < 1 || restart > kG3MaxRestart) return fail(nullptr, NH_EINVAL, "restart must be in [1, %d]", kG3MaxRestart);
    *bytes = g3_bytes(c, restart, true, nullptr, nullptr, nullptr);
    return NH_OK;
}

nh_status nh_global_solve(nh_ctx *c, double alpha, const double *dev_b, const double *dev_x0, double *dev_x,
                          const nh_gmres_opts *opts, void *dev_ws, size_t bytes, nh_solve_stats *stats)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    if (!dev_b || !dev_x) return fail(c, NH_EINVAL, "null arrays");
    if (dev_b == dev_x) return fail(c, NH_EINVAL, "dev_b and dev_x must differ");
    if (!isfinite(alpha) || alpha < 0.0) return fail(c, NH_EINVAL, "alpha must be finite and >= 0");
    if ((st = check_g3_opts(c, opts))) return st;
    if ((st = check_g3_ws(c, opts, false, dev_ws, bytes))) return st;
    G3Work w;
    g3_bytes(c, opts->restart, false, &w, nullptr, (char *)dev_ws);
    if ((st = g3_host(c, &w))) return st;
    if (stats) *stats = nh_solve_stats{};
    int it = 0;
    double rr = 0.0;
    HIPCHK(c, gmres3d(l3_params(c), w, alpha, dev_b, dev_x0, dev_x, opts->restart, opts->max_restarts, opts->rtol,
                      opts->precondition != 0, c->stream, &it, &rr));
    g3_count(stats, it, rr, opts->rtol);
    if (!(rr <= opts->rtol)) return fail(c, NH_ENOCONV, "global GMRES: relative residual %.3e > %.3e", rr, opts->rtol);
    return NH_OK;
}

nh_status nh_imex3d_step(nh_ctx *c, double t, double dt, const nh_gmres_opts *opts, void *dev_ws, size_t bytes,
                         nh_solve_stats *stats)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    if (!isfinite(t) || !(dt > 0.0) || !isfinite(dt)) return fail(c, NH_EINVAL, "bad time step");
    if ((st = check_g3_opts(c, opts))) return st;
    if ((st = check_g3_ws(c, opts, true, dev_ws, bytes))) return st;
    G3Work w;
    double *a[8];
    g3_bytes(c, opts->restart, true, &w, a, (char *)dev_ws);
    if ((st = g3_host(c, &w))) return st;
    if (stats) *stats = nh_solve_stats{};
    static const Ark2 ark;
    const long n = kNF * (long)c->U;
    const L3Params h = l3_params(c);
    double *Q1 = c->q[0];
    double *S[3] = {a[0], a[1], a[2]};
    double *Lx[2] = {a[3], a[4]};
    double *Q[3] = {Q1, a[5], a[6]};
    double *R = a[7];
    bool missed = false;
    for (int i = 0; i < 3; ++i) {
        if (i > 0) {
            // R = q^n + dt sum_{j<i} [A_ij S_j + (At_ij - A_ij) L_j]
            LinComb lc{};
            int ns = 0;
            for (int j = 0; j < i; ++j) {
                lc.src[ns] = S[j]; lc.c[ns++] = dt * ark.A[i][j];
                lc.src[ns] = Lx[j]; lc.c[ns++] = dt * (ark.At[i][j] - ark.A[i][j]);
            }
            HIPCHK(c, launch_axpy_multi(n, Q1, ns, lc, R, c->stream));
            int it = 0;
            double rr = 0.0;
            HIPCHK(c, gmres3d(h, w, dt * ark.At[i][i], R, R, Q[i], opts->restart, opts->max_restarts, opts->rtol,
                              opts->precondition != 0, c->stream, &it, &rr));
            g3_count(stats, it, rr, opts->rtol);
            missed = missed || !(rr <= opts->rtol);
        }
        HIPCHK(c, run_stage(c, t + ark.c[i] * dt, Q[i], nullptr, S[i], 0.0, 0.0, 1.0));
        if (i < 2) HIPCHK(c, launch_l3(h, Q[i], Lx[i], 0.0, 1.0, c->stream));
    }
    LinComb lc{};
    for (int j = 0; j < 3; ++j) { lc.src[j] = S[j]; lc.c[j] = dt * ark.b[j]; }
    HIPCHK(c, launch_axpy_multi(n, Q1, 3, lc, Q1, c->stream));
    if (missed) return fail(c, NH_ENOCONV, "3D-IMEX step: a stage solve missed rtol");
    return NH_OK;
}

}  // extern "C"

extern "C" {
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
    if (c->g3s_host) {
        (void)hipHostFree(c->g3s_host);
        for (hipEvent_t e : c->g3ev) (void)hipEventDestroy(e);
    }
    delete c;
    return NH_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ column MLP
struct nh_mlp {
    MlpNet net;
    long max_batch;
    int step;
    int passes;   // network applications per initial guess (nh_mlp_set_passes)
    float decay;  // decoupled weight decay of the hidden path (nh_mlp_set_decay)
    hipStream_t stream;
    bool sticky;
    std::string err;
};

namespace {

struct MlpLayout {
    size_t params[5], acts[11], feat, scale, total;
};

long mlp_nparam()
{
    return (long)kMlpHid * kMlpIn + kMlpHid + (long)kMlpHid * kMlpHid + kMlpHid + (long)kMlpOut * kMlpHid + kMlpOut +
           (long)kMlpOut * kMlpIn;
}

MlpLayout mlp_layout(long B)
{
    MlpLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const long np = mlp_nparam();
    for (int i = 0; i < 4; ++i) L.params[i] = take(sizeof(float) * np);   // master grad m v
    L.params[4] = take(sizeof(uint16_t) * np);                             // half
    L.acts[0] = take(sizeof(float) * B * kMlpHid);     // Z1
    L.acts[1] = take(sizeof(float) * B * kMlpHid);     // Z2
    L.acts[2] = take(sizeof(float) * B * kMlpOut);     // Y
    L.acts[3] = take(sizeof(float) * B * kMlpOut);     // dY
    L.acts[4] = take(sizeof(float) * B * kMlpHid);     // dH
    L.acts[5] = take(sizeof(float) * B * kMlpHid);     // dZ
    L.acts[6] = take(sizeof(float) * kMlpLossBlocks);  // part
    L.acts[7] = take(sizeof(float) * 4);               // loss
    L.acts[8] = take(sizeof(uint16_t) * B * kMlpHid);  // H1
    L.acts[9] = take(sizeof(uint16_t) * B * kMlpHid);  // H2
    // split-K partials of the weight gradients, and the row-chunk partials
    // of the bias gradients
    const size_t colsum_part = (size_t)((B + kMlpColRows - 1) / kMlpColRows) * kMlpOut;
    L.acts[10] = take(sizeof(float) * std::max<size_t>((size_t)kMlpSlices * kMlpOut * kMlpIn, colsum_part));
    L.feat = take(sizeof(uint16_t) * B * kMlpIn);
    L.scale = take(sizeof(double) * B);
    L.total = off;
    return L;
}

nh_status mfail(nh_mlp *m, nh_status code, const char *msg)
{
    if (m) {
        m->err = msg;
        if (code == NH_EHIP) m->sticky = true;
    }
    return fail(nullptr, code, "%s", msg);
}

#define MLPCHK(m, call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return mfail((m), NH_EHIP, hipGetErrorString(e_));             \
    } while (0)

nh_status mlp_guard(const nh_mlp *m, int64_t batch)
{
    if (!m) return fail(nullptr, NH_EINVAL, "null MLP");
    if (m->sticky) return NH_ESTATE;
    if (batch <= 0 || batch > m->max_batch || batch % 64 != 0)
        return fail(nullptr, NH_EINVAL, "batch must be a positive multiple of 64 up to the capacity");
    return NH_OK;
}

// Glorot-uniform weights from a 64-bit LCG (seeded), zero biases; the last
// layer and the linear bypass start at zero so an untrained network returns
// the default guess.
void mlp_init_host(uint64_t seed, std::vector<float> &w)
{
    w.assign(mlp_nparam(), 0.0f);
    uint64_t s = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto uni = [&]() {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        return ((s >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
    };
    long off = 0;
    const int fan[3][2] = {{kMlpIn, kMlpHid}, {kMlpHid, kMlpHid}, {kMlpHid, kMlpOut}};
    for (int l = 0; l < 3; ++l) {
        const int fin = fan[l][0], fout = fan[l][1];
        const double a = sqrt(6.0 / (fin + fout));
        for (long i = 0; i < (long)fin * fout; ++i) {
            const int k = (int)(i % fin);
            w[off + i] = (l == 2 || (l == 0 && k >= kMlpNF + 3)) ? 0.0f : (float)(a * uni());
        }
        off += (long)fin * fout + fout;
    }
}

// Column parameters of the feature and guess kernels; the canonical column is
// the LGL nodes of order 4 in each of 16 equal elements of [0, 1].
MlpColParams mlp_col_params(const nh_ctx *c, double alpha)
{
    MlpColParams p{};
    p.nx = c->n[0]; p.ny = c->n[1]; p.nz = c->n[2];
    p.z = c->zl; p.lev = c->lev;
    p.alpha = alpha;
    p.gamma = c->phys.cp / c->phys.cv;
    std::vector<double> xi, w, D;
    lgl_basis(4, xi, w, D);
    for (int k = 0; k < kMlpNC; ++k) {
        const int e = std::min(k / 4, 15);
        p.zc[k] = (e + (xi[k - 4 * e] + 1.0) / 2.0) / 16.0;
    }
    p.zc[0] = 0.0;
    p.zc[kMlpNC - 1] = 1.0;
    return p;
}

}  // namespace

// First pass: x0 = b + N(alpha L_v b); each further pass applies the
// network to the residual its guess leaves, r = b - (I - alpha L_v) x0 (the
// exact correction of x0 is (I - alpha L_v)^-1 r, the same map as for the
// first pass), and adds the predicted correction in place.
nh_status mlp_guess(nh_mlp *m, nh_ctx *c, double alpha, const double *b, double *lb, double *x0)
{
    if (m->sticky) return fail(c, NH_ESTATE, "MLP in error state");
    const HeviParams hp = hevi_params(c);
    const MlpColParams cp = mlp_col_params(c, alpha);
    const long ncol = (long)c->n[0] * c->n[1];
    if (c->n[2] <= mlp_fused_max_nz()) {
        // residuals computed inside the inference kernel
        HIPCHK(c, launch_mlp_infer(cp, hp, m->net, b, false, b, nullptr, alpha, 0, ncol, x0, c->stream));
        for (int k = 1; k < m->passes && alpha > 0.0; ++k)
            HIPCHK(c, launch_mlp_infer(cp, hp, m->net, x0, true, b, nullptr, 1.0, 0, ncol, x0, c->stream));
        return NH_OK;
    }
    HIPCHK(c, launch_lv_apply(hp, b, lb, c->stream, false));
    HIPCHK(c, launch_mlp_infer(cp, hp, m->net, b, false, b, lb, alpha, 0, ncol, x0, c->stream));
    for (int k = 1; k < m->passes && alpha > 0.0; ++k) {
        HIPCHK(c, launch_lv_resid(hp, alpha, b, x0, lb, c->stream));
        HIPCHK(c, launch_mlp_infer(cp, hp, m->net, x0, true, b, lb, 1.0, 0, ncol, x0, c->stream));
    }
    return NH_OK;
}

extern "C" {

nh_status nh_mlp_workspace_bytes(int64_t max_batch, size_t *bytes)
{
    if (!bytes || max_batch <= 0 || max_batch % 64 != 0 || max_batch > (1 << 22))
        return fail(nullptr, NH_EINVAL, "max_batch must be a positive multiple of 64");
    *bytes = mlp_layout(max_batch).total;
    return NH_OK;
}

nh_status nh_mlp_create(int64_t max_batch, uint64_t seed, void *dev_ws, size_t bytes, void *hip_stream,
                        nh_mlp **out)
{
    if (!out) return fail(nullptr, NH_EINVAL, "null output");
    *out = nullptr;
    size_t need;
    nh_status st = nh_mlp_workspace_bytes(max_batch, &need);
    if (st) return st;
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(nullptr, NH_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(nullptr, NH_ESPACE, "MLP workspace %zu < %zu bytes", bytes, need);
    const MlpLayout L = mlp_layout(max_batch);
    nh_mlp *m = new nh_mlp();
    char *w = (char *)dev_ws;
    MlpNet &n = m->net;
    n.nparam = mlp_nparam();
    n.master = (float *)(w + L.params[0]);
    n.grad = (float *)(w + L.params[1]);
    n.m = (float *)(w + L.params[2]);
    n.v = (float *)(w + L.params[3]);
    n.half = w + L.params[4];
    const long offW[3] = {0, (long)kMlpHid * kMlpIn + kMlpHid,
                          (long)kMlpHid * kMlpIn + kMlpHid + (long)kMlpHid * kMlpHid + kMlpHid};
    const long offB[3] = {offW[0] + (long)kMlpHid * kMlpIn, offW[1] + (long)kMlpHid * kMlpHid,
                          offW[2] + (long)kMlpOut * kMlpHid};
    for (int l = 0; l < 3; ++l) {
        n.wh[l] = (const char *)n.half + sizeof(uint16_t) * offW[l];
        n.b[l] = n.master + offB[l];
        n.gw[l] = n.grad + offW[l];
        n.gb[l] = n.grad + offB[l];
    }
    const long offS = offB[2] + kMlpOut;   // linear bypass S [kMlpOut][kMlpIn]
    n.wh[3] = (const char *)n.half + sizeof(uint16_t) * offS;
    n.gw[3] = n.grad + offS;
    n.Z1 = (float *)(w + L.acts[0]); n.Z2 = (float *)(w + L.acts[1]); n.Y = (float *)(w + L.acts[2]);
    n.dY = (float *)(w + L.acts[3]); n.dH = (float *)(w + L.acts[4]); n.dZ = (float *)(w + L.acts[5]);
    n.part = (float *)(w + L.acts[6]); n.loss = (float *)(w + L.acts[7]);
    n.H1 = w + L.acts[8]; n.H2 = w + L.acts[9];
    n.part_k = (float *)(w + L.acts[10]);
    n.feat = w + L.feat; n.scale = (double *)(w + L.scale);
    m->max_batch = max_batch;
    m->step = 0;
    m->passes = 1;
    m->decay = 0.0f;
    m->stream = (hipStream_t)hip_stream;
    m->sticky = false;
    std::vector<float> h;
    mlp_init_host(seed, h);
    hipError_t e = hipMemcpyAsync(n.master, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n.m, 0, sizeof(float) * n.nparam, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n.v, 0, sizeof(float) * n.nparam, m->stream);
    if (e == hipSuccess) e = mlp_sync_half(n, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        delete m;
        return fail(nullptr, NH_EHIP, "nh_mlp_create: %s", hipGetErrorString(e));
    }
    *out = m;
    return NH_OK;
}

nh_status nh_mlp_forward(nh_mlp *m, int64_t batch, const void *dev_x_f16, float *dev_y)
{
    nh_status st = mlp_guard(m, batch);
    if (st) return st;
    if (!dev_x_f16) return mfail(m, NH_EINVAL, "null input");
    MLPCHK(m, mlp_forward(m->net, (int)batch, dev_x_f16, m->stream));
    if (dev_y)
        MLPCHK(m, hipMemcpyAsync(dev_y, m->net.Y, sizeof(float) * batch * kMlpOut, hipMemcpyDeviceToDevice,
                                 m->stream));
    return NH_OK;
}

nh_status nh_mlp_backward(nh_mlp *m, int64_t batch, const void *dev_x_f16, const float *dev_dy)
{
    nh_status st = mlp_guard(m, batch);
    if (st) return st;
    if (!dev_x_f16 || !dev_dy) return mfail(m, NH_EINVAL, "null input");
    MLPCHK(m, mlp_backward(m->net, (int)batch, dev_x_f16, dev_dy, m->stream));
    return NH_OK;
}

nh_status nh_mlp_train_step(nh_mlp *m, int64_t batch, const void *dev_x_f16, const float *dev_t, float lr,
                            float b1, float b2, float eps, float *dev_loss)
{
    nh_status st = mlp_guard(m, batch);
    if (st) return st;
    if (!dev_x_f16 || !dev_t) return mfail(m, NH_EINVAL, "null input");
    if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return mfail(m, NH_EINVAL, "bad Adam hyper-parameters");
    const int M = (int)batch;
    MLPCHK(m, mlp_forward(m->net, M, dev_x_f16, m->stream));
    MLPCHK(m, mlp_loss_grad(m->net, M, dev_t, m->net.loss, m->stream));
    MLPCHK(m, mlp_backward(m->net, M, dev_x_f16, m->net.dY, m->stream));
    ++m->step;
    MLPCHK(m, mlp_adam(m->net, lr, b1, b2, eps, m->step, m->decay, m->stream));
    if (dev_loss)
        MLPCHK(m, hipMemcpyAsync(dev_loss, m->net.loss, sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    return NH_OK;
}

nh_status nh_mlp_adam_step(nh_mlp *m, float lr, float b1, float b2, float eps)
{
    if (!m) return fail(nullptr, NH_EINVAL, "null MLP");
    if (m->sticky) return NH_ESTATE;
    if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return mfail(m, NH_EINVAL, "bad Adam hyper-parameters");
    ++m->step;
    MLPCHK(m, mlp_adam(m->net, lr, b1, b2, eps, m->step, m->decay, m->stream));
    return NH_OK;
}

nh_status nh_mlp_params(nh_mlp *m, float *dev_master, float *dev_grad, int64_t *n)
{
    if (!m) return fail(nullptr, NH_EINVAL, "null MLP");
    if (n) *n = m->net.nparam;
    if (dev_master)
        MLPCHK(m, hipMemcpyAsync(dev_master, m->net.master, sizeof(float) * m->net.nparam, hipMemcpyDeviceToDevice,
                                 m->stream));
    if (dev_grad)
        MLPCHK(m, hipMemcpyAsync(dev_grad, m->net.grad, sizeof(float) * m->net.nparam, hipMemcpyDeviceToDevice,
                                 m->stream));
    return NH_OK;
}

nh_status nh_mlp_set_params(nh_mlp *m, const float *dev_master)
{
    if (!m) return fail(nullptr, NH_EINVAL, "null MLP");
    if (m->sticky) return NH_ESTATE;
    if (!dev_master) return mfail(m, NH_EINVAL, "null parameters");
    MLPCHK(m, hipMemcpyAsync(m->net.master, dev_master, sizeof(float) * m->net.nparam, hipMemcpyDeviceToDevice,
                             m->stream));
    MLPCHK(m, hipMemsetAsync(m->net.m, 0, sizeof(float) * m->net.nparam, m->stream));
    MLPCHK(m, hipMemsetAsync(m->net.v, 0, sizeof(float) * m->net.nparam, m->stream));
    MLPCHK(m, mlp_sync_half(m->net, m->stream));
    m->step = 0;
    return NH_OK;
}

nh_status nh_mlp_samples(nh_mlp *m, nh_ctx *c, double alpha, const double *dev_b, const double *dev_x,
                         int64_t col0, int64_t ncol, void *dev_feat, double *dev_scale, float *dev_tgt,
                         double *dev_tmp, const double *dev_x0)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!m) return fail(c, NH_EINVAL, "null MLP");
    if (!dev_b || !dev_feat || !dev_scale || !dev_tmp || (dev_tgt && !dev_x))
        return fail(c, NH_EINVAL, "null arrays");
    const long nc = (long)c->n[0] * c->n[1];
    if (col0 < 0 || ncol <= 0 || col0 + ncol > nc) return fail(c, NH_EINVAL, "column range outside the lattice");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    const MlpColParams cp = mlp_col_params(c, alpha);
    if (dev_x0) {
        // the residual of the start x0, and the correction x - x0
        HIPCHK(c, launch_lv_resid(hevi_params(c), alpha, dev_b, dev_x0, dev_tmp, c->stream));
        HIPCHK(c, launch_mlp_features(cp, dev_x0, true, dev_tmp, 1.0, dev_x, col0, ncol, dev_feat, dev_scale, dev_tgt,
                                      c->stream));
        return NH_OK;
    }
    HIPCHK(c, launch_lv_apply(hevi_params(c), dev_b, dev_tmp, c->stream, false));
    HIPCHK(c, launch_mlp_features(cp, dev_b, false, dev_tmp, alpha, dev_x, col0, ncol, dev_feat, dev_scale, dev_tgt,
                                  c->stream));
    return NH_OK;
}

nh_status nh_mlp_set_decay(nh_mlp *m, float wd)
{
    if (!m) return fail(nullptr, NH_EINVAL, "null MLP");
    if (!(wd >= 0.0f && wd < 1e30f)) return mfail(m, NH_EINVAL, "weight decay must be finite and >= 0");
    m->decay = wd;
    return NH_OK;
}

nh_status nh_mlp_set_passes(nh_mlp *m, int32_t passes)
{
    if (!m) return fail(nullptr, NH_EINVAL, "null MLP");
    if (passes < 1 || passes > kMlpMaxPasses) return mfail(m, NH_EINVAL, "passes must be 1 .. 4");
    m->passes = passes;
    return NH_OK;
}

nh_status nh_mlp_guess(nh_mlp *m, nh_ctx *c, double alpha, const double *dev_b, double *dev_tmp, double *dev_x0)
{
    nh_status st = guard(c);
    if (st) return st;
    if (!m) return fail(c, NH_EINVAL, "null MLP");
    if (!dev_b || !dev_tmp || !dev_x0) return fail(c, NH_EINVAL, "null arrays");
    if (!c->have_ref) return fail(c, NH_EINVAL, "reference state not set");
    if (!(alpha >= 0.0 && alpha < 1e300)) return fail(c, NH_EINVAL, "alpha must be finite and >= 0");
    return mlp_guess(m, c, alpha, dev_b, dev_tmp, dev_x0);
}

nh_status nh_mlp_last_error(const nh_mlp *m, char *buf, size_t n)
{
    if (!buf || n == 0) return NH_EINVAL;
    snprintf(buf, n, "%s", m ? m->err.c_str() : g_last_global_error.c_str());
    return NH_OK;
}

nh_status nh_mlp_destroy(nh_mlp *m)
{
    if (!m) return NH_EINVAL;
    delete m;
    return NH_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched instances
// Many contexts (uneven limited-area instances, possibly of different
// orders) advanced together: per RK stage one grouped launch per order,
// whose workgroups take (instance, tile) items sorted longest-column-first
// and read their instance's parameters from a device descriptor table; a
// sequence of K steps (3 K launches per order group) is captured once as a
// hipGraph and replayed, after the per-stage descriptors of the next K steps
// are uploaded with one copy.
struct nh_batch {
    std::vector<nh_ctx *> ctx;
    int K, precision;
    // persistent: one persistent launch per (order group, stage) fed by a
    // device counter; concurrent: each order group's chain of launches on a
    // stream of its own inside the graph (the groups' launches overlap)
    bool persistent, concurrent;
    int *counters;        // device [K][3][groups]
    int persist_grid;     // workgroups of a persistent launch (one per CU)
    struct Group {
        int N, variant, nitems;
        int2 *work;   // device
        XcdLists xl;  // the group's items as one contiguous list per XCD
        int maxlen;   // longest of those lists
    };
    std::vector<Group> groups;
    std::vector<int> variant;  // tile variant of each instance (its order group's)
    StageParams *table;  // device [K][3][n]
    std::vector<StageParams> host;
    hipStream_t stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool captured, sticky;
    std::string err;
};

namespace {

// Workspace of a batch: the work lists (sized for the tile variant with the
// most tiles), the per-stage descriptor tables of K steps and the counters of
// the persistent launches (K steps x 3 stages x at most kMaxN - 1 order groups).
size_t batch_tables_bytes(int n, int K) { return align_up(sizeof(StageParams) * (size_t)K * 3 * n); }
// one counter per XCD list of every (step, stage, order group) launch
size_t batch_counter_bytes(int K) { return align_up(sizeof(int) * (size_t)K * 3 * (kMaxN - 1) * kXcds); }

size_t batch_bytes(nh_ctx *const *ctxs, int n, int K)
{
    size_t tiles = 0;
    for (int i = 0; i < n; ++i) {
        size_t most = 0;
        for (int v = 0; v < kTileVariants; ++v) {
            int tx, ty;
            stage_tile(ctxs[i]->N, v, &tx, &ty);
            most = std::max(most, (size_t)((ctxs[i]->n[0] + tx - 1) / tx) * ((ctxs[i]->n[1] + ty - 1) / ty));
        }
        tiles += most;
    }
    return align_up(sizeof(int2) * tiles) + batch_tables_bytes(n, K) + batch_counter_bytes(K);
}

nh_status bfail(nh_batch *b, nh_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) {
        b->err = buf;
        if (code == NH_EHIP) b->sticky = true;
    }
    g_last_global_error = buf;
    return code;
}

#define BCHK(b, call)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return bfail((b), NH_EHIP, "%s: %s", #call, hipGetErrorString(e_));    \
    } while (0)

}  // namespace

extern "C" {

nh_status nh_batch_workspace_bytes(nh_ctx *const *ctxs, int32_t n, int32_t steps_per_graph, size_t *bytes)
{
    if (!ctxs || n < 1 || n > 4096 || steps_per_graph < 1 || steps_per_graph > 1000 || !bytes)
        return fail(nullptr, NH_EINVAL, "bad batch arguments");
    for (int i = 0; i < n; ++i)
        if (!ctxs[i]) return fail(nullptr, NH_EINVAL, "null context %d", i);
    *bytes = batch_bytes(ctxs, n, steps_per_graph);
    return NH_OK;
}

nh_status nh_batch_create(nh_ctx *const *ctxs, int32_t n, int32_t steps_per_graph, const int32_t *tile_variant,
                          void *dev_ws, size_t bytes, void *hip_stream, nh_batch **out)
{
    if (!out) return fail(nullptr, NH_EINVAL, "null output");
    *out = nullptr;
    size_t need;
    nh_status st = nh_batch_workspace_bytes(ctxs, n, steps_per_graph, &need);
    if (st) return st;
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(nullptr, NH_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(nullptr, NH_ESPACE, "batch workspace %zu < %zu bytes", bytes, need);
    if (!hip_stream) return fail(nullptr, NH_EINVAL, "graph capture needs a non-default stream");
    const int prec = ctxs[0]->precision;
    for (int i = 0; i < n; ++i) {
        const nh_ctx *c = ctxs[i];
        if (c->sticky) return fail(nullptr, NH_ESTATE, "context %d is in an error state", i);
        if (!c->have_ref) return fail(nullptr, NH_EINVAL, "context %d has no reference state", i);
        if (c->precision != prec) return fail(nullptr, NH_EINVAL, "all instances must share one precision");
        if (c->hd_on) return fail(nullptr, NH_EUNSUPPORTED, "batched stages do not add the hyper-diffusion term");
        for (int f = 0; f < 4; ++f)
            if (c->nsnap[f]) return fail(nullptr, NH_EUNSUPPORTED, "batched stages fuse only the theta' forcing");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(nullptr, NH_EINVAL, "context %d appears twice", i);
    }
    nh_batch *b = new nh_batch();
    b->ctx.assign(ctxs, ctxs + n);
    b->K = steps_per_graph;
    b->precision = prec;
    b->stream = (hipStream_t)hip_stream;
    b->captured = false;
    b->sticky = false;
    b->graph = nullptr;
    b->exec = nullptr;
    b->persistent = false;
    b->concurrent = false;
    b->persist_grid = 256;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            b->persist_grid = cus;
    }
    char *w = (char *)dev_ws;
    int2 *work = (int2 *)w;
    size_t tiles_total = 0;
    // group by order; items sorted by column length (nel_z) descending
    std::vector<int2> all;
    for (int N = 2; N <= kMaxN; ++N) {
        const int var = tile_variant ? tile_variant[N] : 0;
        if (var < 0 || var >= kTileVariants) {
            delete b;
            return fail(nullptr, NH_EINVAL, "bad tile variant for order %d", N);
        }
        std::vector<std::pair<int, int2>> items;
        for (int i = 0; i < n; ++i) {
            if (ctxs[i]->N != N) continue;
            int tx, ty;
            stage_tile(N, var, &tx, &ty);
            const int ntx = (ctxs[i]->n[0] + tx - 1) / tx, nty = (ctxs[i]->n[1] + ty - 1) / ty;
            for (int t = 0; t < ntx * nty; ++t) items.push_back({ctxs[i]->nel[2], make_int2(i, t)});
        }
        if (items.empty()) continue;
        std::stable_sort(items.begin(), items.end(),
                         [](const std::pair<int, int2> &a, const std::pair<int, int2> &c) { return a.first > c.first; });
        // cut the sorted sequence (instances whole and in order, tiles
        // row-major) into kXcds contiguous runs of about equal cost (column
        // length): XCD x works through run x, so its concurrent workgroups
        // are neighbouring tiles whose halos meet in its L2
        nh_batch::Group g{N, var, (int)items.size(), work + tiles_total, XcdLists{}, 1};
        {
            double total = 0.0;
            for (auto &it : items) total += it.first;
            double acc = 0.0;
            int x = 0;
            g.xl.off[0] = 0;
            for (int j = 0; j < (int)items.size(); ++j) {
                acc += items[j].first;
                while (x < kXcds - 1 && acc >= total * (x + 1) / kXcds) g.xl.off[++x] = j + 1;
            }
            while (x < kXcds) g.xl.off[++x] = (int)items.size();
            for (int y = 0; y < kXcds; ++y) g.maxlen = std::max(g.maxlen, g.xl.off[y + 1] - g.xl.off[y]);
        }
        for (auto &it : items) all.push_back(it.second);
        tiles_total += items.size();
        b->groups.push_back(g);
    }
    b->variant.assign(n, 0);
    for (int i = 0; i < n; ++i)
        for (const auto &g : b->groups)
            if (g.N == ctxs[i]->N) b->variant[i] = g.variant;
    // descriptor tables and counters sit after the work lists (sized for the
    // tile variant with the most tiles)
    b->table = (StageParams *)(w + (need - batch_counter_bytes(steps_per_graph) -
                                    batch_tables_bytes(n, steps_per_graph)));
    b->counters = (int *)(w + (need - batch_counter_bytes(steps_per_graph)));
    b->host.resize((size_t)steps_per_graph * 3 * n);
    hipError_t e = hipMemcpyAsync(work, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return fail(nullptr, NH_EHIP, "nh_batch_create: %s", hipGetErrorString(e));
    }
    *out = b;
    return NH_OK;
}

nh_status nh_batch_step(nh_batch *b, double t, double dt, int32_t nsteps)
{
    if (!b) return fail(nullptr, NH_EINVAL, "null batch");
    if (b->sticky) return NH_ESTATE;
    if (nsteps < 0 || nsteps % b->K != 0)
        return bfail(b, NH_EINVAL, "nsteps must be a multiple of the %d steps per graph", b->K);
    if (!isfinite(t) || !isfinite(dt)) return bfail(b, NH_EINVAL, "bad time arguments");
    const int n = (int)b->ctx.size();
    for (int i = 0; i < n; ++i) {
        if (b->ctx[i]->sticky) return bfail(b, NH_ESTATE, "context %d in an error state", i);
        if (b->ctx[i]->hd_on)
            return bfail(b, NH_EUNSUPPORTED, "context %d has hyper-diffusion on: batched stages do not add it", i);
        for (int f = 0; f < 4; ++f)
            if (b->ctx[i]->nsnap[f])
                return bfail(b, NH_EUNSUPPORTED, "context %d has forcing on field %d: batched stages fuse only the "
                                                 "theta' forcing", i, f);
        if (b->ctx[i]->precision != b->precision)
            return bfail(b, NH_EINVAL, "context %d changed precision after the batch was created", i);
    }
    const double ca[3] = {0.0, 0.75, 1.0 / 3.0}, cb[3] = {1.0, 0.25, 2.0 / 3.0}, cc[3] = {1.0, 0.25, 2.0 / 3.0};
    const double ct[3] = {0.0, 1.0, 0.5};
    for (int r = 0; r < nsteps / b->K; ++r) {
        for (int k = 0; k < b->K; ++k) {
            const double ts = t + (double)(r * b->K + k) * dt;
            for (int s = 0; s < 3; ++s)
                for (int i = 0; i < n; ++i) {
                    nh_ctx *c = b->ctx[i];
                    const double *qs = s == 0 ? c->q[0] : (s == 1 ? c->q[1] : c->q[2]);
                    double *o = s == 0 ? c->q[1] : (s == 1 ? c->q[2] : c->q[0]);
                    b->host[((size_t)k * 3 + s) * n + i] =
                        stage_params(c, ts + ct[s] * dt, qs, s == 0 ? nullptr : c->q[0], o, ca[s], cb[s], cc[s] * dt,
                                     b->variant[i]);
                }
        }
        BCHK(b, hipMemcpyAsync(b->table, b->host.data(), sizeof(StageParams) * b->host.size(),
                               hipMemcpyHostToDevice, b->stream));
        if (!b->captured) {
            const int ng = (int)b->groups.size();
            // fork/join streams and events of the concurrent form (default
            // priority), released once the capture has ended
            std::vector<hipStream_t> gs;
            std::vector<hipEvent_t> ev;
            hipError_t e = hipSuccess;
            if (b->concurrent) {
                for (int g = 0; g < ng && e == hipSuccess; ++g) {
                    hipStream_t st = nullptr;
                    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
                    if (e == hipSuccess) gs.push_back(st);
                }
                for (int g = 0; g <= ng && e == hipSuccess; ++g) {
                    hipEvent_t x = nullptr;
                    e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
                    if (e == hipSuccess) ev.push_back(x);
                }
            }
            auto release = [&]() {
                for (auto st : gs) (void)hipStreamDestroy(st);
                for (auto x : ev) (void)hipEventDestroy(x);
            };
            if (e != hipSuccess) {
                release();
                return bfail(b, NH_EHIP, "streams for the concurrent form: %s", hipGetErrorString(e));
            }
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                release();
                return bfail(b, NH_EHIP, "begin capture: %s", hipGetErrorString(e));
            }
            // counters are cleared by a fill kernel (not a memset node)
            if (b->persistent) e = launch_zero_ints(b->counters, b->K * 3 * (kMaxN - 1) * kXcds, b->stream);
            if (b->concurrent && e == hipSuccess) {
                e = hipEventRecord(ev[ng], b->stream);
                for (int g = 0; g < ng && e == hipSuccess; ++g) e = hipStreamWaitEvent(gs[g], ev[ng], 0);
            }
            auto launch = [&](int k, int s, int g) {
                const auto &G = b->groups[g];
                int *ctr = b->persistent ? b->counters + (((size_t)k * 3 + s) * (kMaxN - 1) + g) * kXcds : nullptr;
                return launch_stage_batched(G.N, b->precision, G.variant, b->table + ((size_t)k * 3 + s) * n, G.work,
                                            G.xl, G.maxlen, ctr, b->persist_grid,
                                            b->concurrent ? gs[g] : b->stream);
            };
            if (b->concurrent) {
                for (int g = 0; g < ng && e == hipSuccess; ++g)
                    for (int k = 0; k < b->K && e == hipSuccess; ++k)
                        for (int s = 0; s < 3 && e == hipSuccess; ++s) e = launch(k, s, g);
                for (int g = 0; g < ng && e == hipSuccess; ++g) {
                    e = hipEventRecord(ev[g], gs[g]);
                    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev[g], 0);
                }
            } else {
                for (int k = 0; k < b->K && e == hipSuccess; ++k)
                    for (int s = 0; s < 3 && e == hipSuccess; ++s)
                        for (int g = 0; g < ng && e == hipSuccess; ++g) e = launch(k, s, g);
            }
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
            release();
            if (e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return bfail(b, NH_EHIP, "capture: %s", hipGetErrorString(e));
            }
            if (e2 != hipSuccess) return bfail(b, NH_EHIP, "end capture: %s", hipGetErrorString(e2));
            b->graph = graph;
            BCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->captured = true;
        }
        BCHK(b, hipGraphLaunch(b->exec, b->stream));
    }
    return NH_OK;
}

nh_status nh_batch_set_mode(nh_batch *b, int32_t persistent, int32_t concurrent_groups)
{
    if (!b) return fail(nullptr, NH_EINVAL, "null batch");
    if (b->sticky) return NH_ESTATE;
    if ((persistent != 0 && persistent != 1) || (concurrent_groups != 0 && concurrent_groups != 1))
        return bfail(b, NH_EINVAL, "mode flags must be 0 or 1");
    b->persistent = persistent != 0;
    b->concurrent = concurrent_groups != 0;
    // the next step captures the graph again
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured = false;
    return NH_OK;
}

nh_status nh_batch_last_error(const nh_batch *b, char *buf, size_t n)
{
    if (!buf || n == 0) return NH_EINVAL;
    snprintf(buf, n, "%s", b ? b->err.c_str() : g_last_global_error.c_str());
    return NH_OK;
}

nh_status nh_batch_destroy(nh_batch *b)
{
    if (!b) return NH_EINVAL;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return NH_OK;
}

}  // extern "C"
