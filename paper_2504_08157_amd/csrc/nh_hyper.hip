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

// out[f] = scale * L q[f] (or out[f] += scale * L q[f] with accumulate) for
// the 5 fields of q [5][U]; one thread per node, x taps coalesced, y and z
// taps strided (cached).  Zero taps are skipped.
__global__ void __launch_bounds__(256) hd_laplace_kernel(HyperParams h, const double *__restrict__ q,
                                                         double *__restrict__ out, double scale, int accumulate)
{
    const long nxy = (long)h.nx * h.ny;
    const long U = nxy * h.nz;
    const int N = h.N, NC = 2 * N + 1;
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < U; I += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(I % h.nx), iy = (int)((I / h.nx) % h.ny), iz = (int)(I / nxy);
        double acc[kNF];
#pragma unroll
        for (int f = 0; f < kNF; ++f) acc[f] = 0.0;
        // x
        {
            const double *S = h.sx + (long)ix * NC;
            for (int o = 0; o < NC; ++o) {
                const double cf = S[o];
                if (cf == 0.0) continue;
                int j = ix + o - N;
                if (j < 0 || j >= h.nx) {
                    if (!h.perx) continue;
                    j += j < 0 ? h.nx : -h.nx;
                }
                const long J = I + (j - ix);
#pragma unroll
                for (int f = 0; f < kNF; ++f) acc[f] += cf * q[f * U + J];
            }
        }
        // y
        {
            const double *S = h.sy + (long)iy * NC;
            for (int o = 0; o < NC; ++o) {
                const double cf = S[o];
                if (cf == 0.0) continue;
                int j = iy + o - N;
                if (j < 0 || j >= h.ny) {
                    if (!h.pery) continue;
                    j += j < 0 ? h.ny : -h.ny;
                }
                const long J = I + (long)(j - iy) * h.nx;
#pragma unroll
                for (int f = 0; f < kNF; ++f) acc[f] += cf * q[f * U + J];
            }
        }
        // z (walls)
        {
            const double *S = h.sz + (long)iz * NC;
            for (int o = 0; o < NC; ++o) {
                const double cf = S[o];
                if (cf == 0.0) continue;
                const int j = iz + o - N;
                if (j < 0 || j >= h.nz) continue;
                const long J = I + (long)(j - iz) * nxy;
#pragma unroll
                for (int f = 0; f < kNF; ++f) acc[f] += cf * q[f * U + J];
            }
        }
#pragma unroll
        for (int f = 0; f < kNF; ++f) out[f * U + I] = (accumulate ? out[f * U + I] : 0.0) + scale * acc[f];
    }
}

hipError_t launch_hd_laplace(const HyperParams &h, const double *q, double *out, double scale, bool accumulate,
                             hipStream_t s)
{
    const long U = (long)h.nx * h.ny * h.nz;
    long blocks = (U + 255) / 256;
    if (blocks > 65535L * 8) blocks = 65535L * 8;
    hipLaunchKernelGGL(hd_laplace_kernel, dim3((unsigned)blocks), dim3(256), 0, s, h, q, out, scale,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace nh
