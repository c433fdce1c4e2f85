// kernels_logcoef.hip -- the differentiable form: a 7-point diffusion operator whose
// per-cell coefficients are k = exp(theta), and the adjoint scatter of its gradient.
//
// Pattern: cell c = x + nx*(y + ny*z); row c lists its neighbours in increasing column
// order (z-1, y-1, x-1, c, x+1, y+1, z+1), missing neighbours omitted.  Face coefficient
// w = 2 k_c k_j / (k_c + k_j) (harmonic mean), a_cj = -w; a missing neighbour is a ghost
// cell with the cell's own k and adds k_c to the diagonal.
//
// One thread per cell; both kernels gather from neighbours, so no atomics are needed.
#include "amg_internal.h"

namespace amgmi {

constexpr int TPB = 256;

struct Cell {
    int64_t nb[6];
    int cnt;        // neighbours present
    int nlower;     // neighbours with a smaller index (they precede the diagonal)
};

__device__ __forceinline__ Cell neighbours(int nx, int ny, int nz, int64_t c) {
    const int64_t pl = (int64_t)nx * ny;
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / pl);
    Cell r;
    r.cnt = 0;
    if (z > 0) r.nb[r.cnt++] = c - pl;
    if (y > 0) r.nb[r.cnt++] = c - nx;
    if (x > 0) r.nb[r.cnt++] = c - 1;
    r.nlower = r.cnt;
    if (x < nx - 1) r.nb[r.cnt++] = c + 1;
    if (y < ny - 1) r.nb[r.cnt++] = c + nx;
    if (z < nz - 1) r.nb[r.cnt++] = c + pl;
    return r;
}

// Offset of row c in the CSR arrays: 7c minus the entries of earlier rows that are
// missing because those cells touch the boundary (one count per missing face).
__device__ __forceinline__ int64_t row_start(int nx, int ny, int nz, int64_t c) {
    const int64_t pl = (int64_t)nx * ny;
    const int64_t line = c / nx, plane = c / pl;
    const int x = (int)(c % nx), y = (int)(line % ny), z = (int)plane;
    const int64_t x0 = line + (x > 0 ? 1 : 0);                        // earlier cells with x = 0
    const int64_t x1 = line;                                          // earlier cells with x = nx-1
    const int64_t y0 = plane * nx + (y > 0 ? nx : x);                 // earlier cells with y = 0
    const int64_t y1 = plane * nx + (y == ny - 1 ? x : 0);            // earlier cells with y = ny-1
    const int64_t z0 = z > 0 ? pl : c;                                // earlier cells with z = 0
    const int64_t z1 = z == nz - 1 ? c - (int64_t)(nz - 1) * pl : 0;  // earlier cells with z = nz-1
    return 7 * c - (x0 + x1 + y0 + y1 + z0 + z1);
}

__global__ void k_logcoef7_assemble(int nx, int ny, int nz, const double* __restrict__ theta,
                                    double* __restrict__ val) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (c >= n) return;
    const Cell cl = neighbours(nx, ny, nz, c);
    const double kc = exp(theta[c]);
    int64_t pos = row_start(nx, ny, nz, c);
    double diag = 0.0;
    int64_t dpos = pos + cl.nlower;
    for (int q = 0; q < cl.cnt; ++q) {
        const double kj = exp(theta[cl.nb[q]]);
        const double w = 2.0 * kc * kj / (kc + kj);
        diag += w;
        const int64_t p = pos + q + (q >= cl.nlower ? 1 : 0);
        val[p] = -w;
    }
    diag += (6 - cl.cnt) * kc;
    val[dpos] = diag;
}

// g_c = -lambda^T (dA/dtheta_c) u.  With dw/dtheta_c = k_c dw/dk_c = 2 k_c k_j^2 / (k_c + k_j)^2
// for each face of c, and d(ghost term)/dtheta_c = k_c:
//   g_c = -sum_faces dw (lambda_c - lambda_j)(u_c - u_j) - (missing faces) k_c lambda_c u_c.
__global__ void k_logcoef7_adjoint(int nx, int ny, int nz, const double* __restrict__ theta,
                                   const double* __restrict__ u, const double* __restrict__ lam,
                                   double* __restrict__ grad) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (c >= n) return;
    const Cell cl = neighbours(nx, ny, nz, c);
    const double kc = exp(theta[c]);
    const double lc = lam[c], uc = u[c];
    double g = 0.0;
    for (int q = 0; q < cl.cnt; ++q) {
        const int64_t j = cl.nb[q];
        const double kj = exp(theta[j]);
        const double dw = 2.0 * kc * kj * kj / ((kc + kj) * (kc + kj));
        g -= dw * (lc - lam[j]) * (uc - u[j]);
    }
    g -= (6 - cl.cnt) * kc * lc * uc;
    grad[c] = g;
}

static unsigned cell_blocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    return (unsigned)(b > 0 ? b : 1);
}

void launch_logcoef7_assemble(int nx, int ny, int nz, const double* theta, double* val, hipStream_t s) {
    k_logcoef7_assemble<<<cell_blocks((int64_t)nx * ny * nz), TPB, 0, s>>>(nx, ny, nz, theta, val);
    HIP_LAUNCH_CHECK();
}

void launch_logcoef7_adjoint(int nx, int ny, int nz, const double* theta, const double* u, const double* lam,
                             double* grad, hipStream_t s) {
    k_logcoef7_adjoint<<<cell_blocks((int64_t)nx * ny * nz), TPB, 0, s>>>(nx, ny, nz, theta, u, lam, grad);
    HIP_LAUNCH_CHECK();
}

}  // namespace amgmi
