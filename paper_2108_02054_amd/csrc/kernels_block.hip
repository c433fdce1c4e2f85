// kernels_block.hip -- damped block Jacobi for systems with B unknowns per node (the
// paper's 4x4-block systems, Section 4, where every matrix value is a block and the
// Jacobi smoother inverts the diagonal block).  Unknown b of node I is row I*B + b; the
// smoother of a level holds omega * D_I^{-1} for every node, row-major, B*B values per node.
//
// The inverse is Gauss-Jordan elimination with partial pivoting on [D_I | I], in the
// order of its definition (the first row of largest magnitude in the column is the pivot),
// with separately rounded products, so that in FP64 it reproduces the definition's
// rounding.  B is a compile-time constant (2..8): the working block stays in registers.
#include "amg_internal.h"

#pragma clang fp contract(off)

namespace amgmi {

constexpr int TPB_B = 256;

// One thread per node.  Values are read in T (FP64, or the FP32 copies of a mixed
// hierarchy), the elimination runs in FP64 and the result is stored in T.  A zero pivot
// (singular block) sets flags[F_NOT_SPD] when flags is given; the block then holds
// non-finite values.
template <int B, typename T>
__global__ __launch_bounds__(TPB_B) void k_block_inv(int nn, const int* __restrict__ ptr, const int* __restrict__ col,
                                                     const T* __restrict__ val, double omega, T* __restrict__ m,
                                                     int* __restrict__ flags) {
    const int I = xcd_block() * TPB_B + threadIdx.x;
    if (I >= nn) return;
    double W[B][2 * B];
#pragma unroll
    for (int a = 0; a < B; ++a) {
#pragma unroll
        for (int q = 0; q < 2 * B; ++q) W[a][q] = (q == B + a) ? 1.0 : 0.0;
    }
    const int c0 = I * B;
#pragma unroll
    for (int a = 0; a < B; ++a) {
        const int r = c0 + a;
        int k = ptr[r];
        const int e = ptr[r + 1];
        while (k < e && col[k] < c0) ++k;  // first entry of the diagonal block
#pragma unroll
        for (int q = 0; q < B; ++q) {
            // every stored block is full, so these are columns c0 .. c0 + B - 1
            if (k + q < e && col[k + q] == c0 + q) W[a][q] = (double)val[k + q];
        }
    }
    bool singular = false;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        int piv = k;
        double best = fabs(W[k][k]);
#pragma unroll
        for (int a = k + 1; a < B; ++a) {
            const double v = fabs(W[a][k]);
            if (v > best) {
                best = v;
                piv = a;
            }
        }
        if (best == 0.0) singular = true;
        // swap rows k and piv (selects, so the block stays in registers)
#pragma unroll
        for (int a = k + 1; a < B; ++a) {
            if (a == piv) {
#pragma unroll
                for (int q = 0; q < 2 * B; ++q) {
                    const double t = W[k][q];
                    W[k][q] = W[a][q];
                    W[a][q] = t;
                }
            }
        }
        const double d = W[k][k];
#pragma unroll
        for (int q = 0; q < 2 * B; ++q) W[k][q] = W[k][q] / d;
#pragma unroll
        for (int a = 0; a < B; ++a) {
            if (a == k) continue;
            const double f = W[a][k];
#pragma unroll
            for (int q = 0; q < 2 * B; ++q) W[a][q] = W[a][q] - f * W[k][q];
        }
    }
    if (singular && flags != nullptr) atomicOr(&flags[F_NOT_SPD], 1);
    T* out = m + (size_t)I * B * B;
#pragma unroll
    for (int a = 0; a < B; ++a) {
#pragma unroll
        for (int q = 0; q < B; ++q) out[a * B + q] = (T)(omega * W[a][B + q]);
    }
}

// uout_i = uin_i + sum_q M_I[a][q] r_{I*B+q} for row i = I*B + a (uin == nullptr: zero);
// the block row product is summed in column order before it is added.
template <int B, typename T>
__global__ __launch_bounds__(TPB_B) void k_block_apply(int n, const T* __restrict__ m, const T* __restrict__ r,
                                                       const T* __restrict__ uin, T* __restrict__ uout) {
    const int i = xcd_block() * TPB_B + threadIdx.x;
    if (i >= n) return;
    const int base = i - i % B;
    const T* mi = m + (size_t)i * B;
    T s = 0;
#pragma unroll
    for (int q = 0; q < B; ++q) s = s + mi[q] * r[base + q];
    uout[i] = uin != nullptr ? uin[i] + s : s;
}

static unsigned bgrid(int64_t n) {
    const int64_t b = (n + TPB_B - 1) / TPB_B;
    return (unsigned)(b > 0 ? b : 1);
}

#define AMG_WITH_B(B_, ...)                                             \
    switch (B_) {                                                       \
        case 2: { constexpr int B = 2; __VA_ARGS__; } break;            \
        case 3: { constexpr int B = 3; __VA_ARGS__; } break;            \
        case 4: { constexpr int B = 4; __VA_ARGS__; } break;            \
        case 5: { constexpr int B = 5; __VA_ARGS__; } break;            \
        case 6: { constexpr int B = 6; __VA_ARGS__; } break;            \
        case 7: { constexpr int B = 7; __VA_ARGS__; } break;            \
        case 8: { constexpr int B = 8; __VA_ARGS__; } break;            \
        default: throw Fail{AMG_ERR_ARG, "block_size must be 1 .. 8"}; \
    }

template <typename T>
void launch_block_inv(const Csr& A, int B_, double omega, T* m, int* flags, hipStream_t s) {
    const int nn = A.nrows / B_;
    AMG_WITH_B(B_, k_block_inv<B, T><<<bgrid(nn), TPB_B, 0, s>>>(nn, A.ptr, A.col, A.v<T>(), omega, m, flags));
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_block_apply(int n, int B_, const T* m, const T* r, const T* uin, T* uout, hipStream_t s) {
    AMG_WITH_B(B_, k_block_apply<B, T><<<bgrid(n), TPB_B, 0, s>>>(n, m, r, uin, uout));
    HIP_LAUNCH_CHECK();
}

template void launch_block_inv<double>(const Csr&, int, double, double*, int*, hipStream_t);
template void launch_block_inv<float>(const Csr&, int, double, float*, int*, hipStream_t);
template void launch_block_apply<double>(int, int, const double*, const double*, const double*, double*, hipStream_t);
template void launch_block_apply<float>(int, int, const float*, const float*, const float*, float*, hipStream_t);

}  // namespace amgmi
