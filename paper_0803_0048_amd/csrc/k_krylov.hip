// Krylov building blocks for right-preconditioned restarted GMRES and
// BiCGSTAB on gfx950.
//
// The paper keeps inner products sequential so that their bits do not depend
// on the number of threads (Sec. 3.5).  Here every reduction instead has one
// fixed shape that depends only on the vector length: 16384 lanes each sum a
// strided subsequence in ascending order from +0.0, then lanes are combined
// pairwise at strides 1, 2, 4, ..., 8192 (IEEE addition is commutative, so
// which lane of a pair does the add does not matter).  The launch is
// 64 blocks x 256 threads = 16384 threads; strides 1..32 are combined inside a
// wavefront with shuffles, 64 and 128 through LDS, 256..8192 over the 64
// block partials by whichever kernel consumes the result.  SpMV sums every
// row from +0.0 in ascending column order, one thread per row.
#include "kernels.h"

namespace tpilu {

__global__ void k_spmv(int32_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ v, const double* __restrict__ x,
                       const double* __restrict__ b_minus, double* __restrict__ y) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s = s + v[p] * x[ci[p]];
        y[i] = b_minus ? b_minus[i] - s : s;
    }
}

hipError_t launch_spmv(int32_t n, const int64_t* rp, const int32_t* ci, const double* v,
                       const double* x, const double* b_minus, double* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int blocks = std::min((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_spmv, dim3(blocks), dim3(256), 0, s, n, rp, ci, v, x, b_minus, y);
    return hipGetLastError();
}

// pairwise tree inside a wavefront: lane l (l a multiple of 2w) += lane l+w
__device__ __forceinline__ double wave_tree(double s) {
    const int lane = lane_id();
    for (int w = 1; w < kWave; w <<= 1) {
        const double o = __shfl_down(s, w, kWave);
        if ((lane & (2 * w - 1)) == 0) s = s + o;
    }
    return s;
}

__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     double* __restrict__ partial) {
    __shared__ double sh[4];
    const int64_t l = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
    double s = 0.0;
    for (int64_t e = l; e < n; e += kDotLanes) s = s + x[e] * y[e];
    s = wave_tree(s);
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) sh[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double a = sh[0] + sh[1];  // stride 64
        const double c = sh[2] + sh[3];
        partial[blockIdx.x] = a + c;     // stride 128
    }
}

// strides 256..8192: tree over the 64 block partials
__device__ __forceinline__ double tree64(const double* __restrict__ partial) {
    double p[kDotBlocks];
#pragma unroll
    for (int b = 0; b < kDotBlocks; ++b) p[b] = partial[b];
#pragma unroll
    for (int w = 1; w < kDotBlocks; w <<= 1) {
#pragma unroll
        for (int b = 0; b < kDotBlocks; b += 2 * w) p[b] = p[b] + p[b + w];
    }
    return p[0];
}

hipError_t launch_dot_partial(int64_t n, const double* x, const double* y, double* partial,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(kDotThreads), 0, s, n, x, y, partial);
    return hipGetLastError();
}

__global__ void k_dot_final(const double* __restrict__ partial, double* out, int sqrt_it) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double r = tree64(partial);
        if (sqrt_it) r = __builtin_sqrt(r);
        *out = r;
    }
}

hipError_t launch_dot_final(const double* partial, double* out, int sqrt_it, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, s, partial, out, sqrt_it);
    return hipGetLastError();
}

// scalar of a finished reduction, computed once per block and broadcast
__device__ __forceinline__ double block_scalar(const double* partial, int sqrt_it) {
    __shared__ double sc;
    if (threadIdx.x == 0) {
        double r = tree64(partial);
        sc = sqrt_it ? __builtin_sqrt(r) : r;
    }
    __syncthreads();
    return sc;
}

// MGS step: h = <w, v> (from its partials); H slot <- h; w <- w - h v
__global__ __launch_bounds__(256) void k_gm_axpy_h(int64_t n, const double* __restrict__ partial,
                                                   double* hslot, double* __restrict__ w,
                                                   const double* __restrict__ v) {
    const double h = block_scalar(partial, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *hslot = h;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        w[e] = w[e] - h * v[e];
}

hipError_t launch_gm_axpy_h(int64_t n, const double* partial, double* hslot, double* w,
                            const double* v, hipStream_t s) {
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_gm_axpy_h, dim3(blocks), dim3(256), 0, s, n, partial, hslot, w, v);
    return hipGetLastError();
}

// h_{j+1,j} = ||w||; v_{j+1} = w / h_{j+1,j} when it is not zero
__global__ __launch_bounds__(256) void k_gm_norm_scale(int64_t n, const double* __restrict__ partial,
                                                       double* hslot, const double* __restrict__ w,
                                                       double* __restrict__ vnext) {
    const double hn = block_scalar(partial, 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) *hslot = hn;
    if (hn == 0.0) return;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        vnext[e] = w[e] / hn;
}

hipError_t launch_gm_norm_scale(int64_t n, const double* partial, double* hslot, const double* w,
                                double* vnext, hipStream_t s) {
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_gm_norm_scale, dim3(blocks), dim3(256), 0, s, n, partial, hslot, w, vnext);
    return hipGetLastError();
}

// cycle start: beta = ||r||, g_0 = beta, v_0 = r / beta
__global__ __launch_bounds__(256) void k_gm_start(int64_t n, const double* __restrict__ partial,
                                                  double* beta_slot, double* g0,
                                                  const double* __restrict__ r,
                                                  double* __restrict__ v0) {
    const double beta = block_scalar(partial, 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *beta_slot = beta;
        *g0 = beta;
    }
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        v0[e] = r[e] / beta;
}

hipError_t launch_gm_start(int64_t n, const double* partial, double* beta_slot, double* g0,
                           const double* r, double* v0, hipStream_t s) {
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_gm_start, dim3(blocks), dim3(256), 0, s, n, partial, beta_slot, g0, r, v0);
    return hipGetLastError();
}

// The rotation that zeroes b against a: rho = sqrt(a*a + b*b) (each product
// and the sum rounded on its own, no hypot), c = a / rho, s = b / rho, all
// correctly rounded binary64 operations.
struct Rotation {
    double rho, c, s;
};
__device__ __forceinline__ Rotation givens_rotation(double a, double b) {
    Rotation r;
    r.rho = __builtin_sqrt(a * a + b * b);
    r.c = a / r.rho;
    r.s = b / r.rho;
    return r;
}

__global__ void k_givens_batch(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                               double* rho, double* c, double* s) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const Rotation r = givens_rotation(a[i], b[i]);
        rho[i] = r.rho;
        c[i] = r.c;
        s[i] = r.s;
    }
}

hipError_t launch_givens_batch(int64_t n, const double* a, const double* b, double* rho, double* c, double* s,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_givens_batch, dim3(blocks), dim3(256), 0, st, n, a, b, rho, c, s);
    return hipGetLastError();
}

// Givens: apply rotations 0..j-1 to column j of H, form rotation j with
// rho = sqrt(a*a + b*b) (no hypot), update g, count the iteration and decide
// whether the cycle stops (|g_{j+1}| <= tol, maxit reached, or breakdown).
// H is (m+1) x m, row-major: H[i * m + j].
__global__ void k_gm_givens(double* H, double* cs, double* sn, double* g, int32_t m, int32_t j,
                            double tol, int32_t* iters, int32_t maxit, double* hist, int32_t* stop) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double hn = H[(j + 1) * m + j];
    for (int32_t i = 0; i < j; ++i) {
        const double a = H[i * m + j], c = H[(i + 1) * m + j];
        const double tau = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = cs[i] * c - sn[i] * a;
        H[i * m + j] = tau;
    }
    const Rotation rot = givens_rotation(H[j * m + j], H[(j + 1) * m + j]);
    cs[j] = rot.c;
    sn[j] = rot.s;
    H[j * m + j] = rot.rho;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const int32_t it = *iters;
    const double res = __builtin_fabs(g[j + 1]);
    if (hist) hist[it] = res;
    *iters = it + 1;
    *stop = (res <= tol || it + 1 >= maxit || hn == 0.0) ? 1 : 0;
}

hipError_t launch_gm_givens(double* H, double* cs, double* sn, double* g, int32_t m, int32_t j,
                            double tol, int32_t* iters, int32_t maxit, double* hist,
                            int32_t* stop, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(64), 0, s, H, cs, sn, g, m, j, tol, iters, maxit,
                       hist, stop);
    return hipGetLastError();
}

// back substitution H(0:jj, 0:jj) y = g, i descending, running subtraction
// in ascending l
__global__ void k_gm_backsub(const double* H, const double* g, double* yv, int32_t m, int32_t jj) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int32_t i = jj - 1; i >= 0; --i) {
        double s = g[i];
        for (int32_t l = i + 1; l < jj; ++l) s = s - H[i * m + l] * yv[l];
        yv[i] = s / H[i * m + i];
    }
}

hipError_t launch_gm_backsub(const double* H, const double* g, double* yv, int32_t m, int32_t jj,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_gm_backsub, dim3(1), dim3(64), 0, s, H, g, yv, m, jj);
    return hipGetLastError();
}

// u_e = sum_i y_i v_{i,e}, from +0.0 in ascending i
__global__ void k_gm_combine(int64_t n, const double* __restrict__ V, const double* __restrict__ yv,
                             int32_t jj, double* __restrict__ u) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t i = 0; i < jj; ++i) s = s + yv[i] * V[(int64_t)i * n + e];
        u[e] = s;
    }
}

hipError_t launch_gm_combine(int64_t n, const double* V, const double* yv, int32_t jj, double* u,
                             hipStream_t s) {
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_gm_combine, dim3(blocks), dim3(256), 0, s, n, V, yv, jj, u);
    return hipGetLastError();
}

__global__ void k_axpy1(int64_t n, double* __restrict__ x, const double* __restrict__ z) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        x[e] = x[e] + z[e];
}

hipError_t launch_axpy1(int64_t n, double* x, const double* z, hipStream_t s) {
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_axpy1, dim3(blocks), dim3(256), 0, s, n, x, z);
    return hipGetLastError();
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace tpilu

namespace tpilu {

// ----------------------------------------------------------------------------------
// BiCGSTAB steps.  Scalars live in sc[] on the device (kBi* slots); every
// thread that needs one derives it from the same stored values with the same
// expression, so all of them hold the same bits.
// ----------------------------------------------------------------------------------
// rho_old <- rho, rho <- (rs, r) from its partials
__global__ void k_bi_rho(const double* __restrict__ partial, double* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc[kBiRhoOld] = sc[kBiRho];
        sc[kBiRho] = tree64(partial);
    }
}

// p <- r (first pass) or p_e <- r_e + beta * (p_e - omega * v_e),
// beta = (rho / rho_old) * (alpha / omega)
__global__ __launch_bounds__(256) void k_bi_p(int64_t n, int first, const double* __restrict__ sc,
                                              const double* __restrict__ r, double* __restrict__ p,
                                              const double* __restrict__ v) {
    const double omega = sc[kBiOmega];
    const double beta = (sc[kBiRho] / sc[kBiRhoOld]) * (sc[kBiAlpha] / omega);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = first ? r[e] : r[e] + beta * (p[e] - omega * v[e]);
}

// rv = (rs, v); alpha = rho / rv (rv == 0: breakdown flag, alpha left alone)
__global__ void k_bi_alpha(const double* __restrict__ partial, double* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double rv = tree64(partial);
        sc[kBiRv] = rv;
        if (rv != 0.0) sc[kBiAlpha] = sc[kBiRho] / rv;
    }
}

// s_e = r_e - alpha * v_e (skipped after a breakdown)
__global__ __launch_bounds__(256) void k_bi_s(int64_t n, const double* __restrict__ sc, const double* __restrict__ r,
                                              const double* __restrict__ v, double* __restrict__ s) {
    if (sc[kBiRv] == 0.0) return;
    const double alpha = sc[kBiAlpha];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        s[e] = r[e] - alpha * v[e];
}

// x_e = x_e + alpha * ph_e (the exit after the first half of a step)
__global__ __launch_bounds__(256) void k_bi_x_half(int64_t n, const double* __restrict__ sc, double* __restrict__ x,
                                                   const double* __restrict__ ph) {
    const double alpha = sc[kBiAlpha];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] = x[e] + alpha * ph[e];
}

// ts = (t, s), tt = (t, t); omega = ts / tt (tt == 0: breakdown, omega left alone)
__global__ void k_bi_omega(const double* __restrict__ pts, const double* __restrict__ ptt, double* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double ts = tree64(pts), tt = tree64(ptt);
        sc[kBiTt] = tt;
        if (tt != 0.0) sc[kBiOmega] = ts / tt;
    }
}

// x_e = (x_e + alpha * ph_e) + omega * sh_e; r_e = s_e - omega * t_e (skipped after a breakdown)
__global__ __launch_bounds__(256) void k_bi_xr(int64_t n, const double* __restrict__ sc, double* __restrict__ x,
                                               double* __restrict__ r, const double* __restrict__ ph,
                                               const double* __restrict__ sh, const double* __restrict__ s,
                                               const double* __restrict__ t) {
    if (sc[kBiTt] == 0.0) return;
    const double alpha = sc[kBiAlpha], omega = sc[kBiOmega];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        x[e] = (x[e] + alpha * ph[e]) + omega * sh[e];
        r[e] = s[e] - omega * t[e];
    }
}

namespace {
int vec_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }
}  // namespace

hipError_t launch_bi(int op, int64_t n, int first, const double* pa, const double* pb, double* sc, double* x,
                     double* r, const double* a1, const double* a2, const double* a3, const double* a4,
                     hipStream_t s) {
    switch (op) {
        case kBiOpRho:
            hipLaunchKernelGGL(k_bi_rho, dim3(1), dim3(64), 0, s, pa, sc);
            break;
        case kBiOpP:  // r = a1, p = x (in/out), v = a2
            hipLaunchKernelGGL(k_bi_p, dim3(vec_blocks(n)), dim3(256), 0, s, n, first, sc, a1, x, a2);
            break;
        case kBiOpAlpha:
            hipLaunchKernelGGL(k_bi_alpha, dim3(1), dim3(64), 0, s, pa, sc);
            break;
        case kBiOpS:  // r = a1, v = a2, s = x
            hipLaunchKernelGGL(k_bi_s, dim3(vec_blocks(n)), dim3(256), 0, s, n, sc, a1, a2, x);
            break;
        case kBiOpXHalf:  // x, ph = a1
            hipLaunchKernelGGL(k_bi_x_half, dim3(vec_blocks(n)), dim3(256), 0, s, n, sc, x, a1);
            break;
        case kBiOpOmega:
            hipLaunchKernelGGL(k_bi_omega, dim3(1), dim3(64), 0, s, pa, pb, sc);
            break;
        case kBiOpXR:  // x, r, ph = a1, sh = a2, s = a3, t = a4
            hipLaunchKernelGGL(k_bi_xr, dim3(vec_blocks(n)), dim3(256), 0, s, n, sc, x, r, a1, a2, a3, a4);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tpilu
