// Bandwidth-bound tensor kernels of the compression step (gfx950).
//
// These kernels move each element once: the structured MPO application
// (the one-qubit gates and the operator-Schmidt factors of the two-qubit
// gates, Sec. IV.B.2 / eq:SVD), layout changes of site tensors, precision
// conversions, FP64 reductions, the selection of eigenvectors for the
// truncation and the per-row step of sequential sampling.  Threads are mapped
// so that consecutive lanes touch consecutive addresses of the fastest index.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mpsk {

static inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 1048576) g = 1048576;  // grid-stride loops cover the rest
    if (g < 1) g = 1;
    return (unsigned)g;
}

// ---------------------------------------------------------------- MPO ------
template <typename T>
struct MpoOpT {
    int r_in, r_out, lo, H, out_ws;
    T re[16], im[16];
};

template <typename T>
__global__ __launch_bounds__(256) void mpo_apply_kernel(MpoOpT<T> op, int64_t P, int64_t Q,
                                                        const T* __restrict__ in_re,
                                                        const T* __restrict__ in_im,
                                                        T* __restrict__ out_re,
                                                        T* __restrict__ out_im) {
    const int r_in = op.r_in, r_out = op.r_out, lo = op.lo, H = op.H;
    const int64_t w_in = (int64_t)H * r_in * lo, w_out = (int64_t)H * r_out * lo;
    const int64_t total = P * H * lo * Q;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = idx % Q;
        int64_t rest = idx / Q;
        const int64_t l = rest % lo;
        rest /= lo;
        const int64_t h = rest % H;
        const int64_t p = rest / H;
        T xr[8], xi[8];  // [a_in][t], r_in <= 4
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a < r_in) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int64_t off = ((p * w_in + (h * r_in + a) * lo + l) * 2 + t) * Q + q;
                    xr[a * 2 + t] = in_re[off];
                    xi[a * 2 + t] = in_im[off];
                }
            }
        }
        for (int ao = 0; ao < r_out; ++ao) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                T ar = 0, ai = 0;
                for (int a = 0; a < r_in; ++a) {
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int c = ((ao * r_in + a) * 2 + s) * 2 + t;
                        const T orr = op.re[c], oii = op.im[c];
                        ar += orr * xr[a * 2 + t] - oii * xi[a * 2 + t];
                        ai += orr * xi[a * 2 + t] + oii * xr[a * 2 + t];
                    }
                }
                const int64_t wo = (h * r_out + ao) * lo + l;
                const int64_t off = op.out_ws ? ((p * w_out + wo) * 2 + s) * Q + q : ((p * 2 + s) * w_out + wo) * Q + q;
                out_re[off] = ar;
                out_im[off] = ai;
            }
        }
    }
}

template <typename T>
hipError_t mpo_apply(const MpoSiteOp& op, int64_t P, int64_t Q, const T* in_re, const T* in_im,
                     T* out_re, T* out_im, hipStream_t stream) {
    if (op.r_in < 1 || op.r_out < 1 || op.r_in > 4 || op.r_out > 4 || op.r_in * op.r_out > 4)
        return hipErrorInvalidValue;
    MpoOpT<T> o;
    o.r_in = op.r_in; o.r_out = op.r_out; o.lo = op.lo; o.H = op.H; o.out_ws = op.out_ws;
    for (int i = 0; i < 16; ++i) { o.re[i] = (T)op.re[i]; o.im[i] = (T)op.im[i]; }
    const int64_t total = P * op.H * op.lo * Q;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(mpo_apply_kernel<T>, dim3(grid_for(total, 256)), dim3(256), 0, stream, o, P,
                       Q, in_re, in_im, out_re, out_im);
    return hipGetLastError();
}
template hipError_t mpo_apply<float>(const MpoSiteOp&, int64_t, int64_t, const float*, const float*,
                                     float*, float*, hipStream_t);
template hipError_t mpo_apply<double>(const MpoSiteOp&, int64_t, int64_t, const double*,
                                      const double*, double*, double*, hipStream_t);

// -------------------------------------------------------- site layouts -----
template <typename T>
__global__ __launch_bounds__(256) void site_to_view_kernel(const double* __restrict__ re,
                                                           const double* __restrict__ im, int Dl,
                                                           int Dr, int swap_legs,
                                                           T* __restrict__ ore,
                                                           T* __restrict__ oim) {
    const int64_t total = (int64_t)Dl * 2 * Dr;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t src;
        if (!swap_legs) {
            src = idx;
        } else {
            // output [b][s][a] (b < Dr, a < Dl) from input [a][s][b]
            const int64_t a = idx % Dl;
            const int64_t s = (idx / Dl) % 2;
            const int64_t b = idx / (2 * (int64_t)Dl);
            src = (a * 2 + s) * Dr + b;
        }
        ore[idx] = (T)re[src];
        oim[idx] = (T)im[src];
    }
}

template <typename T>
hipError_t site_to_view(const double* re, const double* im, int Dl, int Dr, int swap_legs, T* ore,
                        T* oim, hipStream_t stream) {
    const int64_t total = (int64_t)Dl * 2 * Dr;
    hipLaunchKernelGGL(site_to_view_kernel<T>, dim3(grid_for(total, 256)), dim3(256), 0, stream, re,
                       im, Dl, Dr, swap_legs, ore, oim);
    return hipGetLastError();
}
template hipError_t site_to_view<float>(const double*, const double*, int, int, int, float*, float*,
                                        hipStream_t);
template hipError_t site_to_view<double>(const double*, const double*, int, int, int, double*,
                                         double*, hipStream_t);

// ------------------------------------------------------- conversions ------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void convert_kernel(const TI* __restrict__ re,
                                                      const TI* __restrict__ im, int64_t n,
                                                      TO* __restrict__ ore, TO* __restrict__ oim) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        ore[i] = (TO)re[i];
        oim[i] = (TO)im[i];
    }
}

template <typename TI, typename TO>
hipError_t convert_planar(const TI* re, const TI* im, int64_t n, TO* ore, TO* oim,
                          hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((convert_kernel<TI, TO>), dim3(grid_for(n, 256)), dim3(256), 0, stream, re, im,
                       n, ore, oim);
    return hipGetLastError();
}
template hipError_t convert_planar<float, double>(const float*, const float*, int64_t, double*,
                                                  double*, hipStream_t);
template hipError_t convert_planar<double, float>(const double*, const double*, int64_t, float*,
                                                  float*, hipStream_t);
template hipError_t convert_planar<double, double>(const double*, const double*, int64_t, double*,
                                                   double*, hipStream_t);
template hipError_t convert_planar<float, float>(const float*, const float*, int64_t, float*,
                                                 float*, hipStream_t);

template <typename T>
__global__ void fill_kernel(T* re, T* im, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        re[i] = v;
        im[i] = 0;
    }
}

template <typename T>
hipError_t fill_planar(T* re, T* im, int64_t n, double value, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n, 256)), dim3(256), 0, stream, re, im, n,
                       (T)value);
    return hipGetLastError();
}
template hipError_t fill_planar<float>(float*, float*, int64_t, double, hipStream_t);
template hipError_t fill_planar<double>(double*, double*, int64_t, double, hipStream_t);

// -------------------------------------------------------- reductions ------
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block sum of a per-thread value; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    __syncthreads();
    return s;
}

template <typename T>
__global__ __launch_bounds__(256) void norm2_partial_kernel(const T* __restrict__ re,
                                                            const T* __restrict__ im, int64_t n,
                                                            double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = re[i], b = im[i];
        acc += a * a + b * b;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial, int np,
                                                           double* __restrict__ out) {
    __shared__ double sh[4];
    double acc = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = s;
}

template <typename T>
hipError_t norm2(const T* re, const T* im, int64_t n, double* partial, double* out,
                 hipStream_t stream) {
    int nb = (int)((n + 255) / 256);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(norm2_partial_kernel<T>, dim3(nb), dim3(256), 0, stream, re, im, n, partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, stream, partial, nb, out);
    return hipGetLastError();
}
template hipError_t norm2<float>(const float*, const float*, int64_t, double*, double*, hipStream_t);
template hipError_t norm2<double>(const double*, const double*, int64_t, double*, double*,
                                  hipStream_t);

// --------------------------------------------------- eigen plumbing --------
// Row-major planar Hermitian rho -> interleaved column-major.  Column-major
// element (i, j) sits at p = i + j n, where the row-major array holds
// rho[j][i] = conj(rho[i][j]).
__global__ __launch_bounds__(256) void pack_herm_kernel(const double* __restrict__ re,
                                                        const double* __restrict__ im, int64_t nn,
                                                        double* __restrict__ out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nn;
         p += (int64_t)gridDim.x * blockDim.x) {
        out[2 * p] = re[p];
        out[2 * p + 1] = -im[p];
    }
}

hipError_t pack_hermitian(const double* re, const double* im, int n, double* out_z,
                          hipStream_t stream) {
    const int64_t nn = (int64_t)n * n;
    hipLaunchKernelGGL(pack_herm_kernel, dim3(grid_for(nn, 256)), dim3(256), 0, stream, re, im, nn,
                       out_z);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void take_top_kernel(const double* __restrict__ ev, int n, int k,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ ore,
                                                       double* __restrict__ oim) {
    const int64_t total = (int64_t)n * k;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx % k;       // output column (largest first)
        const int64_t r = idx / k;       // row
        const int64_t src = r + (int64_t)(n - 1 - c) * n;
        const double s = scale ? scale[c] : 1.0;
        ore[idx] = ev[2 * src] * s;
        oim[idx] = ev[2 * src + 1] * s;
    }
}

hipError_t take_top_eigvecs(const double* evec_z, int n, int k, const double* scale_dev,
                            double* out_re, double* out_im, hipStream_t stream) {
    const int64_t total = (int64_t)n * k;
    hipLaunchKernelGGL(take_top_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, evec_z, n,
                       k, scale_dev, out_re, out_im);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void scaled_adjoint_kernel(const double* __restrict__ re,
                                                             const double* __restrict__ im, int m,
                                                             int k, const double* __restrict__ s,
                                                             double* __restrict__ ore,
                                                             double* __restrict__ oim) {
    const int64_t total = (int64_t)m * k;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = idx % m;     // output [row < k][col < m]
        const int64_t row = idx / m;
        const int64_t src = col * k + row;
        ore[idx] = s[row] * re[src];
        oim[idx] = -s[row] * im[src];
    }
}

hipError_t scaled_adjoint(const double* in_re, const double* in_im, int m, int k, const double* s_dev,
                          double* out_re, double* out_im, hipStream_t stream) {
    const int64_t total = (int64_t)m * k;
    hipLaunchKernelGGL(scaled_adjoint_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, in_re,
                       in_im, m, k, s_dev, out_re, out_im);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_cols_kernel(double* re, double* im, int64_t m, int k,
                                                         const double* __restrict__ s) {
    const int64_t total = m * k;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const double f = s[idx % k];
        re[idx] *= f;
        im[idx] *= f;
    }
}

hipError_t scale_columns(double* re, double* im, int64_t m, int k, const double* s_dev,
                         hipStream_t stream) {
    const int64_t total = m * k;
    hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, re, im, m,
                       k, s_dev);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void scale_scalar_kernel(T* re, T* im, int64_t n,
                                                           const double* __restrict__ s) {
    const T f = (T)(*s);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        re[i] *= f;
        im[i] *= f;
    }
}

template <typename T>
hipError_t scale_by_device_scalar(T* re, T* im, int64_t n, const double* s_dev, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_scalar_kernel<T>, dim3(grid_for(n, 256)), dim3(256), 0, stream, re, im, n,
                       s_dev);
    return hipGetLastError();
}
template hipError_t scale_by_device_scalar<float>(float*, float*, int64_t, const double*, hipStream_t);
template hipError_t scale_by_device_scalar<double>(double*, double*, int64_t, const double*,
                                                   hipStream_t);

// ------------------------------------------------------------ Philox ------
// Philox-4x32-10 from its published definition (Salmon et al., SC'11):
// S-box multipliers 0xD2511F53, 0xCD9E8D57; key increments 0x9E3779B9,
// 0xBB67AE85; ten rounds.
__device__ inline void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                    uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
}

__device__ inline double philox_uniform53(uint64_t seed, uint64_t sample, uint32_t site) {
    uint32_t c0 = site, c1 = (uint32_t)sample, c2 = (uint32_t)(sample >> 32), c3 = 0x5A4D5053u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        philox_round(c0, c1, c2, c3, k0, k1);
    }
    const uint64_t bits = (((uint64_t)c0 << 21) | (c1 >> 11)) & ((1ull << 53) - 1);
    return (double)bits * (1.0 / 9007199254740992.0);
}

// One block of 256 threads per row.
template <typename T>
__global__ __launch_bounds__(256) void select_rows_kernel(const T* __restrict__ ure,
                                                          const T* __restrict__ uim, int64_t S,
                                                          int D, int sampling,
                                                          const uint8_t* __restrict__ bits_in,
                                                          uint64_t seed, int64_t sample0, int site,
                                                          T* __restrict__ vre, T* __restrict__ vim,
                                                          uint8_t* __restrict__ bits_out) {
    __shared__ double sh[4];
    __shared__ double pr[2];
    for (int64_t r = blockIdx.x; r < S; r += gridDim.x) {
        const T* r0 = ure + r * 2 * D;
        const T* i0 = uim + r * 2 * D;
        int t;
        double scale = 1.0;
        if (sampling) {
            double a0 = 0, a1 = 0;
            for (int c = threadIdx.x; c < D; c += blockDim.x) {
                const double x0 = r0[c], y0 = i0[c], x1 = r0[D + c], y1 = i0[D + c];
                a0 += x0 * x0 + y0 * y0;
                a1 += x1 * x1 + y1 * y1;
            }
            const double s0 = block_sum(a0, sh);
            const double s1 = block_sum(a1, sh);
            if (threadIdx.x == 0) { pr[0] = s0; pr[1] = s1; }
            __syncthreads();
            const double p0 = pr[0], p1 = pr[1];
            const double u = philox_uniform53(seed, (uint64_t)(sample0 + r), (uint32_t)site);
            t = (u < p0 / (p0 + p1)) ? 0 : 1;
            scale = 1.0 / sqrt(t == 0 ? p0 : p1);
            __syncthreads();
        } else {
            t = bits_in[r];
        }
        for (int c = threadIdx.x; c < D; c += blockDim.x) {
            vre[r * D + c] = (T)(r0[t * D + c] * scale);
            vim[r * D + c] = (T)(i0[t * D + c] * scale);
        }
        if (threadIdx.x == 0 && bits_out) bits_out[r] = (uint8_t)t;
    }
}

template <typename T>
hipError_t select_rows(const T* u_re, const T* u_im, int64_t S, int D, int sampling,
                       const uint8_t* bits_in, uint64_t seed, int64_t sample0, int site, T* v_re,
                       T* v_im, uint8_t* bits_out, hipStream_t stream) {
    if (S <= 0) return hipSuccess;
    const unsigned nb = (unsigned)(S < 65536 ? S : 65536);
    hipLaunchKernelGGL(select_rows_kernel<T>, dim3(nb), dim3(256), 0, stream, u_re, u_im, S, D,
                       sampling, bits_in, seed, sample0, site, v_re, v_im, bits_out);
    return hipGetLastError();
}
template hipError_t select_rows<float>(const float*, const float*, int64_t, int, int, const uint8_t*,
                                       uint64_t, int64_t, int, float*, float*, uint8_t*, hipStream_t);
template hipError_t select_rows<double>(const double*, const double*, int64_t, int, int,
                                        const uint8_t*, uint64_t, int64_t, int, double*, double*,
                                        uint8_t*, hipStream_t);

// ------------------------------------------------------------- Z leg ------
__global__ __launch_bounds__(256) void apply_z_kernel(const double* __restrict__ re,
                                                      const double* __restrict__ im, int Dl, int Dr,
                                                      double* __restrict__ ore,
                                                      double* __restrict__ oim) {
    const int64_t total = (int64_t)Dl * 2 * Dr;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)((idx / Dr) % 2);
        const double f = s ? -1.0 : 1.0;
        ore[idx] = f * re[idx];
        oim[idx] = f * im[idx];
    }
}

hipError_t apply_z_phys(const double* re, const double* im, int Dl, int Dr, double* out_re,
                        double* out_im, hipStream_t stream) {
    const int64_t total = (int64_t)Dl * 2 * Dr;
    hipLaunchKernelGGL(apply_z_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, re, im, Dl,
                       Dr, out_re, out_im);
    return hipGetLastError();
}

}  // namespace mpsk

namespace mpsk {

// ------------------------------------------------- k-major site copies ----
// View tensor V[a][s][x] (dims Dl_v, 2, Dr_v) written as O[(s Dr_v + x) Dl_v + a],
// i.e. the (2 Dr_v) x Dl_v matrix whose rows are contiguous in a.  The stored
// tensor is [Dl_v][2][Dr_v] when swap_legs == 0 and [Dr_v][2][Dl_v] otherwise.
__global__ __launch_bounds__(256) void site_to_kmajor_kernel(const double* __restrict__ re,
                                                             const double* __restrict__ im, int Dlv,
                                                             int Drv, int swap_legs,
                                                             float* __restrict__ ore,
                                                             float* __restrict__ oim) {
    const int64_t total = (int64_t)Dlv * 2 * Drv;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = idx % Dlv;
        const int64_t sx = idx / Dlv;           // s * Drv + x
        const int64_t s = sx / Drv, x = sx % Drv;
        const int64_t src = swap_legs ? ((x * 2 + s) * Dlv + a) : ((a * 2 + s) * Drv + x);
        ore[idx] = (float)re[src];
        oim[idx] = (float)im[src];
    }
}

hipError_t site_to_kmajor(const double* re, const double* im, int Dlv, int Drv, int swap_legs, float* ore,
                          float* oim, hipStream_t stream) {
    const int64_t total = (int64_t)Dlv * 2 * Drv;
    hipLaunchKernelGGL(site_to_kmajor_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, re, im, Dlv, Drv,
                       swap_legs, ore, oim);
    return hipGetLastError();
}

// out (k x m, FP32) = in^H for a row-major m x k FP64 planar matrix
__global__ __launch_bounds__(256) void adjoint_to_f32_kernel(const double* __restrict__ re,
                                                             const double* __restrict__ im, int64_t m,
                                                             int64_t k, float* __restrict__ ore,
                                                             float* __restrict__ oim) {
    const int64_t total = m * k;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = idx % m, row = idx / m;      // output [row < k][col < m]
        const int64_t src = col * k + row;
        ore[idx] = (float)re[src];
        oim[idx] = (float)(-im[src]);
    }
}

hipError_t adjoint_to_f32(const double* re, const double* im, int64_t m, int64_t k, float* ore, float* oim,
                          hipStream_t stream) {
    const int64_t total = m * k;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_to_f32_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, re, im, m, k, ore,
                       oim);
    return hipGetLastError();
}

// Planar row-major (rows x cols) <-> interleaved column-major (LAPACK layout),
// through 64 x 64 LDS tiles so that both sides are read and written in order.
__global__ __launch_bounds__(256) void rm_planar_to_cm_kernel(const double* __restrict__ re,
                                                             const double* __restrict__ im, int64_t rows,
                                                             int64_t cols, double2* __restrict__ out) {
    __shared__ double2 t[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int a = ty; a < 64; a += 4) {
        const int64_t r = r0 + a, c = c0 + tx;
        if (r < rows && c < cols) t[a][tx] = make_double2(re[r * cols + c], im[r * cols + c]);
    }
    __syncthreads();
    for (int a = ty; a < 64; a += 4) {
        const int64_t c = c0 + a, r = r0 + tx;
        if (r < rows && c < cols) out[r + c * rows] = t[tx][a];
    }
}

__global__ __launch_bounds__(256) void cm_to_rm_planar_kernel(const double2* __restrict__ in, int64_t rows,
                                                             int64_t cols, double* __restrict__ re,
                                                             double* __restrict__ im) {
    __shared__ double2 t[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int a = ty; a < 64; a += 4) {
        const int64_t c = c0 + a, r = r0 + tx;
        if (r < rows && c < cols) t[tx][a] = in[r + c * rows];
    }
    __syncthreads();
    for (int a = ty; a < 64; a += 4) {
        const int64_t r = r0 + a, c = c0 + tx;
        if (r < rows && c < cols) {
            re[r * cols + c] = t[a][tx].x;
            im[r * cols + c] = t[a][tx].y;
        }
    }
}

hipError_t rm_planar_to_cm(const double* re, const double* im, int64_t rows, int64_t cols, double* out_z,
                           hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL(rm_planar_to_cm_kernel, grid, dim3(256), 0, stream, re, im, rows, cols, (double2*)out_z);
    return hipGetLastError();
}

hipError_t cm_to_rm_planar(const double* in_z, int64_t rows, int64_t cols, double* re, double* im,
                           hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL(cm_to_rm_planar_kernel, grid, dim3(256), 0, stream, (const double2*)in_z, rows, cols, re, im);
    return hipGetLastError();
}

}  // namespace mpsk
