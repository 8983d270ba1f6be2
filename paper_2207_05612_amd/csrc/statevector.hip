// Exact statevector kernels (gfx950): the brute-force state U|0> that the
// paper uses to measure the true fidelity F (eq:F-sup) and the linear
// cross-entropy F_B (eq:FB-sup) of its MPS, kept in HBM for up to ~32 qubits.
//
// Amplitudes are FP64 planar (re block, then im block); chain site q is bit
// n-1-q of the index (site 0 most significant).  A gate touches every
// amplitude once: each thread owns the amplitudes a two-qubit (or one-qubit)
// gate mixes, so a pass streams 2 x 16 bytes per amplitude and the kernels are
// bound by HBM bandwidth.  Consecutive threads own consecutive index groups; the
// two-qubit passes pair neighbouring amplitudes into 16-byte accesses.  Reductions use a fixed grid and fixed-order partial sums, so
// their results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace mpsk {

static inline unsigned sv_grid(uint64_t n, int block) {
    uint64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;   // grid-stride loops cover the rest
    if (g < 1) g = 1;
    return (unsigned)g;
}

// x with a zero bit inserted at position p
__device__ inline uint64_t insert_zero(uint64_t x, int p) {
    const uint64_t low = x & ((1ull << p) - 1);
    return ((x >> p) << (p + 1)) | low;
}

__global__ __launch_bounds__(256) void sv_fill_kernel(double* __restrict__ re, double* __restrict__ im, uint64_t dim,
                                                      uint64_t one_at) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * blockDim.x) {
        re[i] = i == one_at ? 1.0 : 0.0;
        im[i] = 0.0;
    }
}

// y = U x for the 4 amplitudes of one group (row and column index 2 s_a + s_b).
__device__ inline void sv_mix4(const SvGate2& g, const double* xr, const double* xi, double* yr, double* yi) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double ar = 0, ai = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ar += g.re[r * 4 + c] * xr[c] - g.im[r * 4 + c] * xi[c];
            ai += g.re[r * 4 + c] * xi[c] + g.im[r * 4 + c] * xr[c];
        }
        yr[r] = ar;
        yi[r] = ai;
    }
}

// U (4 x 4) on the qubits at bit positions pa and pb, both >= 1.  A thread owns
// the groups 2u and 2u + 1: bit 0 is untouched by the gate, so their amplitudes
// are neighbours and every access is one 16-byte load or store.
__global__ __launch_bounds__(256) void sv_2q_kernel(double* __restrict__ re, double* __restrict__ im, uint64_t units,
                                                    int pa, int pb, SvGate2 g) {
    const int lo = min(pa, pb), hi = max(pa, pb);
    const uint64_t off[4] = {0, 1ull << pb, 1ull << pa, (1ull << pa) | (1ull << pb)};
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < units;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = insert_zero(insert_zero(2 * u, lo), hi);
        double2 vr[4], vi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            vr[r] = *(const double2*)(re + base + off[r]);
            vi[r] = *(const double2*)(im + base + off[r]);
        }
        double xr[4], xi[4], yr0[4], yi0[4], yr1[4], yi1[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            xr[r] = vr[r].x;
            xi[r] = vi[r].x;
        }
        sv_mix4(g, xr, xi, yr0, yi0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            xr[r] = vr[r].y;
            xi[r] = vi[r].y;
        }
        sv_mix4(g, xr, xi, yr1, yi1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            *(double2*)(re + base + off[r]) = make_double2(yr0[r], yr1[r]);
            *(double2*)(im + base + off[r]) = make_double2(yi0[r], yi1[r]);
        }
    }
}

// U (4 x 4) on bit 0 and the bit at position hi: the two amplitudes of a group
// that differ in bit 0 are neighbours, one 16-byte access each.  a_low says
// whether bit 0 is the gate's first qubit (s_a) or its second (s_b).
__global__ __launch_bounds__(256) void sv_2q_bit0_kernel(double* __restrict__ re, double* __restrict__ im,
                                                         uint64_t groups, int hi, int a_low, SvGate2 g) {
    const uint64_t other = 1ull << hi;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < groups;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = insert_zero(2 * t, hi);
        const double2 pr = *(const double2*)(re + base), pi = *(const double2*)(im + base);
        const double2 qr = *(const double2*)(re + base + other), qi = *(const double2*)(im + base + other);
        // bit 0 is s_a: (base, base + 1) holds s_a = 0, 1 at s_b = 0; otherwise it holds s_b = 0, 1 at s_a = 0
        const double xr[4] = {pr.x, a_low ? qr.x : pr.y, a_low ? pr.y : qr.x, qr.y};
        const double xi[4] = {pi.x, a_low ? qi.x : pi.y, a_low ? pi.y : qi.x, qi.y};
        double yr[4], yi[4];
        sv_mix4(g, xr, xi, yr, yi);
        *(double2*)(re + base) = make_double2(yr[0], a_low ? yr[2] : yr[1]);
        *(double2*)(im + base) = make_double2(yi[0], a_low ? yi[2] : yi[1]);
        *(double2*)(re + base + other) = make_double2(a_low ? yr[1] : yr[2], yr[3]);
        *(double2*)(im + base + other) = make_double2(a_low ? yi[1] : yi[2], yi[3]);
    }
}

// U (2 x 2) on the qubit at bit position p.
__global__ __launch_bounds__(256) void sv_1q_kernel(double* __restrict__ re, double* __restrict__ im, uint64_t pairs,
                                                    int p, SvGate1 g) {
    const uint64_t ip = 1ull << p;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < pairs;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i0 = insert_zero(t, p), i1 = i0 | ip;
        const double ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
        re[i0] = g.re[0] * ar - g.im[0] * ai + g.re[1] * br - g.im[1] * bi;
        im[i0] = g.re[0] * ai + g.im[0] * ar + g.re[1] * bi + g.im[1] * br;
        re[i1] = g.re[2] * ar - g.im[2] * ai + g.re[3] * br - g.im[3] * bi;
        im[i1] = g.re[2] * ai + g.im[2] * ar + g.re[3] * bi + g.im[3] * br;
    }
}

__global__ __launch_bounds__(256) void sv_gather_kernel(const double* __restrict__ re, const double* __restrict__ im,
                                                        const int64_t* __restrict__ idx, int64_t count,
                                                        double* __restrict__ out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        out[2 * t] = re[idx[t]];
        out[2 * t + 1] = im[idx[t]];
    }
}

// Per block: sum conj(phi) psi (re, im), sum |phi|^2 |psi|^2, sum |phi|^2, sum |psi|^2.
constexpr int SV_RED_BLOCK = 256;
__global__ __launch_bounds__(SV_RED_BLOCK) void sv_compare_kernel(const double* __restrict__ pr,
                                                                  const double* __restrict__ pi,
                                                                  const double* __restrict__ qr,
                                                                  const double* __restrict__ qi, uint64_t dim,
                                                                  double* __restrict__ partials) {
    double s[5] = {0, 0, 0, 0, 0};
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * blockDim.x) {
        const double a = pr[i], b = pi[i], c = qr[i], d = qi[i];
        s[0] += a * c + b * d;          // conj(phi) psi
        s[1] += a * d - b * c;
        const double p2 = a * a + b * b, q2 = c * c + d * d;
        s[2] += p2 * q2;
        s[3] += p2;
        s[4] += q2;
    }
    __shared__ double red[5][SV_RED_BLOCK];
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = SV_RED_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k) partials[(size_t)blockIdx.x * 5 + k] = red[k][0];
}

hipError_t sv_fill(double* re, double* im, uint64_t dim, uint64_t one_at, hipStream_t s) {
    hipLaunchKernelGGL(sv_fill_kernel, dim3(sv_grid(dim, 256)), dim3(256), 0, s, re, im, dim, one_at);
    return hipGetLastError();
}

hipError_t sv_apply_2q(double* re, double* im, int n, int pa, int pb, const SvGate2& g, hipStream_t s) {
    if (n < 2 || pa == pb || pa < 0 || pb < 0 || pa >= n || pb >= n) return hipErrorInvalidValue;
    // the 16-byte accesses need re and im at even offsets from a 16-byte boundary
    if ((reinterpret_cast<uintptr_t>(re) | reinterpret_cast<uintptr_t>(im)) & 15) return hipErrorInvalidValue;
    const uint64_t groups = 1ull << (n - 2);
    if (pa == 0 || pb == 0) {
        const int hi = max(pa, pb);
        hipLaunchKernelGGL(sv_2q_bit0_kernel, dim3(sv_grid(groups, 256)), dim3(256), 0, s, re, im, groups, hi,
                           pa == 0 ? 1 : 0, g);
    } else {
        const uint64_t units = groups / 2;   // n >= 3 here, so groups is even
        hipLaunchKernelGGL(sv_2q_kernel, dim3(sv_grid(units, 256)), dim3(256), 0, s, re, im, units, pa, pb, g);
    }
    return hipGetLastError();
}

hipError_t sv_apply_1q(double* re, double* im, int n, int p, const SvGate1& g, hipStream_t s) {
    if (n < 1 || p < 0 || p >= n) return hipErrorInvalidValue;
    const uint64_t pairs = 1ull << (n - 1);
    hipLaunchKernelGGL(sv_1q_kernel, dim3(sv_grid(pairs, 256)), dim3(256), 0, s, re, im, pairs, p, g);
    return hipGetLastError();
}

hipError_t sv_gather(const double* re, const double* im, const int64_t* idx, int64_t count, double* out,
                     hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(sv_gather_kernel, dim3(sv_grid((uint64_t)count, 256)), dim3(256), 0, s, re, im, idx, count, out);
    return hipGetLastError();
}

int sv_compare_blocks() { return 4096; }

hipError_t sv_compare(const double* pr, const double* pi, const double* qr, const double* qi, uint64_t dim,
                      double* partials, hipStream_t s) {
    hipLaunchKernelGGL(sv_compare_kernel, dim3(sv_compare_blocks()), dim3(SV_RED_BLOCK), 0, s, pr, pi, qr, qi, dim,
                       partials);
    return hipGetLastError();
}

}  // namespace mpsk
