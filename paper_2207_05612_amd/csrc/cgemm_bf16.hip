// Split-precision complex GEMM on CDNA4 BF16 matrix cores (gfx950).
//
// C (M x N, FP32) = A (M x K) B^T (B stored N x K), planar complex, both
// operands FP32 with k contiguous.  Every FP32 operand x is split into S BF16
// terms x = x_0 + ... + x_{S-1} (each the BF16 rounding of what remains), and a
// real product keeps the terms x_a y_b with a + b < S, accumulated in FP32 by
// v_mfma_f32_32x32x16_bf16:
//   S = 3 (cgemm_bf16x3_nt_kernel): six products hh, hm, mh, mm, hl, lh; the
//         dropped terms are below 2^-24 of the product (about FP32 accuracy);
//   S = 2 (cgemm_bf16x2_nt_kernel): three products hh, hl, lh; the dropped
//         term x_l y_l and the residual of the two-term split are about 2^-16
//         of the product.
// A complex product is four such real products.
//
// Tiling: 512 threads = 8 wavefronts (4 x 2), wave tile 64 x 64 complex
// (2 x 2 MFMA tiles of 32 x 32), block tile 256 x 128, BK = 16 (one MFMA k
// step), two wavefronts per SIMD so that one wave's MFMAs cover the other's
// waits.  LDS holds [split][re|im][k/8][row][8] so that the 8 consecutive k
// of one MFMA lane are one 16-byte read and the 32 lanes of a row group read
// consecutive 16-byte words.  Two LDS buffers (144 KiB for S = 3) overlap the
// next tile's loads with the current tile's 96 (S = 3) or 48 (S = 2) MFMAs
// per wave.  Block ids map to tiles XCD-first, then in groups of 8 tile rows.
//
// Two ways to fill LDS, with the same terms, tiles and MFMA order (and so the
// same bits):
//   * staging (cgemm_bf16x{3,2}_nt_kernel): each k tile is loaded as float4
//     and split in registers on the way into LDS; fragments are read per split
//     pair to keep each wave under 256 registers.  The allocation-free entry
//     point uses it (it needs no memory beyond the operands).
//   * planes (split_planes*_kernel, then cgemm_bf16x{3,2}_planes_kernel): each
//     operand is split once into BF16 planes laid out like the LDS tiles, and
//     the product kernel moves them into LDS with direct global-to-LDS loads.
//     The compression step uses it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "internal.h"

namespace mpsk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct SplitArgs {
    const float* a_re;
    const float* a_im;
    const float* b_re;
    const float* b_im;
    float* c_re;
    float* c_im;
    int64_t lda, ldb, ldc;
    int M, N, K;
    int gm, gn;
    int kchunk;             // k range of split blockIdx.y
    int64_t split_stride;   // C offset of split y
};

__device__ inline float bf16_to_float(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// FP32 -> BF16 bits by the hardware conversion (v_cvt_pk_bf16_f32): round to nearest even
__device__ inline unsigned short bf16_rne(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }

__device__ inline void split3(float x, unsigned short& h, unsigned short& m, unsigned short& l) {
    h = bf16_rne(x);
    const float r1 = x - bf16_to_float(h);
    m = bf16_rne(r1);
    const float r2 = r1 - bf16_to_float(m);
    l = bf16_rne(r2);
}

constexpr int SBM = 256, SBN = 128, SBK = 16;
constexpr int NT = 512;   // threads per block: 8 wavefronts, 4 (m) x 2 (n)
// LDS element offset of (split s, part p, chunk c, row r) in a [3][2][2][rows][8] tile
template <int ROWS>
__device__ inline int lds_off(int s, int p, int c, int r) { return ((((s * 2 + p) * 2 + c) * ROWS) + r) * 8; }

template <int S, bool VEC>
__device__ __forceinline__ void cgemm_split_body(const SplitArgs& g) {
    __shared__ __attribute__((aligned(16))) unsigned short As[2][S * 2 * 2 * SBM * 8];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][S * 2 * 2 * SBN * 8];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave >> 1) * 64;
    const int wn0 = (wave & 1) * 64;

    int pid = blockIdx.x;
    const int nb = g.gm * g.gn;
    if ((nb & 7) == 0) pid = (pid & 7) * (nb >> 3) + (pid >> 3);
    constexpr int GROUP = 8;
    const int group = pid / (GROUP * g.gn);
    const int first_m = group * GROUP;
    const int gsz = min(g.gm - first_m, GROUP);
    const int tm = first_m + (pid % gsz);
    const int tn = (pid % (GROUP * g.gn)) / gsz;
    const int m0 = tm * SBM, n0 = tn * SBN;
    const int M = g.M, N = g.N;
    const int kbeg = blockIdx.y * g.kchunk;
    const int K = min(g.K, kbeg + g.kchunk);
    float* const c_re = g.c_re + blockIdx.y * g.split_stride;
    float* const c_im = g.c_im + blockIdx.y * g.split_stride;

    // staging: a tile plane is rows x 16 k in groups of 4 consecutive k (4 groups per row);
    // A has 1024 groups per plane (threads take groups tid, tid + 512), B has 512 (group tid)
    float4 ar[2], ai[2], br, bi;
    // rows past M (N) are read from the last valid row and zeroed when staged, so the loads of
    // full k tiles carry no per-lane condition and stay in flight across the MFMAs
    bool a_ok[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) a_ok[u] = m0 + ((tid + NT * u) >> 2) < M;
    const bool b_ok = n0 + (tid >> 2) < N;

    auto ld4_full = [&](const float* base, int64_t ld, int row, int k) -> float4 {
        const float* p = base + (int64_t)row * ld + k;
        if (VEC) return *(const float4*)p;
        return make_float4(p[0], p[1], p[2], p[3]);
    };
    auto ld4_tail = [&](const float* base, int64_t ld, int row, int rows_valid, int k) -> float4 {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            t[e] = (row < rows_valid && k + e < K) ? base[(int64_t)row * ld + k + e] : 0.f;
        return make_float4(t[0], t[1], t[2], t[3]);
    };
    // a k tile with every k < K
    auto load_full = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int grp = tid + NT * u;
            const int row = min(m0 + (grp >> 2), M - 1), k = k0 + (grp & 3) * 4;
            ar[u] = ld4_full(g.a_re, g.lda, row, k);
            ai[u] = ld4_full(g.a_im, g.lda, row, k);
        }
        const int row = min(n0 + (tid >> 2), N - 1), k = k0 + (tid & 3) * 4;
        br = ld4_full(g.b_re, g.ldb, row, k);
        bi = ld4_full(g.b_im, g.ldb, row, k);
    };
    // the last, partial k tile
    auto load_tail = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int grp = tid + NT * u;
            const int row = grp >> 2, k = k0 + (grp & 3) * 4;
            ar[u] = ld4_tail(g.a_re, g.lda, m0 + row, M, k);
            ai[u] = ld4_tail(g.a_im, g.lda, m0 + row, M, k);
        }
        const int row = tid >> 2, k = k0 + (tid & 3) * 4;
        br = ld4_tail(g.b_re, g.ldb, n0 + row, N, k);
        bi = ld4_tail(g.b_im, g.ldb, n0 + row, N, k);
    };
    typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
    auto put = [&](unsigned short* base, int rows, int p, int row, int kq, float4 v, bool ok) {
        const float x[4] = {ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f};
        u16x4 h, m, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (S == 3) {
                unsigned short a, b, c;
                split3(x[e], a, b, c);
                h[e] = a; m[e] = b; l[e] = c;
            } else {
                h[e] = bf16_rne(x[e]);
                m[e] = bf16_rne(x[e] - bf16_to_float(h[e]));
            }
        }
        const int chunk = kq >> 3, sub = kq & 7;
        const int plane = 2 * rows * 8;   // elements per (split, part) for both chunks
        const int off = ((p * 2 + chunk) * rows + row) * 8 + sub;
        *(u16x4*)&base[off] = h;
        *(u16x4*)&base[off + 2 * plane] = m;
        if (S == 3) *(u16x4*)&base[off + 4 * plane] = l;
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int grp = tid + NT * u;
            const int row = grp >> 2, kq = (grp & 3) * 4;
            put(As[buf], SBM, 0, row, kq, ar[u], a_ok[u]);
            put(As[buf], SBM, 1, row, kq, ai[u], a_ok[u]);
        }
        const int row = tid >> 2, kq = (tid & 3) * 4;
        put(Bs[buf], SBN, 0, row, kq, br, b_ok);
        put(Bs[buf], SBN, 1, row, kq, bi, b_ok);
    };

    f32x16 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc_re[i][j][v] = 0.f; acc_im[i][j][v] = 0.f; }

    const int lrow = lane & 31;
    const int lchunk = lane >> 5;
    auto compute = [&](int buf) {
        // kept split pairs (sa, sb) with sa + sb < S, grouped by the A split
#pragma unroll
        for (int sa = 0; sa < S; ++sa) {
            bf16x8 fa[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int p = 0; p < 2; ++p)
                    fa[i][p] = *(const bf16x8*)&As[buf][lds_off<SBM>(sa, p, lchunk, wm0 + i * 32 + lrow)];
            for (int sb = 0; sb < S - sa; ++sb) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 fbr = *(const bf16x8*)&Bs[buf][lds_off<SBN>(sb, 0, lchunk, wn0 + j * 32 + lrow)];
                    const bf16x8 fbi = *(const bf16x8*)&Bs[buf][lds_off<SBN>(sb, 1, lchunk, wn0 + j * 32 + lrow)];
                    // -b_im: flip the sign bit of each BF16 (two per 32-bit word)
                    const u32x4 t = __builtin_bit_cast(u32x4, fbi) ^ 0x80008000u;
                    const bf16x8 fbn = __builtin_bit_cast(bf16x8, t);
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fbr, acc_re[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fbi, acc_im[i][j], 0, 0, 0);
                        acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][1], fbn, acc_re[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][1], fbr, acc_im[i][j], 0, 0, 0);
                    }
                }
            }
        }
    };

    // full k tiles first, then at most one partial tile
    const int nk_full = (K - kbeg) / SBK;
    const bool tail = (K - kbeg) % SBK != 0;
    if (nk_full > 0) load_full(kbeg);
    else load_tail(kbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int kt = 0; kt + 1 < nk_full; ++kt) {
        load_full(kbeg + (kt + 1) * SBK);
        __builtin_amdgcn_sched_barrier(0);   // issue the next tile's loads before this tile's MFMAs
        compute(buf);
        __builtin_amdgcn_sched_barrier(0);   // and consume them only after the MFMAs
        store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    if (nk_full > 0 && tail) {
        load_tail(kbeg + nk_full * SBK);
        compute(buf);
        store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    compute(buf);

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = m0 + wm0 + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
                const int c = n0 + wn0 + j * 32 + lrow;
                if (r < M && c < N) {
                    const int64_t off = (int64_t)r * g.ldc + c;
                    c_re[off] = acc_re[i][j][v];
                    c_im[off] = acc_im[i][j][v];
                }
            }
}

template <bool VEC>
__global__ __launch_bounds__(NT, 1) void cgemm_bf16x3_nt_kernel(SplitArgs g) {
    cgemm_split_body<3, VEC>(g);
}
template <bool VEC>
__global__ __launch_bounds__(NT, 1) void cgemm_bf16x2_nt_kernel(SplitArgs g) {
    cgemm_split_body<2, VEC>(g);
}

static hipError_t launch_split(int terms, int M, int N, int K, CView<float> A, CView<float> B, CViewMut<float> C,
                               int ksplit, int64_t split_stride, hipStream_t stream) {
    if (M <= 0 || N <= 0) return hipSuccess;
    SplitArgs g;
    g.a_re = A.re; g.a_im = A.im; g.lda = A.ld;
    g.b_re = B.re; g.b_im = B.im; g.ldb = B.ld;
    g.c_re = C.re; g.c_im = C.im; g.ldc = C.ld;
    g.M = M; g.N = N; g.K = K;
    g.gm = (M + SBM - 1) / SBM;
    g.gn = (N + SBN - 1) / SBN;
    if (ksplit < 1) ksplit = 1;
    g.kchunk = (((K + ksplit - 1) / ksplit) + SBK - 1) / SBK * SBK;
    if (g.kchunk < SBK) g.kchunk = SBK;
    ksplit = (K + g.kchunk - 1) / g.kchunk;
    if (ksplit < 1) ksplit = 1;
    g.split_stride = ksplit > 1 ? split_stride : 0;
    const int64_t nblocks = (int64_t)g.gm * g.gn;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    // float4 staging needs 16-byte aligned rows (leading dimensions and plane bases)
    const bool vec = (A.ld % 4 == 0) && (B.ld % 4 == 0) &&
                     ((((uintptr_t)A.re) | ((uintptr_t)A.im) | ((uintptr_t)B.re) | ((uintptr_t)B.im)) & 15) == 0;
    const dim3 grid((unsigned)nblocks, (unsigned)ksplit);
    if (terms == 3) {
        if (vec)
            hipLaunchKernelGGL(cgemm_bf16x3_nt_kernel<true>, grid, dim3(NT), 0, stream, g);
        else
            hipLaunchKernelGGL(cgemm_bf16x3_nt_kernel<false>, grid, dim3(NT), 0, stream, g);
    } else if (terms == 2) {
        if (vec)
            hipLaunchKernelGGL(cgemm_bf16x2_nt_kernel<true>, grid, dim3(NT), 0, stream, g);
        else
            hipLaunchKernelGGL(cgemm_bf16x2_nt_kernel<false>, grid, dim3(NT), 0, stream, g);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operands split once per product.  The kernels above split every k tile as it
// is staged, so a row of A is split again for every tile column of C and a row
// of B for every tile row.  Here split_planes_kernel writes the S BF16 terms of
// an operand once, as planes, and the product kernel streams the planes from
// memory straight into LDS (global_load_lds_dwordx4: no registers, no VALU).
// The terms, the LDS layout, the MFMA sequence and the k tiles (k padded to a
// multiple of 16 with zeros) are those of the kernels above, so both give
// bit-identical products.
//
// Plane layout: plane (s, p) (term s, part p = re / im) of an operand of
// `rows` rows holds R x Kp BF16 values, R = rows rounded up to the tile (256
// for A, 128 for B), Kp = K rounded up to 16, entries beyond K and rows past
// `rows` zero; it starts at ((s * 2 + p) R Kp) and stores (row, k) at
// ((k / 8) R + row) 8 + k mod 8: the 8 k of one MFMA lane are 16 bytes, and
// consecutive rows follow each other.  That is the LDS layout of a tile, so
// one wavefront load moves 64 rows x 16 bytes, 1 KiB of contiguous memory.

typedef float f32x4v __attribute__((ext_vector_type(4)));

// One block step covers 64 rows x 4 groups of 8 k: each wavefront writes one
// group of 64 rows (1 KiB contiguous), and the four wavefronts together read
// whole 128-byte lines of the source rows.
template <int S, bool VEC>
__global__ __launch_bounds__(256) void split_planes_kernel(const float* __restrict__ re, const float* __restrict__ im,
                                                           int64_t ld, int rows, int rows_pad, int K, int Kp,
                                                           unsigned short* __restrict__ planes) {
    const int gpr = Kp >> 3;                       // groups of 8 k per row
    const int nkb = (gpr + 3) >> 2;                // blocks of 4 groups
    const int64_t units = (int64_t)(rows_pad >> 6) * nkb;
    const int64_t plane = (int64_t)rows_pad * Kp;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t row = (u / nkb) * 64 + (threadIdx.x & 63);
        const int kg = (int)(u % nkb) * 4 + (threadIdx.x >> 6);
        if (kg >= gpr) continue;
        const int k0 = kg * 8;
        const bool live = row < rows;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float* src = (p ? im : re) + (live ? row : 0) * ld + k0;
            float x[8];
            if (!live) {
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = 0.f;
            } else if (VEC && k0 + 8 <= K) {
                const f32x4v lo = *(const f32x4v*)src, hi = *(const f32x4v*)(src + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) { x[e] = lo[e]; x[e + 4] = hi[e]; }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = k0 + e < K ? src[e] : 0.f;
            }
            u16x8 h, m, l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (S == 3) {
                    unsigned short a, b, c;
                    split3(x[e], a, b, c);
                    h[e] = a; m[e] = b; l[e] = c;
                } else {
                    h[e] = bf16_rne(x[e]);
                    m[e] = bf16_rne(x[e] - bf16_to_float(h[e]));
                }
            }
            unsigned short* dst = planes + (int64_t)p * plane + ((int64_t)kg * rows_pad + row) * 8;
            *(u16x8*)dst = h;
            *(u16x8*)(dst + 2 * plane) = m;
            if (S == 3) *(u16x8*)(dst + 4 * plane) = l;
        }
    }
}

// The same planes for the transposed operand X = src^T, src K x rows row-major
// (leading dimension ld): plane entry (r, k) is src[k][r].  Lane r of a
// wavefront reads 8 rows of src at column r (coalesced across lanes) and
// writes the 16 bytes of (r, 8 k), consecutive lanes consecutive.
template <int S>
__global__ __launch_bounds__(256) void split_planes_t_kernel(const float* __restrict__ re, const float* __restrict__ im,
                                                             int64_t ld, int rows, int rows_pad, int K, int Kp,
                                                             unsigned short* __restrict__ planes) {
    const int gpr = Kp >> 3;
    const int nkb = (gpr + 3) >> 2;
    const int64_t units = (int64_t)(rows_pad >> 6) * nkb;
    const int64_t plane = (int64_t)rows_pad * Kp;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t row = (u / nkb) * 64 + (threadIdx.x & 63);
        const int kg = (int)(u % nkb) * 4 + (threadIdx.x >> 6);
        if (kg >= gpr) continue;
        const int k0 = kg * 8;
        const bool live = row < rows;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float* src = (p ? im : re) + (live ? row : 0);
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = (live && k0 + e < K) ? src[(int64_t)(k0 + e) * ld] : 0.f;
            u16x8 h, m, l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (S == 3) {
                    unsigned short a, b, c;
                    split3(x[e], a, b, c);
                    h[e] = a; m[e] = b; l[e] = c;
                } else {
                    h[e] = bf16_rne(x[e]);
                    m[e] = bf16_rne(x[e] - bf16_to_float(h[e]));
                }
            }
            unsigned short* dst = planes + (int64_t)p * plane + ((int64_t)kg * rows_pad + row) * 8;
            *(u16x8*)dst = h;
            *(u16x8*)(dst + 2 * plane) = m;
            if (S == 3) *(u16x8*)(dst + 4 * plane) = l;
        }
    }
}

struct PlaneArgs {
    const unsigned short* a;   // planes of A (M rows)
    const unsigned short* b;   // planes of B (N rows)
    float* c_re;
    float* c_im;
    int64_t ldc;
    int M, N, Kp;
    int gm, gn;
    int kchunk;                // k range of split blockIdx.y (a multiple of 16)
    int64_t split_stride;      // C offset of split y
};

// 16 bytes per lane from global memory into LDS: lane l of the wavefront reads
// base + lane_bytes (base the same in every lane, lane_bytes zero-extended, so
// that the load takes the scalar-base form) and writes lds_wave_base + 16 l.
// The base goes through readfirstlane: it is uniform anyway, and the compiler
// then keeps it in scalar registers instead of forming one 64-bit vector
// address per load outside the k loop.
typedef const __attribute__((address_space(1))) char* gchar_ptr;
__device__ __forceinline__ void dma16(const unsigned short* base, unsigned lane_bytes, unsigned short* lds_wave_base) {
    const uint64_t v = (uint64_t)base;
    const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)((gchar_ptr)u + lane_bytes),
                                     (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}

template <int S>
__device__ __forceinline__ void cgemm_planes_body(const PlaneArgs& g) {
    // two buffers as separate objects, so that the compiler can tell the LDS
    // reads of one buffer from the loads in flight into the other
    __shared__ __attribute__((aligned(16))) unsigned short As0[S * 2 * 2 * SBM * 8];
    __shared__ __attribute__((aligned(16))) unsigned short As1[S * 2 * 2 * SBM * 8];
    __shared__ __attribute__((aligned(16))) unsigned short Bs0[S * 2 * 2 * SBN * 8];
    __shared__ __attribute__((aligned(16))) unsigned short Bs1[S * 2 * 2 * SBN * 8];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave >> 1) * 64;
    const int wn0 = (wave & 1) * 64;

    int pid = blockIdx.x;
    const int nb = g.gm * g.gn;
    if ((nb & 7) == 0) pid = (pid & 7) * (nb >> 3) + (pid >> 3);
    constexpr int GROUP = 8;
    const int group = pid / (GROUP * g.gn);
    const int first_m = group * GROUP;
    const int gsz = min(g.gm - first_m, GROUP);
    const int tm = first_m + (pid % gsz);
    const int tn = (pid % (GROUP * g.gn)) / gsz;
    const int m0 = tm * SBM, n0 = tn * SBN;
    const int M = g.M, N = g.N;
    const int kbeg = blockIdx.y * g.kchunk;
    const int nk = (min(g.Kp, kbeg + g.kchunk) - kbeg) / SBK;
    float* const c_re = g.c_re + blockIdx.y * g.split_stride;
    float* const c_im = g.c_im + blockIdx.y * g.split_stride;
    // padded rows and plane sizes
    const int64_t ra = (int64_t)g.gm * SBM, rbn = (int64_t)g.gn * SBN;
    const int64_t pa = ra * g.Kp, pb = rbn * g.Kp;
    const int wv = __builtin_amdgcn_readfirstlane(wave);   // the wavefront index as a scalar
    const unsigned lane_bytes = (unsigned)lane * 16u;

    // One k tile is 16 S wavefront loads for A ((s, p, c) x 4 blocks of 64 rows)
    // and 8 S for B; wavefront w issues loads w, w + 8, ...  Each load moves the
    // 16 bytes (8 k) of 64 consecutive rows, 1 KiB contiguous in the planes.
    auto issue = [&](unsigned short* as, unsigned short* bs, int k0) {
        const int kg0 = k0 >> 3;
#pragma unroll
        for (int u = 0; u < 3 * S; ++u) {
            const int q = wv + 8 * u;
            if (u < 2 * S) {
                const int rb = q & 3, spc = q >> 2, c = spc & 1, sp = spc >> 1;
                const unsigned short* base = g.a + (sp * pa + ((int64_t)(kg0 + c) * ra + m0 + rb * 64) * 8);
                dma16(base, lane_bytes, as + (spc * SBM + rb * 64) * 8);
            } else {
                const int qb = q - 16 * S;
                const int rb = qb & 1, spc = qb >> 1, c = spc & 1, sp = spc >> 1;
                const unsigned short* base = g.b + (sp * pb + ((int64_t)(kg0 + c) * rbn + n0 + rb * 64) * 8);
                dma16(base, lane_bytes, bs + (spc * SBN + rb * 64) * 8);
            }
        }
    };

    f32x16 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc_re[i][j][v] = 0.f; acc_im[i][j][v] = 0.f; }

    const int lrow = lane & 31;
    const int lchunk = lane >> 5;
    auto compute = [&](const unsigned short* as, const unsigned short* bs) {
#pragma unroll
        for (int sa = 0; sa < S; ++sa) {
            bf16x8 fa[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int p = 0; p < 2; ++p)
                    fa[i][p] = *(const bf16x8*)&as[lds_off<SBM>(sa, p, lchunk, wm0 + i * 32 + lrow)];
            for (int sb = 0; sb < S - sa; ++sb) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 fbr = *(const bf16x8*)&bs[lds_off<SBN>(sb, 0, lchunk, wn0 + j * 32 + lrow)];
                    const bf16x8 fbi = *(const bf16x8*)&bs[lds_off<SBN>(sb, 1, lchunk, wn0 + j * 32 + lrow)];
                    // -b_im: flip the sign bit of each BF16 (two per 32-bit word)
                    const u32x4 t = __builtin_bit_cast(u32x4, fbi) ^ 0x80008000u;
                    const bf16x8 fbn = __builtin_bit_cast(bf16x8, t);
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fbr, acc_re[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fbi, acc_im[i][j], 0, 0, 0);
                        acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][1], fbn, acc_re[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][1], fbr, acc_im[i][j], 0, 0, 0);
                    }
                }
            }
        }
    };

    // Tile t is in buffer t mod 2.  The loads of tile t + 1 are issued before
    // the MFMAs of tile t; the wait and the barrier after them make tile t + 1
    // visible and end every wavefront's reads of tile t before its buffer is
    // loaded again.
    if (nk > 0) {
        issue(As0, Bs0, kbeg);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    for (int kt = 0; kt < nk; ++kt) {
        const bool odd = kt & 1;
        if (kt + 1 < nk) issue(odd ? As0 : As1, odd ? Bs0 : Bs1, kbeg + (kt + 1) * SBK);
        compute(odd ? As1 : As0, odd ? Bs1 : Bs0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = m0 + wm0 + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
                const int c = n0 + wn0 + j * 32 + lrow;
                if (r < M && c < N) {
                    const int64_t off = (int64_t)r * g.ldc + c;
                    c_re[off] = acc_re[i][j][v];
                    c_im[off] = acc_im[i][j][v];
                }
            }
}

__global__ __launch_bounds__(NT, 1) void cgemm_bf16x3_planes_kernel(PlaneArgs g) { cgemm_planes_body<3>(g); }
__global__ __launch_bounds__(NT, 1) void cgemm_bf16x2_planes_kernel(PlaneArgs g) { cgemm_planes_body<2>(g); }

static int64_t pad_rows(int rows, bool is_a) {
    const int t = is_a ? SBM : SBN;
    return ((int64_t)rows + t - 1) / t * t;
}

int64_t split_planes_elems(int terms, int rows, int K, bool is_a) {
    return (int64_t)terms * 2 * pad_rows(rows, is_a) * (((int64_t)K + SBK - 1) / SBK * SBK);
}

hipError_t split_planes(int terms, int rows, int K, bool is_a, CView<float> X, unsigned short* planes,
                        hipStream_t stream) {
    if (rows <= 0 || K <= 0) return hipSuccess;
    if (terms != 2 && terms != 3) return hipErrorInvalidValue;
    const int Kp = (K + SBK - 1) / SBK * SBK;
    const int64_t rp = pad_rows(rows, is_a);
    if (rp > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t units = (rp >> 6) * (((Kp >> 3) + 3) >> 2);
    const unsigned grid = (unsigned)std::min<int64_t>(units, 65536);
    const bool vec = (X.ld % 4 == 0) && ((((uintptr_t)X.re) | ((uintptr_t)X.im)) & 15) == 0;
    const int r = rows, rpi = (int)rp;
    if (terms == 3) {
        if (vec) hipLaunchKernelGGL((split_planes_kernel<3, true>), dim3(grid), dim3(256), 0, stream, X.re, X.im, X.ld, r, rpi, K, Kp, planes);
        else hipLaunchKernelGGL((split_planes_kernel<3, false>), dim3(grid), dim3(256), 0, stream, X.re, X.im, X.ld, r, rpi, K, Kp, planes);
    } else {
        if (vec) hipLaunchKernelGGL((split_planes_kernel<2, true>), dim3(grid), dim3(256), 0, stream, X.re, X.im, X.ld, r, rpi, K, Kp, planes);
        else hipLaunchKernelGGL((split_planes_kernel<2, false>), dim3(grid), dim3(256), 0, stream, X.re, X.im, X.ld, r, rpi, K, Kp, planes);
    }
    return hipGetLastError();
}

hipError_t split_planes_t(int terms, int rows, int K, bool is_a, CView<float> Xt, unsigned short* planes,
                          hipStream_t stream) {
    if (rows <= 0 || K <= 0) return hipSuccess;
    if (terms != 2 && terms != 3) return hipErrorInvalidValue;
    const int Kp = (K + SBK - 1) / SBK * SBK;
    const int64_t rp = pad_rows(rows, is_a);
    if (rp > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t units = (rp >> 6) * (((Kp >> 3) + 3) >> 2);
    const unsigned grid = (unsigned)std::min<int64_t>(units, 65536);
    const int r = rows, rpi = (int)rp;
    if (terms == 3)
        hipLaunchKernelGGL((split_planes_t_kernel<3>), dim3(grid), dim3(256), 0, stream, Xt.re, Xt.im, Xt.ld, r, rpi, K, Kp, planes);
    else
        hipLaunchKernelGGL((split_planes_t_kernel<2>), dim3(grid), dim3(256), 0, stream, Xt.re, Xt.im, Xt.ld, r, rpi, K, Kp, planes);
    return hipGetLastError();
}

// The product of split operands; the k chunks of ksplit are those of launch_split.
static hipError_t launch_planes(int terms, int M, int N, int K, const unsigned short* pa, const unsigned short* pb,
                                CViewMut<float> C, int ksplit, int64_t split_stride, hipStream_t stream) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (terms != 2 && terms != 3) return hipErrorInvalidValue;
    PlaneArgs g;
    g.a = pa; g.b = pb;
    g.c_re = C.re; g.c_im = C.im; g.ldc = C.ld;
    g.M = M; g.N = N;
    g.Kp = (K + SBK - 1) / SBK * SBK;
    g.gm = (M + SBM - 1) / SBM;
    g.gn = (N + SBN - 1) / SBN;
    if (ksplit < 1) ksplit = 1;
    g.kchunk = (((K + ksplit - 1) / ksplit) + SBK - 1) / SBK * SBK;
    if (g.kchunk < SBK) g.kchunk = SBK;
    ksplit = (K + g.kchunk - 1) / g.kchunk;
    if (ksplit < 1) ksplit = 1;
    g.split_stride = ksplit > 1 ? split_stride : 0;
    const int64_t nblocks = (int64_t)g.gm * g.gn;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    // 16-byte aligned planes for the 16-byte loads
    if (((((uintptr_t)pa) | ((uintptr_t)pb)) & 15) != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nblocks, (unsigned)ksplit);
    if (terms == 3) hipLaunchKernelGGL(cgemm_bf16x3_planes_kernel, grid, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(cgemm_bf16x2_planes_kernel, grid, dim3(NT), 0, stream, g);
    return hipGetLastError();
}

hipError_t cgemm_bf16_planes(int terms, int M, int N, int K, const unsigned short* pa, const unsigned short* pb,
                             CViewMut<float> C, hipStream_t stream) {
    return launch_planes(terms, M, N, K, pa, pb, C, 1, 0, stream);
}

hipError_t cgemm_bf16_planes_splitk(int terms, int M, int N, int K, const unsigned short* pa,
                                    const unsigned short* pb, float* ws_re, float* ws_im, int ksplit,
                                    hipStream_t stream) {
    return launch_planes(terms, M, N, K, pa, pb, {ws_re, ws_im, N}, ksplit, (int64_t)M * N, stream);
}

hipError_t cgemm_bf16_nt(int terms, int M, int N, int K, CView<float> A, CView<float> B, CViewMut<float> C,
                         hipStream_t stream) {
    return launch_split(terms, M, N, K, A, B, C, 1, 0, stream);
}

hipError_t cgemm_bf16_nt_splitk(int terms, int M, int N, int K, CView<float> A, CView<float> B, float* ws_re,
                                float* ws_im, int ksplit, hipStream_t stream) {
    return launch_split(terms, M, N, K, A, B, {ws_re, ws_im, N}, ksplit, (int64_t)M * N, stream);
}

}  // namespace mpsk
