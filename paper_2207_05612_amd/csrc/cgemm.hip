// Complex planar GEMM on CDNA4 matrix cores (gfx950).
//
// Every contraction of the compression step (environments, two-site local
// tensor, Gram matrices of the truncation, sampling) is a dense complex
// matrix product; here each complex multiply-add is four real MFMA products
// on planar (separate real / imaginary) operands:
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br.
//
// Tiling: 256 threads = 4 wavefronts of 64 lanes in a 2 x 2 arrangement.
// FP32 uses v_mfma_f32_32x32x2_f32 (wave tile 64 x 64 complex, block tile
// 128 x 128, BK = 16); FP64 uses v_mfma_f64_16x16x4_f64 (wave tile 64 x 32,
// block tile 128 x 64, BK = 8).  Operand tiles go global -> registers -> LDS
// with k-major rows ([k][m] and [k][n]) so that the lanes of one MFMA operand
// read consecutive LDS words; two LDS buffers let the next tile's global loads
// overlap the current tile's MFMAs with one barrier per k-tile.  Launches map
// block ids to tiles XCD-first (8 XCDs, each with its own L2) and then in
// groups of 8 tile rows so that neighbouring tiles share operand panels in L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace mpsk {

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
    static constexpr int MT = 32;  // output tile edge
    static constexpr int KT = 2;   // k per instruction
    static constexpr int NACC = 16;
    typedef float acc_t __attribute__((ext_vector_type(16)));
    __device__ static inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    // row of accumulator element v held by lane l (column = l % 32)
    __device__ static inline int row(int v, int lane) { return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); }
};

template <>
struct Mfma<double> {
    static constexpr int MT = 16;
    static constexpr int KT = 4;
    static constexpr int NACC = 4;
    typedef double acc_t __attribute__((ext_vector_type(4)));
    __device__ static inline acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int v, int lane) { return v * 4 + (lane >> 4); }
};

template <typename TIn, typename TAcc>
struct GemmArgs {
    const TIn* a_re;
    const TIn* a_im;
    const TIn* b_re;
    const TIn* b_im;
    TAcc* c_re;
    TAcc* c_im;
    int64_t lda, ldb, ldc;
    int M, N, K;
    int gm, gn;
    int lower_only;   // only the tiles that hold an element with column <= row: blockIdx.x
                      // enumerates them row by row (n_active of them)
    int n_active;
    int kchunk;       // k range of split blockIdx.y: [y kchunk, (y+1) kchunk)
    int64_t split_stride;   // C offset of split y (partial sums); 0 without split
    int64_t sa, sb, sc;     // batch strides (elements) of A, B, C: batch z = blockIdx.z
};

// SUB: C -= A B instead of C = A B.
template <typename TIn, typename TAcc, int OPA, int OPB, int BM, int BN, int BK, bool SUB = false>
__global__ __launch_bounds__(256) void cgemm_kernel(GemmArgs<TIn, TAcc> g) {
    using MF = Mfma<TAcc>;
    constexpr int MT = MF::MT;
    constexpr int WM = BM / 2, WN = BN / 2;        // wave tile
    constexpr int TM = WM / MT, TN = WN / MT;       // MFMA tiles per wave
    constexpr int PADA = (sizeof(TAcc) == 8) ? 4 : 4;
    constexpr int LDA_S = BM + PADA, LDB_S = BN + PADA;
    constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
    static_assert(BM * BK % 256 == 0 && BN * BK % 256 == 0, "tile/thread mismatch");

    __shared__ TAcc As[2][2][BK][LDA_S];
    __shared__ TAcc Bs[2][2][BK][LDB_S];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave >> 1) * WM;
    const int wn0 = (wave & 1) * WN;

    // ---- tile mapping: XCD-contiguous, then grouped rows (or, for lower-triangle
    //      products, the active tiles row by row, so that every XCD gets the same count)
    int pid = blockIdx.x;
    const int nb = g.lower_only ? g.n_active : g.gm * g.gn;
    if ((nb & 7) == 0) pid = (pid & 7) * (nb >> 3) + (pid >> 3);
    int tm, tn;
    if (g.lower_only) {
        int r = 0, rem = pid;
        for (;;) {
            const int cnt = min(g.gn, (BM * r + BM - 1) / BN + 1);
            if (rem < cnt || r + 1 >= g.gm) break;
            rem -= cnt;
            ++r;
        }
        tm = r;
        tn = rem;
    } else {
        constexpr int GROUP = 8;
        const int group = pid / (GROUP * g.gn);
        const int first_m = group * GROUP;
        const int gsz = min(g.gm - first_m, GROUP);
        tm = first_m + (pid % gsz);
        tn = (pid % (GROUP * g.gn)) / gsz;
    }
    const int m0 = tm * BM, n0 = tn * BN;
    if (g.lower_only && (n0 > m0 + BM - 1 || tn >= g.gn)) return;   // not an active tile (uniform per block)

    const int M = g.M, N = g.N;
    // split-K: this block sums k in [kbeg, K) of its own chunk
    const int kbeg = blockIdx.y * g.kchunk;
    const int K = min(g.K, kbeg + g.kchunk);
    const int64_t bz = blockIdx.z;
    TAcc* const c_re = g.c_re + blockIdx.y * g.split_stride + bz * g.sc;
    TAcc* const c_im = g.c_im + blockIdx.y * g.split_stride + bz * g.sc;
    const TIn* const a_re = g.a_re + bz * g.sa;
    const TIn* const a_im = g.a_im + bz * g.sa;
    const TIn* const b_re = g.b_re + bz * g.sb;
    const TIn* const b_im = g.b_im + bz * g.sb;

    TIn ra_re[EA], ra_im[EA], rb_re[EB], rb_im[EB];

    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int i = 0; i < EA; ++i) {
            const int idx = tid + 256 * i;
            int m, k;
            if (OPA == OP_N) { k = idx % BK; m = idx / BK; }
            else             { m = idx % BM; k = idx / BM; }
            const int gm_ = m0 + m, gk = k0 + k;
            TIn vr = 0, vi = 0;
            if (gm_ < M && gk < K) {
                const int64_t off = (OPA == OP_N) ? (int64_t)gm_ * g.lda + gk : (int64_t)gk * g.lda + gm_;
                vr = a_re[off];
                vi = a_im[off];
            }
            ra_re[i] = vr;
            ra_im[i] = vi;
        }
#pragma unroll
        for (int i = 0; i < EB; ++i) {
            const int idx = tid + 256 * i;
            int n, k;
            if (OPB == OP_N) { n = idx % BN; k = idx / BN; }
            else             { k = idx % BK; n = idx / BK; }
            const int gn_ = n0 + n, gk = k0 + k;
            TIn vr = 0, vi = 0;
            if (gn_ < N && gk < K) {
                const int64_t off = (OPB == OP_N) ? (int64_t)gk * g.ldb + gn_ : (int64_t)gn_ * g.ldb + gk;
                vr = b_re[off];
                vi = b_im[off];
            }
            rb_re[i] = vr;
            rb_im[i] = vi;
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int i = 0; i < EA; ++i) {
            const int idx = tid + 256 * i;
            int m, k;
            if (OPA == OP_N) { k = idx % BK; m = idx / BK; }
            else             { m = idx % BM; k = idx / BM; }
            // conjugation is applied here, after the MFMAs of the current tile, so that
            // the loads stay in flight until then
            As[buf][0][k][m] = (TAcc)ra_re[i];
            As[buf][1][k][m] = OPA == OP_C ? -(TAcc)ra_im[i] : (TAcc)ra_im[i];
        }
#pragma unroll
        for (int i = 0; i < EB; ++i) {
            const int idx = tid + 256 * i;
            int n, k;
            if (OPB == OP_N) { n = idx % BN; k = idx / BN; }
            else             { k = idx % BK; n = idx / BK; }
            Bs[buf][0][k][n] = (TAcc)rb_re[i];
            Bs[buf][1][k][n] = OPB == OP_C ? -(TAcc)rb_im[i] : (TAcc)rb_im[i];
        }
    };

    typename MF::acc_t acc_re[TM][TN], acc_im[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < MF::NACC; ++v) { acc_re[i][j][v] = 0; acc_im[i][j][v] = 0; }

    const int nk = (K - kbeg + BK - 1) / BK;
    load_tiles(kbeg);
    store_tiles(0);
    __syncthreads();

    const int lrow = lane % MT;
    const int lk = lane / MT;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_tiles(kbeg + (kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += MF::KT) {
            TAcc ar[TM], ai[TM], nai[TM], br[TN], bi[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                ar[i] = As[buf][0][kk + lk][wm0 + i * MT + lrow];
                ai[i] = As[buf][1][kk + lk][wm0 + i * MT + lrow];
                nai[i] = -ai[i];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                br[j] = Bs[buf][0][kk + lk][wn0 + j * MT + lrow];
                bi[j] = Bs[buf][1][kk + lk][wn0 + j * MT + lrow];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc_re[i][j] = MF::mma(ar[i], br[j], acc_re[i][j]);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc_im[i][j] = MF::mma(ar[i], bi[j], acc_im[i][j]);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc_re[i][j] = MF::mma(nai[i], bi[j], acc_re[i][j]);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc_im[i][j] = MF::mma(ai[i], br[j], acc_im[i][j]);
        }
        if (kt + 1 < nk) store_tiles(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < MF::NACC; ++v) {
                const int r = m0 + wm0 + i * MT + MF::row(v, lane);
                const int c = n0 + wn0 + j * MT + lrow;
                if (r < M && c < N) {
                    const int64_t off = (int64_t)r * g.ldc + c;
                    if (SUB) {
                        c_re[off] -= acc_re[i][j][v];
                        c_im[off] -= acc_im[i][j][v];
                    } else {
                        c_re[off] = acc_re[i][j][v];
                        c_im[off] = acc_im[i][j][v];
                    }
                }
            }
}

template <typename TIn, typename TAcc, int BM, int BN, int BK>
static hipError_t launch(int opa, int opb, int M, int N, int K, CView<TIn> A, CView<TIn> B,
                         CViewMut<TAcc> C, hipStream_t stream, int lower_only = 0, int ksplit = 1,
                         int64_t split_stride = 0, int sub = 0, int batch = 1, int64_t sa = 0, int64_t sb = 0,
                         int64_t sc = 0) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs<TIn, TAcc> g;
    g.a_re = A.re; g.a_im = A.im; g.lda = A.ld;
    g.b_re = B.re; g.b_im = B.im; g.ldb = B.ld;
    g.c_re = C.re; g.c_im = C.im; g.ldc = C.ld;
    g.M = M; g.N = N; g.K = K;
    g.gm = (M + BM - 1) / BM;
    g.gn = (N + BN - 1) / BN;
    g.lower_only = lower_only;
    g.n_active = 0;
    if (lower_only)
        for (int r = 0; r < g.gm; ++r) g.n_active += std::min(g.gn, (BM * r + BM - 1) / BN + 1);
    g.sa = sa;
    g.sb = sb;
    g.sc = sc;
    if (batch < 1 || batch > 65535) return hipErrorInvalidValue;
    if (ksplit < 1) ksplit = 1;
    g.kchunk = (((K + ksplit - 1) / ksplit) + BK - 1) / BK * BK;
    if (g.kchunk < BK) g.kchunk = BK;
    ksplit = (K + g.kchunk - 1) / g.kchunk;
    if (ksplit < 1) ksplit = 1;
    g.split_stride = ksplit > 1 ? split_stride : 0;
    const int64_t nblocks = lower_only ? (int64_t)g.n_active : (int64_t)g.gm * g.gn;
    if ((int64_t)g.gm * g.gn > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblocks, (unsigned)ksplit, (unsigned)batch), block(256);
#define MPS_GEMM_CASE(OA, OB)                                                                     \
    if (opa == OA && opb == OB) {                                                                 \
        hipLaunchKernelGGL((cgemm_kernel<TIn, TAcc, OA, OB, BM, BN, BK>), grid, block, 0, stream, g); \
        return hipGetLastError();                                                                 \
    }
    if (sub) {
        // the subtracting forms exist for the FP64 back-transformation only (C^H N and N N)
        if (sizeof(TAcc) != 8 || opb != OP_N || (opa != OP_C && opa != OP_N)) return hipErrorInvalidValue;
        if (opa == OP_C)
            hipLaunchKernelGGL((cgemm_kernel<TIn, TAcc, OP_C, OP_N, BM, BN, BK, true>), grid, block, 0, stream, g);
        else
            hipLaunchKernelGGL((cgemm_kernel<TIn, TAcc, OP_N, OP_N, BM, BN, BK, true>), grid, block, 0, stream, g);
        return hipGetLastError();
    }
    MPS_GEMM_CASE(OP_N, OP_N)
    MPS_GEMM_CASE(OP_N, OP_T)
    MPS_GEMM_CASE(OP_N, OP_C)
    MPS_GEMM_CASE(OP_C, OP_N)
    MPS_GEMM_CASE(OP_C, OP_T)
    MPS_GEMM_CASE(OP_C, OP_C)
#undef MPS_GEMM_CASE
    return hipErrorInvalidValue;
}

hipError_t cgemm_f32(int opa, int opb, int M, int N, int K, CView<float> A, CView<float> B,
                     CViewMut<float> C, hipStream_t stream) {
    return launch<float, float, 128, 128, 16>(opa, opb, M, N, K, A, B, C, stream);
}

int splitk_chunks(int K, int ksplit, int bk) {
    if (ksplit < 1) ksplit = 1;
    int kc = (((K + ksplit - 1) / ksplit) + bk - 1) / bk * bk;
    if (kc < bk) kc = bk;
    return (K + kc - 1) / kc;
}

hipError_t cgemm_f32_splitk(int opa, int opb, int M, int N, int K, CView<float> A, CView<float> B,
                            float* ws_re, float* ws_im, int ksplit, hipStream_t stream) {
    // partial sums of split y go to ws + y M N (row-major, ld = N)
    return launch<float, float, 128, 128, 16>(opa, opb, M, N, K, A, B, {ws_re, ws_im, N}, stream, 0, ksplit,
                                              (int64_t)M * N);
}

// C[r][c] = sum_y ws[y][r][c], summed in FP64 in split order (deterministic)
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* __restrict__ wre,
                                                            const float* __restrict__ wim, int nsplit,
                                                            int64_t M, int64_t N, float* __restrict__ cre,
                                                            float* __restrict__ cim, int64_t ldc) {
    const int64_t total = M * N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        double sr = 0, si = 0;
        for (int y = 0; y < nsplit; ++y) {
            sr += wre[y * total + idx];
            si += wim[y * total + idx];
        }
        const int64_t r = idx / N, c = idx % N;
        cre[r * ldc + c] = (float)sr;
        cim[r * ldc + c] = (float)si;
    }
}

hipError_t splitk_reduce(const float* ws_re, const float* ws_im, int nsplit, int64_t M, int64_t N, float* c_re,
                         float* c_im, int64_t ldc, hipStream_t stream) {
    const int64_t total = M * N;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 1048576) g = 1048576;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)g), dim3(256), 0, stream, ws_re, ws_im, nsplit, M, N,
                       c_re, c_im, ldc);
    return hipGetLastError();
}

hipError_t cgemm_f64(int opa, int opb, int M, int N, int K, CView<double> A, CView<double> B,
                     CViewMut<double> C, hipStream_t stream, int lower_only) {
    return launch<double, double, 128, 64, 8>(opa, opb, M, N, K, A, B, C, stream, lower_only);
}

hipError_t cgemm_f64_sub(int opa, int opb, int M, int N, int K, CView<double> A, CView<double> B, CViewMut<double> C,
                         hipStream_t stream) {
    return launch<double, double, 128, 64, 8>(opa, opb, M, N, K, A, B, C, stream, 0, 1, 0, 1);
}

hipError_t cgemm_f64_batched_sub(int M, int N, int K, CView<double> A, int64_t sa, CView<double> B, int64_t sb,
                                 CViewMut<double> C, int64_t sc, int batch, hipStream_t stream) {
    return launch<double, double, 128, 64, 8>(OP_N, OP_N, M, N, K, A, B, C, stream, 0, 1, 0, 1, batch, sa, sb, sc);
}

hipError_t cgemm_f64_batched(int opa, int opb, int M, int N, int K, CView<double> A, int64_t sa, CView<double> B,
                             int64_t sb, CViewMut<double> C, int64_t sc, int batch, hipStream_t stream) {
    return launch<double, double, 128, 64, 8>(opa, opb, M, N, K, A, B, C, stream, 0, 1, 0, 0, batch, sa, sb, sc);
}

hipError_t cgemm_f64_batched_splitk(int opa, int opb, int M, int N, int K, CView<double> A, int64_t sa,
                                    CView<double> B, int64_t sb, double* ws_re, double* ws_im, int ksplit, int batch,
                                    hipStream_t stream) {
    // partial sums of split y, batch z at ws + (y batch + z) M N: reduce as (batch M) x N
    return launch<double, double, 128, 64, 8>(opa, opb, M, N, K, A, B, {ws_re, ws_im, N}, stream, 0, ksplit,
                                              (int64_t)batch * M * N, 0, batch, sa, sb, (int64_t)M * N);
}

hipError_t cgemm_f32in_f64(int opa, int opb, int M, int N, int K, CView<float> A,
                           CView<float> B, CViewMut<double> C, hipStream_t stream, int lower_only) {
    return launch<float, double, 128, 64, 8>(opa, opb, M, N, K, A, B, C, stream, lower_only);
}

hipError_t cgemm_f32in_f64_splitk(int opa, int opb, int M, int N, int K, CView<float> A, CView<float> B,
                                  double* ws_re, double* ws_im, int ksplit, int lower_only, hipStream_t stream) {
    return launch<float, double, 128, 64, 8>(opa, opb, M, N, K, A, B, {ws_re, ws_im, N}, stream, lower_only, ksplit,
                                             (int64_t)M * N);
}

hipError_t cgemm_f64_splitk(int opa, int opb, int M, int N, int K, CView<double> A, CView<double> B,
                            double* ws_re, double* ws_im, int ksplit, int lower_only, hipStream_t stream) {
    return launch<double, double, 128, 64, 8>(opa, opb, M, N, K, A, B, {ws_re, ws_im, N}, stream, lower_only, ksplit,
                                              (int64_t)M * N);
}

// C[r][c] = sum_y ws[y][r][c] in split order (FP64 partials)
__global__ __launch_bounds__(256) void splitk_reduce64_kernel(const double* __restrict__ wre,
                                                              const double* __restrict__ wim, int nsplit,
                                                              int64_t M, int64_t N, double* __restrict__ cre,
                                                              double* __restrict__ cim, int64_t ldc) {
    const int64_t total = M * N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        double sr = 0, si = 0;
        for (int y = 0; y < nsplit; ++y) {
            sr += wre[y * total + idx];
            si += wim[y * total + idx];
        }
        const int64_t r = idx / N, c = idx % N;
        cre[r * ldc + c] = sr;
        cim[r * ldc + c] = si;
    }
}

hipError_t splitk_reduce64(const double* ws_re, const double* ws_im, int nsplit, int64_t M, int64_t N, double* c_re,
                           double* c_im, int64_t ldc, hipStream_t stream) {
    const int64_t total = M * N;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 1048576) g = 1048576;
    hipLaunchKernelGGL(splitk_reduce64_kernel, dim3((unsigned)g), dim3(256), 0, stream, ws_re, ws_im, nsplit, M, N,
                       c_re, c_im, ldc);
    return hipGetLastError();
}

}  // namespace mpsk
