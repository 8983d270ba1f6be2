// Internal declarations shared by the HIP sources of the DMRG library.
// Not part of the public ABI (see include/mps_dmrg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpsk {

// Operand modes of the complex GEMM C = op(A) op(B).
//   A: OP_N = row-major M x K;  OP_C = conj-transpose of a row-major K x M.
//   B: OP_N = row-major K x N;  OP_T = transpose of a row-major N x K;
//      OP_C = conj-transpose of a row-major N x K.
enum Op { OP_N = 0, OP_T = 1, OP_C = 2 };

// A planar complex matrix view: re[] and im[] with row stride ld (elements).
template <typename T>
struct CView {
    const T* re;
    const T* im;
    int64_t ld;
};
template <typename T>
struct CViewMut {
    T* re;
    T* im;
    int64_t ld;
};

// Complex GEMM, C (M x N) = op(A) op(B), overwriting C.
//   TIn  element type of A and B (float or double)
//   TAcc arithmetic / output type (float with TIn=float; double with either)
// lower_only: only tiles holding elements with column <= row are computed
// (for Hermitian products whose consumer reads the lower triangle only).
// Returns hipSuccess or the launch error.
hipError_t cgemm_f32(int opa, int opb, int M, int N, int K, CView<float> A, CView<float> B,
                     CViewMut<float> C, hipStream_t stream);
hipError_t cgemm_f64(int opa, int opb, int M, int N, int K, CView<double> A, CView<double> B,
                     CViewMut<double> C, hipStream_t stream, int lower_only = 0);
hipError_t cgemm_f32in_f64(int opa, int opb, int M, int N, int K, CView<float> A,
                           CView<float> B, CViewMut<double> C, hipStream_t stream, int lower_only = 0);

// Split-K FP32 complex GEMM: the K range is cut into chunks of whole k-tiles;
// chunk y writes its partial product to ws + y M N (ld N).  splitk_chunks()
// gives the number of chunks a request for ksplit produces; splitk_reduce()
// sums them in FP64 in chunk order into C.
int splitk_chunks(int K, int ksplit, int bk);
hipError_t cgemm_f32_splitk(int opa, int opb, int M, int N, int K, CView<float> A, CView<float> B,
                            float* ws_re, float* ws_im, int ksplit, hipStream_t stream);
hipError_t splitk_reduce(const float* ws_re, const float* ws_im, int nsplit, int64_t M, int64_t N, float* c_re,
                         float* c_im, int64_t ldc, hipStream_t stream);
hipError_t cgemm_bf16_nt_splitk(int terms, int M, int N, int K, CView<float> A, CView<float> B, float* ws_re,
                                float* ws_im, int ksplit, hipStream_t stream);
// FP64-accumulating split-K variants (BK = 8), used by the Gram matrices of the truncation
hipError_t cgemm_f32in_f64_splitk(int opa, int opb, int M, int N, int K, CView<float> A, CView<float> B,
                                  double* ws_re, double* ws_im, int ksplit, int lower_only, hipStream_t stream);
hipError_t cgemm_f64_splitk(int opa, int opb, int M, int N, int K, CView<double> A, CView<double> B,
                            double* ws_re, double* ws_im, int ksplit, int lower_only, hipStream_t stream);
hipError_t splitk_reduce64(const double* ws_re, const double* ws_im, int nsplit, int64_t M, int64_t N, double* c_re,
                           double* c_im, int64_t ldc, hipStream_t stream);

// Split-precision complex GEMM: C (M x N) = A (M x K) B^T with B stored N x K,
// FP32 operands split into `terms` BF16 terms (3: six BF16 MFMA products per
// real product, about FP32 accuracy; 2: three products, about 2^-16 relative),
// FP32 accumulation.
hipError_t cgemm_bf16_nt(int terms, int M, int N, int K, CView<float> A, CView<float> B, CViewMut<float> C,
                         hipStream_t stream);

// The same product with each operand split once beforehand.  split_planes
// writes the `terms` BF16 terms of an operand (rows x K, FP32 planar) as
// planes of split_planes_elems() elements (rows padded to the product's tile,
// 256 for the A operand, 128 for B; k padded to 16; the padding zero; stored
// by groups of 8 k, rows consecutive within a group, as the tiles sit in LDS);
// cgemm_bf16_planes(_splitk) multiplies two such operands and gives the same
// bits as cgemm_bf16_nt(_splitk) on the FP32 operands.  Planes must be 16-byte
// aligned.
int64_t split_planes_elems(int terms, int rows, int K, bool is_a);
hipError_t split_planes(int terms, int rows, int K, bool is_a, CView<float> X, unsigned short* planes,
                        hipStream_t stream);
// The planes of X = Xt^T for Xt (K x rows, FP32 planar, row-major): the split of
// a transposed operand without forming it.
hipError_t split_planes_t(int terms, int rows, int K, bool is_a, CView<float> Xt, unsigned short* planes,
                          hipStream_t stream);
hipError_t cgemm_bf16_planes(int terms, int M, int N, int K, const unsigned short* pa, const unsigned short* pb,
                             CViewMut<float> C, hipStream_t stream);
hipError_t cgemm_bf16_planes_splitk(int terms, int M, int N, int K, const unsigned short* pa,
                                    const unsigned short* pb, float* ws_re, float* ws_im, int ksplit,
                                    hipStream_t stream);

// Structured MPO application on one site.
//   in  [P][w_in][2 (t)][Q],  out [P][2 (s)][w_out][Q]
//   w_in = H * r_in * lo, w_out = H * r_out * lo; one of r_in, r_out is 1.
//   out[p][s][(h r_out + a_out) lo + l][q] =
//       sum_{a_in, t} op[a_out][a_in][s][t] in[p][(h r_in + a_in) lo + l][t][q]
// One factor of a site's MPO tensor: it maps the bond digit of one gate
// (stride lo, H combinations of the more significant digits) from r_in to
// r_out values and the physical index t to s.  Input layout [P][w_in][2 (t)][Q];
// output [P][2 (s)][w_out][Q], or [P][w_out][2 (s)][Q] when out_ws is set (the
// input layout of the next factor, for sites where several layers act).
struct MpoSiteOp {
    int r_in, r_out, lo, H;
    int out_ws;
    double re[16], im[16];     // [(a_out * r_in + a_in) * 4 + s * 2 + t]
};
template <typename T>
hipError_t mpo_apply(const MpoSiteOp& op, int64_t P, int64_t Q, const T* in_re, const T* in_im,
                     T* out_re, T* out_im, hipStream_t stream);

// Site tensor (FP64 planar, [Dl][2][Dr]) -> working copy, optionally with the
// virtual legs swapped ([Dr][2][Dl]) and converted to T.
template <typename T>
hipError_t site_to_view(const double* re, const double* im, int Dl, int Dr, int swap_legs,
                        T* out_re, T* out_im, hipStream_t stream);

// View tensor V[a][s][x] (dims Dl_v, 2, Dr_v) as the k-major (2 Dr_v) x Dl_v
// FP32 matrix O[(s Dr_v + x) Dl_v + a]; stored layout as in site_to_view.
hipError_t site_to_kmajor(const double* re, const double* im, int Dlv, int Drv, int swap_legs, float* ore,
                          float* oim, hipStream_t stream);


// out (k x m, FP32) = in^H of a row-major m x k FP64 planar matrix.
hipError_t adjoint_to_f32(const double* re, const double* im, int64_t m, int64_t k, float* ore, float* oim,
                          hipStream_t stream);

// Element-wise conversion of a planar array of n complex numbers.
template <typename TI, typename TO>
hipError_t convert_planar(const TI* re, const TI* im, int64_t n, TO* ore, TO* oim,
                          hipStream_t stream);

// Fill a planar array with (value, 0).
template <typename T>
hipError_t fill_planar(T* re, T* im, int64_t n, double value, hipStream_t stream);

// sum |x|^2 of a planar array, deterministic two-pass reduction in FP64.
// partial must hold at least 1024 doubles; result written to *out (device).
template <typename T>
hipError_t norm2(const T* re, const T* im, int64_t n, double* partial, double* out,
                 hipStream_t stream);

// Planar row-major rows x cols <-> interleaved column-major (LAPACK layout).
hipError_t rm_planar_to_cm(const double* re, const double* im, int64_t rows, int64_t cols, double* out_z,
                           hipStream_t stream);
hipError_t cm_to_rm_planar(const double* in_z, int64_t rows, int64_t cols, double* re, double* im,
                           hipStream_t stream);

// Row-major planar Hermitian n x n -> interleaved column-major (LAPACK layout).
// Only the row-major lower triangle is meaningful on input; it becomes the
// column-major upper triangle, which is what the eigensolver reads.
hipError_t pack_hermitian(const double* re, const double* im, int n, double* out_z,
                          hipStream_t stream);

// From rocSOLVER's eigenvectors (interleaved, column-major, ascending
// eigenvalues) take the k columns of the largest eigenvalues, largest first,
// into a row-major planar n x k matrix; optionally scale column c by scale[c].
hipError_t take_top_eigvecs(const double* evec_z, int n, int k, const double* scale_dev,
                            double* out_re, double* out_im, hipStream_t stream);

// out (k x m row-major) = diag(s) * in^H where in is m x k row-major; planar.
hipError_t scaled_adjoint(const double* in_re, const double* in_im, int m, int k,
                          const double* s_dev, double* out_re, double* out_im,
                          hipStream_t stream);

// Scale the columns of a planar row-major m x k matrix by s[c] (device array).
hipError_t scale_columns(double* re, double* im, int64_t m, int k, const double* s_dev,
                         hipStream_t stream);

// Scale a planar array by a device scalar: x *= (*s).
template <typename T>
hipError_t scale_by_device_scalar(T* re, T* im, int64_t n, const double* s_dev,
                                  hipStream_t stream);

// Sequential-product step of sampling / amplitude evaluation.
//   U [S][2][D] (planar); for row r choose t: given (bits_in) or sampled from
//   p_t = ||U[r][t][:]||^2 with the Philox draw of (seed, sample0 + r, site);
//   V_out[r][:] = U[r][t][:] (normalised when sampling).  bits_out[r] = t.
template <typename T>
hipError_t select_rows(const T* u_re, const T* u_im, int64_t S, int D, int sampling,
                       const uint8_t* bits_in, uint64_t seed, int64_t sample0, int site,
                       T* v_re, T* v_im, uint8_t* bits_out, hipStream_t stream);

// Transfer-matrix step for <Z_i Z_j>: E'[b][b'] = sum_{a,a',s} conj(A[a][s][b]) w_s E[a][a'] A[a'][s][b']
// done with two GEMMs by the caller; this applies w_s = (+1, -1) to the physical leg.
hipError_t apply_z_phys(const double* re, const double* im, int Dl, int Dr, double* out_re,
                        double* out_im, hipStream_t stream);

// ---------------------------------------------------------------- hetrd.hip
// Persistent-kernel Householder tridiagonalisation (n <= hetrd_max_n()).
int hetrd_max_n();
size_t hetrd_workspace_bytes(int n);
// Full Hermitian matrix (column-major, interleaved complex) from the lower
// triangle of a row-major planar matrix.
hipError_t hermitian_full_colmajor(const double* re, const double* im, int n, double* out_z, hipStream_t stream);
// a_z: full Hermitian matrix (column-major interleaved, lda = n, read only);
// d (n), e (n - 1) real; tau_z (n - 1 complex); vh: planar row-major
// (n - 1) x n, row i = conj(v_i).  *abort_flag points at a device int that
// is non-zero when the kernel gave up waiting (results then invalid).
hipError_t hetrd_persistent(const double* a_z, int n, double* d, double* e, double* tau_z, double* vh_re,
                            double* vh_im, void* ws, size_t ws_bytes, int** abort_flag, hipStream_t stream);
// One reduction's arguments (as for hetrd_persistent).
struct TrRequest {
    const double* a_z;
    int n;
    double* d;
    double* e;
    double* tau_z;
    double* vh_re;
    double* vh_im;
    void* ws;
    size_t ws_bytes;
    int** abort_flag;
};
// Up to hetrd_batch_max() reductions of order > 128 in one cooperative launch on `stream`
// (instance i on hetrd_workgroups(n_i) workgroups; at most 256 in total); each instance
// keeps its own workspace, flags and abort flag.
int hetrd_batch_max();
int hetrd_workgroups(int n);
hipError_t hetrd_persistent_multi(const TrRequest* reqs, int count, hipStream_t stream);
// Divide-and-conquer eigen-decomposition of the real symmetric tridiagonal
// matrix (d, e) of order n <= stedc_dc_max_n(), all on the device: d is
// replaced by the eigenvalues in ascending order and z (column-major, leading
// dimension ldz) receives the orthonormal eigenvectors; e is not modified.
// ws: stedc_dc_workspace_bytes(n) bytes of device memory.
int stedc_dc_max_n();
size_t stedc_dc_workspace_bytes(int n);
hipError_t stedc_dc(int n, double* d, const double* e, double* z, int ldz, void* ws, size_t ws_bytes,
                    hipStream_t stream);

// Reflectors per block of the blocked back-transformation of an order-n
// reduction (64, or 256 above order 512).
int wy_block(int n);
// The 64 x 64 diagonal sub-blocks of the T factors of the compact WY forms
// I - V_b T_b V_b^H of nblk blocks of nb reflectors (nb a multiple of 64):
// S_b = V_b^H V_b and T_b planar row-major nb x nb, block b at b nb^2; tau
// interleaved complex, nblk nb entries (tau = 0 marks an identity
// reflector).  Sub-blocks off the diagonal are not written.
hipError_t wy_t_diag_factors(const double* s_re, const double* s_im, int nblk, int nb, const double* tau_z,
                             double* t_re, double* t_im, hipStream_t stream);
// Top-k eigenvectors of a real column-major eigenvector matrix (ascending
// eigenvalues) as planar complex row-major n x k, largest first.
hipError_t take_top_real_eigvecs(const double* evec, int n, int k, double* out_re, double* out_im, hipStream_t stream);
// Batched FP64 GEMMs: batch z uses A + z sa, B + z sb, C + z sc (elements).
// The split-K form writes the partial sums of split y, batch z to
// ws + (y batch + z) M N; splitk_reduce64 over (batch M) x N sums them.
hipError_t cgemm_f64_batched(int opa, int opb, int M, int N, int K, CView<double> A, int64_t sa, CView<double> B,
                             int64_t sb, CViewMut<double> C, int64_t sc, int batch, hipStream_t stream);
hipError_t cgemm_f64_batched_splitk(int opa, int opb, int M, int N, int K, CView<double> A, int64_t sa,
                                    CView<double> B, int64_t sb, double* ws_re, double* ws_im, int ksplit, int batch,
                                    hipStream_t stream);
// C -= op(A) op(B) (FP64 complex, same operand conventions as cgemm_f64).
hipError_t cgemm_f64_sub(int opa, int opb, int M, int N, int K, CView<double> A, CView<double> B, CViewMut<double> C,
                         hipStream_t stream);
// C_z -= A_z B_z over a batch (FP64, opa = opb = N): the off-diagonal blocks of merged WY T factors.
hipError_t cgemm_f64_batched_sub(int M, int N, int K, CView<double> A, int64_t sa, CView<double> B, int64_t sb,
                                 CViewMut<double> C, int64_t sc, int batch, hipStream_t stream);

// ---- exact statevector (FP64 planar, chain site q = index bit n-1-q) ----
struct SvGate2 { double re[16], im[16]; };   // [row * 4 + col], row = 2 s_a + s_b
struct SvGate1 { double re[4], im[4]; };     // [row * 2 + col]
hipError_t sv_fill(double* re, double* im, uint64_t dim, uint64_t one_at, hipStream_t s);
// U on the qubits at index bits pa (high bit of U's row) and pb.  re and im must be
// 16-byte aligned (hipErrorInvalidValue otherwise).
hipError_t sv_apply_2q(double* re, double* im, int n, int pa, int pb, const SvGate2& g, hipStream_t s);
hipError_t sv_apply_1q(double* re, double* im, int n, int p, const SvGate1& g, hipStream_t s);
// out[2t], out[2t+1] = amplitude idx[t] (device arrays).
hipError_t sv_gather(const double* re, const double* im, const int64_t* idx, int64_t count, double* out,
                     hipStream_t s);
// sv_compare_blocks() x 5 partial sums: conj(p) q (re, im), |p|^2 |q|^2, |p|^2, |q|^2.
int sv_compare_blocks();
hipError_t sv_compare(const double* pr, const double* pi, const double* qr, const double* qi, uint64_t dim,
                      double* partials, hipStream_t s);

}  // namespace mpsk
