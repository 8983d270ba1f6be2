// Eigen-decomposition of a real symmetric tridiagonal matrix by divide and
// conquer, all on the device.
//
// The FP64 truncation of a two-site step (Sec. VI.A: keep the chi largest
// singular values) reduces its Gram matrix to a real tridiagonal T and needs
// all eigenvalues of T (the discarded weight is their sum beyond the kept
// ones) and the eigenvectors of the kept ones.  This solver replaces the
// library's divide and conquer; every step is a kernel of this file, so the
// host never waits on it.
//
// Tree.  Node (t, i) of depth t covers the rows [floor(i n / 2^t),
// floor((i + 1) n / 2^t)); its children are (t + 1, 2i) and (t + 1, 2i + 1).
// At depth ceil(log2 n) every node holds one row or none, so every boundary
// between rows c - 1 and c splits exactly one node.  With beta = e[c - 1],
//   T = diag(T1, T2) + |beta| w w^T,   w = e_{c-1} + sign(beta) e_c,
// where T1 and T2 have |beta| subtracted from their last and first diagonal
// entries; a leaf row i therefore starts from d[i] - |e[i-1]| - |e[i]| with
// eigenvector 1.  The levels are merged bottom-up, all merges of one depth in
// the same launches.
//
// Merge of the eigen-pairs (D1, Q1), (D2, Q2) of the children:
//   T = Q (D + rho z z^T) Q^T,  Q = diag(Q1, Q2),  rho = 2 |beta|,
//   z = (last row of Q1, sign(beta) first row of Q2) / sqrt(2)  (|z| = 1).
//   1. Sort D ascending (with z and the source columns).  Deflate: an entry
//      with rho |z_i| <= tol is an eigen-pair of the merged problem as it is;
//      of two neighbouring survivors whose Givens rotation, zeroing the first
//      one's z, leaves an off-diagonal |(d_j - d_i) c s| <= tol, the first is
//      deflated with the rotated value (tol = 8 eps max(|D|, rho)).
//   2. The K remaining roots of the secular equation
//        f(lambda) = 1 + rho sum_i z_i^2 / (d_i - lambda) = 0
//      lie one in each gap (d_j, d_{j+1}) and the last in (d_K, d_K + rho).
//      Each is found relative to its nearer pole d_o (lambda = d_o + tau) so
//      that every difference d_i - lambda = (d_i - d_o) - tau keeps its
//      relative accuracy: from the values and derivatives of the sums over
//      the poles below and above the gap, each iterate solves the model with
//      one pole on either side (a quadratic), safeguarded by bisection of the
//      bracket that the sign of f maintains.
//   3. The vector z is recomputed from the roots (Lowner's formula),
//        zhat_i^2 = prod_j (lambda_j - d_i) / (rho prod_{j != i} (d_j - d_i)),
//      so that the computed roots are exact eigenvalues of D + rho zhat
//      zhat^T and the eigenvectors u_j = (zhat_i / (d_i - lambda_j))_i,
//      normalised, are orthogonal to working accuracy.
//   4. The merged eigenvectors are Q u_j: one FP64 matrix-core GEMM per merge
//      (of the gathered, rotated columns of Q), the deflated columns copied.
// Finally the eigenvalues are sorted ascending with their vectors.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.h"

namespace mpsk {
namespace {

constexpr int DC_MAXN = 2048;
constexpr double DC_EPS = 1.1102230246251565e-16;   // 2^-53
constexpr int SEC_PER_LANE = DC_MAXN / 64;           // secular-equation entries held by one lane
constexpr int SEC_MAX_IT = 100;

struct DcArgs {
    int n;
    const double* e;   // n - 1 off-diagonal entries
    double* zw;        // n x n: eigenvectors of the current nodes (diagonal blocks), column-major
    double* qg;        // n x n: gathered (and rotated) columns of the current merges
    double* u;         // n x n: eigenvectors of D + rho zhat zhat^T of the current merges
    double* lam;       // n: eigenvalue of each column of zw
    double* dsrt;      // n: per merge at [a, b): surviving d ascending, then the deflated values
    double* zsrt;      // n: z of the survivors
    double* zhat;      // n
    double* rtau;      // n: root j of merge a: lambda = dsrt[a + rorig] + rtau
    double* rot_c;     // n: Givens rotations of merge a at [a, a + R)
    double* rot_s;
    double* rho;       // n: rho of merge a
    int* colsrc;       // n: source column of each position
    int* posof;        // n: position of each source column
    int* rorig;        // n
    int* rot_p;        // n: source columns of the rotations
    int* rot_q;
    int* kof;          // n: surviving count of merge a (-1: nothing to merge)
    int* rof;          // n: rotation count of merge a
    int* perm;         // n: final order
};

__device__ inline void node_range(int t, int i, int n, int& a, int& b) {
    a = (int)(((int64_t)i * n) >> t);
    b = (int)(((int64_t)(i + 1) * n) >> t);
}

// The node of depth t that holds row p: the largest i with floor(i n / 2^t) <= p.
__device__ inline int node_of(int t, int p, int n) {
    return (int)((((int64_t)(p + 1) << t) + n - 1) / n) - 1;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wave_prod(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v *= __shfl_xor(v, o);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Exclusive prefix sum over the 256 threads of a block; *total gets the sum.
__device__ int block_scan256(int v, int* tmp, int* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wid) off += tmp[w];
        tot += tmp[w];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(256) void dc_init_kernel(int n, const double* __restrict__ d, const double* __restrict__ e,
                                                      double* __restrict__ lam, double* __restrict__ zw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double el = i > 0 ? fabs(e[i - 1]) : 0.0, er = i < n - 1 ? fabs(e[i]) : 0.0;
    lam[i] = d[i] - el - er;
    zw[i + (int64_t)i * n] = 1.0;
}

// Step 1 of the merges of depth t: one workgroup per merge.
__global__ __launch_bounds__(256) void dc_scan_kernel(DcArgs g, int t) {
    const int n = g.n, tid = threadIdx.x;
    int a, b;
    node_range(t, blockIdx.x, n, a, b);
    if (b == a) return;                                     // an empty node owns nothing
    const int c = (int)(((int64_t)(2 * blockIdx.x + 1) * n) >> (t + 1));
    if (c == a || c == b) {                                 // one child: already in place
        if (tid == 0) g.kof[a] = -1;
        return;
    }
    const int m = b - a;
    const double beta = g.e[c - 1];
    const double rho = 2.0 * fabs(beta);
    const double sgn = beta >= 0.0 ? 1.0 : -1.0;

    __shared__ double sd[DC_MAXN], sz[DC_MAXN];
    __shared__ int sc[DC_MAXN], sl[DC_MAXN];
    __shared__ unsigned char typ[DC_MAXN];
    __shared__ int tmp[4];
    __shared__ double red[4];
    __shared__ int flag;

    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    for (int p = tid; p < P2; p += 256) {
        if (p < m) {
            const int col = a + p;
            sd[p] = g.lam[col];
            const double zr = col < c ? g.zw[(c - 1) + (int64_t)col * n] : sgn * g.zw[c + (int64_t)col * n];
            sz[p] = zr * 0.70710678118654752440;
            sc[p] = col;
        } else {
            sd[p] = __builtin_inf();
            sz[p] = 0.0;
            sc[p] = INT_MAX;
        }
    }
    __syncthreads();
    // bitonic sort by (d, source column)
    for (int k = 2; k <= P2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = tid; p < P2; p += 256) {
                const int q = p ^ j;
                if (q > p) {
                    const bool up = (p & k) == 0;
                    const bool gt = sd[p] > sd[q] || (sd[p] == sd[q] && sc[p] > sc[q]);
                    if (gt == up) {
                        const double td = sd[p], tz = sz[p];
                        const int tc = sc[p];
                        sd[p] = sd[q]; sz[p] = sz[q]; sc[p] = sc[q];
                        sd[q] = td; sz[q] = tz; sc[q] = tc;
                    }
                }
            }
            __syncthreads();
        }
    // tolerance
    double dm = 0.0;
    for (int p = tid; p < m; p += 256) dm = fmax(dm, fabs(sd[p]));
    dm = wave_max(dm);
    if ((tid & 63) == 0) red[tid >> 6] = dm;
    __syncthreads();
    const double tol = 8.0 * DC_EPS * fmax(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])), rho);

    // survivors of the small-z test, in order (each thread a contiguous chunk)
    const int CH = (m + 255) / 256;
    const int p0 = min(m, tid * CH), p1 = min(m, p0 + CH);
    int cnt = 0;
    for (int p = p0; p < p1; ++p) {
        const bool s = rho * fabs(sz[p]) > tol;
        typ[p] = s ? 1 : 0;
        cnt += s;
    }
    int S;
    int r = block_scan256(cnt, tmp, &S);
    for (int p = p0; p < p1; ++p)
        if (typ[p]) sl[r++] = p;
    if (tid == 0) flag = 0;
    __syncthreads();
    // does any pair of neighbouring survivors pass the rotation test?
    for (int k = 1 + tid; k < S; k += 256) {
        const int pi = sl[k - 1], pj = sl[k];
        const double s0 = sz[pi], c0 = sz[pj];
        const double tau = hypot(c0, s0);
        const double cc = c0 / tau, ss = -s0 / tau;
        if (fabs((sd[pj] - sd[pi]) * cc * ss) <= tol) flag = 1;
    }
    __syncthreads();
    int R = 0;
    if (flag) {
        // sequential deflation with rotations (rare: close eigenvalues with large z)
        if (tid == 0) {
            int pj = -1;
            for (int p = 0; p < m; ++p) {
                if (!typ[p]) continue;
                if (pj >= 0) {
                    double s0 = sz[pj], c0 = sz[p];
                    const double tau = hypot(c0, s0);
                    const double tt = sd[p] - sd[pj];
                    c0 /= tau;
                    s0 = -s0 / tau;
                    if (fabs(tt * c0 * s0) <= tol) {
                        sz[p] = tau;
                        sz[pj] = 0.0;
                        const double dpj = sd[pj] * c0 * c0 + sd[p] * s0 * s0;
                        sd[p] = sd[pj] * s0 * s0 + sd[p] * c0 * c0;
                        sd[pj] = dpj;
                        typ[pj] = 0;
                        g.rot_p[a + R] = sc[pj];
                        g.rot_q[a + R] = sc[p];
                        g.rot_c[a + R] = c0;
                        g.rot_s[a + R] = s0;
                        ++R;
                    }
                }
                pj = p;
            }
            tmp[0] = R;
        }
        __syncthreads();
        R = tmp[0];
        __syncthreads();
        cnt = 0;
        for (int p = p0; p < p1; ++p) cnt += typ[p];
    }
    int K;
    const int rs = block_scan256(cnt, tmp, &K);
    // scatter: survivors to [a, a + K), deflated to [a + K, b)
    int ks = rs, kd = p0 - rs;
    for (int p = p0; p < p1; ++p) {
        const int pos = typ[p] ? a + ks++ : a + K + kd++;
        g.dsrt[pos] = sd[p];
        g.zsrt[pos] = sz[p];
        g.colsrc[pos] = sc[p];
        g.posof[sc[p]] = pos;
        if (!typ[p]) g.lam[pos] = sd[p];
    }
    if (tid == 0) {
        g.kof[a] = K;
        g.rof[a] = R;
        g.rho[a] = rho;
    }
}

// Gathered columns of each merge: column pos of qg (rows [a, b)) is column
// colsrc[pos] of diag(Q1, Q2).  One workgroup per position.
__global__ __launch_bounds__(256) void dc_gather_kernel(DcArgs g, int t) {
    const int n = g.n, p = blockIdx.x;
    const int i = node_of(t, p, n);
    int a, b;
    node_range(t, i, n, a, b);
    if (g.kof[a] < 0) return;
    const int c = (int)(((int64_t)(2 * i + 1) * n) >> (t + 1));
    const int col = g.colsrc[p];
    const int lo = col < c ? a : c, hi = col < c ? c : b;
    const double* src = g.zw + (int64_t)col * n;
    double* dst = g.qg + (int64_t)p * n;
    for (int r = a + threadIdx.x; r < b; r += 256) dst[r] = (r >= lo && r < hi) ? src[r] : 0.0;
}

// The deflation rotations, in order, on the gathered columns: one thread per row.
__global__ __launch_bounds__(64) void dc_rotate_kernel(DcArgs g, int t) {
    const int n = g.n;
    int a, b;
    node_range(t, blockIdx.x, n, a, b);
    if (b == a || g.kof[a] < 0) return;
    const int R = g.rof[a];
    const int r = a + blockIdx.y * 64 + threadIdx.x;
    if (R == 0 || r >= b) return;
    for (int k = 0; k < R; ++k) {
        double* x = g.qg + r + (int64_t)g.posof[g.rot_p[a + k]] * n;
        double* y = g.qg + r + (int64_t)g.posof[g.rot_q[a + k]] * n;
        const double cc = g.rot_c[a + k], ss = g.rot_s[a + k];
        const double xv = *x, yv = *y;
        *x = cc * xv + ss * yv;
        *y = cc * yv - ss * xv;
    }
}

// Step 2: one wavefront per root.
__global__ __launch_bounds__(256) void dc_secular_kernel(DcArgs g, int t) {
    const int n = g.n, lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    int a, b;
    node_range(t, node_of(t, p, n), n, a, b);
    const int K = g.kof[a];
    const int j = p - a;
    if (K < 0 || j >= K) return;
    const double rho = g.rho[a];
    const double* d = g.dsrt + a;
    const double* z = g.zsrt + a;
    double dv[SEC_PER_LANE], wv[SEC_PER_LANE];
#pragma unroll
    for (int q = 0; q < SEC_PER_LANE; ++q) {
        const int i = lane + 64 * q;
        dv[q] = i < K ? d[i] : 0.0;
        wv[q] = i < K ? rho * z[i] * z[i] : 0.0;
    }
    // sums over the poles i <= j (psi) and i > j (phi) at lambda = d_o + tau
    auto eval = [&](int o, double tau, double& psi, double& dpsi, double& phi, double& dphi) {
        const double d_o = d[o];
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int q = 0; q < SEC_PER_LANE; ++q) {
            const int i = lane + 64 * q;
            if (i < K) {
                const double del = (dv[q] - d_o) - tau;
                const double tm = wv[q] / del;
                const double dt = tm / del;
                if (i <= j) { s0 += tm; s1 += dt; }
                else        { s2 += tm; s3 += dt; }
            }
        }
        psi = wave_sum(s0);
        dpsi = wave_sum(s1);
        phi = wave_sum(s2);
        dphi = wave_sum(s3);
    };
    int o;
    double lo, hi, psi, dpsi, phi, dphi;
    const bool last = j == K - 1;
    if (!last) {
        const double gap = d[j + 1] - d[j];
        eval(j, 0.5 * gap, psi, dpsi, phi, dphi);
        if (1.0 + psi + phi >= 0.0) { o = j;     lo = 0.0;        hi = 0.5 * gap; }
        else                        { o = j + 1; lo = -0.5 * gap; hi = 0.0; }
    } else {
        double wsum = 0;
#pragma unroll
        for (int q = 0; q < SEC_PER_LANE; ++q) wsum += wv[q];
        o = j;
        lo = 0.0;
        hi = wave_sum(wsum);
    }
    const double dl = d[j] - d[o];
    const double dr = last ? 0.0 : d[j + 1] - d[o];
    double tau = o == j ? hi : lo;
    for (int it = 0; it < SEC_MAX_IT; ++it) {
        eval(o, tau, psi, dpsi, phi, dphi);
        const double f = 1.0 + psi + phi;
        if (f < 0.0) lo = fmax(lo, tau);
        else         hi = fmin(hi, tau);
        if (fabs(f) <= 32.0 * DC_EPS * (1.0 + phi - psi) || hi - lo <= 4.0 * DC_EPS * fmax(fabs(lo), fabs(hi))) break;
        const double A = dl - tau;
        const double qq = dpsi * A * A;
        const double pp = psi - dpsi * A;
        double eta;
        if (!last) {
            const double B = dr - tau;
            const double ss = dphi * B * B;
            const double rr = phi - dphi * B;
            const double c0 = 1.0 + pp + rr;
            const double bb = c0 * (A + B) + qq + ss;
            const double cc = A * B * f;
            const double disc = fmax(bb * bb - 4.0 * c0 * cc, 0.0);
            const double den = bb + copysign(sqrt(disc), bb);
            eta = den != 0.0 ? 2.0 * cc / den : 0.0;
        } else {
            const double c0 = 1.0 + pp;
            eta = c0 != 0.0 ? A + qq / c0 : 0.0;
        }
        if (fabs(eta) <= 2.0 * DC_EPS * fabs(tau)) break;
        double nt = tau + eta;
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        tau = nt;
    }
    if (lane == 0) {
        g.rorig[a + j] = o;
        g.rtau[a + j] = tau;
        g.lam[a + j] = d[o] + tau;
    }
}

// Step 3: zhat_i, one wavefront per survivor i.
__global__ __launch_bounds__(256) void dc_zhat_kernel(DcArgs g, int t) {
    const int n = g.n, lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    int a, b;
    node_range(t, node_of(t, p, n), n, a, b);
    const int K = g.kof[a];
    const int i = p - a;
    if (K < 0 || i >= K) return;
    const double rho = g.rho[a];
    const double* d = g.dsrt + a;
    const double di = d[i];
    double v = 1.0;
    for (int j = lane; j < K; j += 64) {
        const double lm = (d[g.rorig[a + j]] - di) + g.rtau[a + j];   // lambda_j - d_i
        double den;
        if (j == K - 1)  den = rho;
        else if (j < i)  den = d[j] - di;
        else             den = d[j + 1] - di;
        v *= lm / den;
    }
    v = wave_prod(v);
    if (lane == 0) g.zhat[a + i] = copysign(sqrt(fmax(v, 0.0)), g.zsrt[a + i]);
}

// Step 3: u_j = (zhat_i / (d_i - lambda_j))_i normalised, one wavefront per root j.
__global__ __launch_bounds__(256) void dc_ucols_kernel(DcArgs g, int t) {
    const int n = g.n, lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    int a, b;
    node_range(t, node_of(t, p, n), n, a, b);
    const int K = g.kof[a];
    const int j = p - a;
    if (K < 0 || j >= K) return;
    const double* d = g.dsrt + a;
    const double d_o = d[g.rorig[a + j]], tau = g.rtau[a + j];
    double uv[SEC_PER_LANE];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < SEC_PER_LANE; ++q) {
        const int i = lane + 64 * q;
        uv[q] = 0.0;
        if (i < K) {
            uv[q] = g.zhat[a + i] / ((d[i] - d_o) - tau);
            s += uv[q] * uv[q];
        }
    }
    const double inv = 1.0 / sqrt(wave_sum(s));
    double* col = g.u + a + (int64_t)(a + j) * n;
#pragma unroll
    for (int q = 0; q < SEC_PER_LANE; ++q) {
        const int i = lane + 64 * q;
        if (i < K) col[i] = uv[q] * inv;
    }
}

// Step 4: zw[a:b, a:a+K] = qg[a:b, a:a+K] u[a:a+K, a:a+K] and the deflated
// columns zw[a:b, a+K:b] = qg[a:b, a+K:b], one 64 x 64 tile per workgroup
// (blockIdx.z = merge).  v_mfma_f64_16x16x4f64 computes the transposed tile
// (u^T qg^T) so that a lane's accumulator elements run down a column.
constexpr int GT = 64, GK = 16;
__global__ __launch_bounds__(256) void dc_gemm_kernel(DcArgs g, int t) {
    const int n = g.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int a, b;
    node_range(t, blockIdx.z, n, a, b);
    const int m = b - a;
    if (m == 0) return;
    const int K = g.kof[a];
    if (K < 0) return;
    const int r0 = blockIdx.x * GT, c0 = blockIdx.y * GT;
    if (r0 >= m || c0 >= m) return;
    const double* qg = g.qg + a + (int64_t)a * n;
    const double* u = g.u + a + (int64_t)a * n;
    double* zw = g.zw + a + (int64_t)a * n;
    if (c0 >= K) {
        for (int idx = tid; idx < GT * GT; idx += 256) {
            const int r = r0 + (idx & (GT - 1)), cc = c0 + idx / GT;
            if (r < m && cc < m) zw[r + (int64_t)cc * n] = qg[r + (int64_t)cc * n];
        }
        return;
    }
    __shared__ double As[2][GK][GT + 2];   // As[k][r] = qg(r0 + r, k0 + k)
    __shared__ double Bs[2][GK][GT + 2];   // Bs[k][c] = u(k0 + k, c0 + c)
    double ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            const int r = idx & (GT - 1), k = idx / GT;            // along r: coalesced
            ra[q] = (r0 + r < m && k0 + k < K) ? qg[(r0 + r) + (int64_t)(k0 + k) * n] : 0.0;
            const int kb = idx & (GK - 1), cb = idx / GK;          // along k: coalesced
            rb[q] = (k0 + kb < K && c0 + cb < K) ? u[(k0 + kb) + (int64_t)(c0 + cb) * n] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            As[buf][idx / GT][idx & (GT - 1)] = ra[q];
            Bs[buf][idx & (GK - 1)][idx / GK] = rb[q];
        }
    };
    typedef double acc_t __attribute__((ext_vector_type(4)));
    acc_t acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = acc_t{0.0, 0.0, 0.0, 0.0};
    const int wr0 = (wave >> 1) * 32, wc0 = (wave & 1) * 32;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int nk = (K + GK - 1) / GK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = As[buf][kk + l4][wr0 + 16 * x + l16];
#pragma unroll
            for (int y = 0; y < 2; ++y) bv[y] = Bs[buf][kk + l4][wc0 + 16 * y + l16];
            // D'[c][r] += sum_k u(k, c) qg(r, k): the first operand indexes the accumulator rows
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], av[x], acc[x][y], 0, 0, 0);
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + wr0 + 16 * x + l16;
                const int cc = c0 + wc0 + 16 * y + 4 * v + l4;
                if (r < m && cc < m) zw[r + (int64_t)cc * n] = cc < K ? acc[x][y][v] : qg[r + (int64_t)cc * n];
            }
}

// Merges of at most SMALL_M rows: every step of a merge in one workgroup, on LDS copies (the
// steps are those of the kernels above; one launch per depth instead of seven).
constexpr int SMALL_M = 64;

// Root j of 1 + sum_i w_i / (d_i - lambda) (w_i = rho z_i^2 > 0, d ascending, K terms in LDS) by
// one thread: the nearer pole o and tau with lambda = d_o + tau, as in dc_secular_kernel.
__device__ void secular_root_serial(const double* d, const double* w, int K, int j, int& o_out, double& tau_out) {
    auto eval = [&](int o, double tau, double& psi, double& dpsi, double& phi, double& dphi) {
        const double d_o = d[o];
        psi = dpsi = phi = dphi = 0.0;
        for (int i = 0; i < K; ++i) {
            const double del = (d[i] - d_o) - tau;
            const double tm = w[i] / del;
            const double dt = tm / del;
            if (i <= j) { psi += tm; dpsi += dt; }
            else        { phi += tm; dphi += dt; }
        }
    };
    int o;
    double lo, hi, psi, dpsi, phi, dphi;
    const bool last = j == K - 1;
    if (!last) {
        const double gap = d[j + 1] - d[j];
        eval(j, 0.5 * gap, psi, dpsi, phi, dphi);
        if (1.0 + psi + phi >= 0.0) { o = j;     lo = 0.0;        hi = 0.5 * gap; }
        else                        { o = j + 1; lo = -0.5 * gap; hi = 0.0; }
    } else {
        double ws = 0.0;
        for (int i = 0; i < K; ++i) ws += w[i];
        o = j;
        lo = 0.0;
        hi = ws;
    }
    const double dl = d[j] - d[o];
    const double dr = last ? 0.0 : d[j + 1] - d[o];
    double tau = o == j ? hi : lo;
    for (int it = 0; it < SEC_MAX_IT; ++it) {
        eval(o, tau, psi, dpsi, phi, dphi);
        const double f = 1.0 + psi + phi;
        if (f < 0.0) lo = fmax(lo, tau);
        else         hi = fmin(hi, tau);
        if (fabs(f) <= 32.0 * DC_EPS * (1.0 + phi - psi) || hi - lo <= 4.0 * DC_EPS * fmax(fabs(lo), fabs(hi))) break;
        const double A = dl - tau;
        const double qq = dpsi * A * A;
        const double pp = psi - dpsi * A;
        double eta;
        if (!last) {
            const double B = dr - tau;
            const double ss = dphi * B * B;
            const double rr = phi - dphi * B;
            const double c0 = 1.0 + pp + rr;
            const double bb = c0 * (A + B) + qq + ss;
            const double cc = A * B * f;
            const double disc = fmax(bb * bb - 4.0 * c0 * cc, 0.0);
            const double den = bb + copysign(sqrt(disc), bb);
            eta = den != 0.0 ? 2.0 * cc / den : 0.0;
        } else {
            const double c0 = 1.0 + pp;
            eta = c0 != 0.0 ? A + qq / c0 : 0.0;
        }
        if (fabs(eta) <= 2.0 * DC_EPS * fabs(tau)) break;
        double nt = tau + eta;
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        tau = nt;
    }
    o_out = o;
    tau_out = tau;
}

__global__ __launch_bounds__(256) void dc_small_merge_kernel(DcArgs g, int t) {
    const int n = g.n, tid = threadIdx.x;
    int a, b;
    node_range(t, blockIdx.x, n, a, b);
    if (b == a) return;
    const int c = (int)(((int64_t)(2 * blockIdx.x + 1) * n) >> (t + 1));
    if (c == a || c == b) return;                          // one child: already in place
    const int m = b - a;                                   // <= SMALL_M
    const double beta = g.e[c - 1];
    const double rho = 2.0 * fabs(beta);
    const double sgn = beta >= 0.0 ? 1.0 : -1.0;

    __shared__ double sd[SMALL_M], sz[SMALL_M], sw[SMALL_M], zh[SMALL_M], rt[SMALL_M];
    __shared__ int sc[SMALL_M], ro[SMALL_M], pos_of[SMALL_M], nd[SMALL_M];
    __shared__ unsigned char typ[SMALL_M];
    __shared__ double qg[SMALL_M][SMALL_M + 1];          // gathered columns, then rotated
    __shared__ double uu[SMALL_M][SMALL_M + 1];          // uu[i][j] = u_j[i]
    __shared__ double rot_c[SMALL_M], rot_s[SMALL_M];
    __shared__ int rot_p[SMALL_M], rot_q[SMALL_M];
    __shared__ int sh_K, sh_R;
    __shared__ double sh_tol;

    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    // 1. sort (d, z, source column) ascending by d
    if (tid < P2) {
        if (tid < m) {
            const int col = a + tid;
            sd[tid] = g.lam[col];
            const double zr = col < c ? g.zw[(c - 1) + (int64_t)col * n] : sgn * g.zw[c + (int64_t)col * n];
            sz[tid] = zr * 0.70710678118654752440;
            sc[tid] = col;
        } else {
            sd[tid] = __builtin_inf();
            sz[tid] = 0.0;
            sc[tid] = INT_MAX;
        }
    }
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (tid < P2) {
                const int q = tid ^ j;
                if (q > tid) {
                    const bool up = (tid & k) == 0;
                    const bool gt = sd[tid] > sd[q] || (sd[tid] == sd[q] && sc[tid] > sc[q]);
                    if (gt == up) {
                        const double td = sd[tid], tz = sz[tid];
                        const int tc = sc[tid];
                        sd[tid] = sd[q]; sz[tid] = sz[q]; sc[tid] = sc[q];
                        sd[q] = td; sz[q] = tz; sc[q] = tc;
                    }
                }
            }
            __syncthreads();
        }
    // 2. deflation (one thread: at most SMALL_M entries), positions: survivors first
    if (tid == 0) {
        double dm = 0.0;
        for (int p = 0; p < m; ++p) dm = fmax(dm, fabs(sd[p]));
        const double tol = 8.0 * DC_EPS * fmax(dm, rho);
        int R = 0, pj = -1;
        for (int p = 0; p < m; ++p) {
            typ[p] = rho * fabs(sz[p]) > tol ? 1 : 0;
            if (!typ[p]) continue;
            if (pj >= 0) {
                double s0 = sz[pj], c0 = sz[p];
                const double tau = hypot(c0, s0);
                const double tt = sd[p] - sd[pj];
                c0 /= tau;
                s0 = -s0 / tau;
                if (fabs(tt * c0 * s0) <= tol) {
                    sz[p] = tau;
                    sz[pj] = 0.0;
                    const double dpj = sd[pj] * c0 * c0 + sd[p] * s0 * s0;
                    sd[p] = sd[pj] * s0 * s0 + sd[p] * c0 * c0;
                    sd[pj] = dpj;
                    typ[pj] = 0;
                    rot_p[R] = pj;
                    rot_q[R] = p;
                    rot_c[R] = c0;
                    rot_s[R] = s0;
                    ++R;
                }
            }
            pj = p;
        }
        int K = 0;
        for (int p = 0; p < m; ++p)
            if (typ[p]) nd[K++] = p;
        int q = K;
        for (int p = 0; p < m; ++p)
            if (!typ[p]) nd[q++] = p;                  // deflated after the survivors
        for (int i = 0; i < m; ++i) pos_of[nd[i]] = i;
        sh_K = K;
        sh_R = R;
        sh_tol = tol;
    }
    __syncthreads();
    const int K = sh_K, R = sh_R;
    // 3. gathered columns in sorted order (explicit zeros off the children's blocks), then the
    //    rotations in order; qg[r][p] is row a + r of sorted entry p's column
    for (int idx = tid; idx < m * m; idx += 256) {
        const int r = idx % m, p = idx / m;
        const int col = sc[p];
        const int lo = col < c ? a : c, hi = col < c ? c : b;
        const int row = a + r;
        qg[r][p] = (row >= lo && row < hi) ? g.zw[row + (int64_t)col * n] : 0.0;
    }
    __syncthreads();
    if (tid < m)
        for (int k = 0; k < R; ++k) {
            const double xv = qg[tid][rot_p[k]], yv = qg[tid][rot_q[k]];
            qg[tid][rot_p[k]] = rot_c[k] * xv + rot_s[k] * yv;
            qg[tid][rot_q[k]] = rot_c[k] * yv - rot_s[k] * xv;
        }
    // survivors' d and w = rho z^2 in nd order
    if (tid < K) {
        const int p = nd[tid];
        rt[tid] = sd[p];
        sw[tid] = rho * sz[p] * sz[p];
        zh[tid] = sz[p];                               // sign of z for the Lowner vector
    }
    __syncthreads();
    // 4. roots (one thread each); rt holds d of the survivors, keep it: roots in zh/ro below
    __shared__ double dsv[SMALL_M], tauv[SMALL_M];
    if (tid < K) dsv[tid] = rt[tid];
    __syncthreads();
    if (tid < K) {
        int o;
        double tau;
        secular_root_serial(dsv, sw, K, tid, o, tau);
        ro[tid] = o;
        tauv[tid] = tau;
        g.lam[a + tid] = dsv[o] + tau;
    }
    if (tid >= K && tid < m) g.lam[a + tid] = sd[nd[tid]];
    __syncthreads();
    // 5. Lowner's update vector
    if (tid < K) {
        const int i = tid;
        const double di = dsv[i];
        double v = 1.0;
        for (int j = 0; j < K; ++j) {
            const double lm = (dsv[ro[j]] - di) + tauv[j];
            double den;
            if (j == K - 1)  den = rho;
            else if (j < i)  den = dsv[j] - di;
            else             den = dsv[j + 1] - di;
            v *= lm / den;
        }
        rt[i] = copysign(sqrt(fmax(v, 0.0)), zh[i]);   // zhat
    }
    __syncthreads();
    // 6. eigenvectors of D + rho zhat zhat^T
    if (tid < K) {
        const int j = tid;
        const double d_o = dsv[ro[j]], tau = tauv[j];
        double s2 = 0.0;
        for (int i = 0; i < K; ++i) {
            const double u = rt[i] / ((dsv[i] - d_o) - tau);
            uu[i][j] = u;
            s2 += u * u;
        }
        const double inv = 1.0 / sqrt(s2);
        for (int i = 0; i < K; ++i) uu[i][j] *= inv;
    }
    __syncthreads();
    // 7. merged vectors: column j < K = sum_i qg[:, nd[i]] u_j[i]; deflated columns copied
    for (int idx = tid; idx < m * m; idx += 256) {
        const int r = idx % m, j = idx / m;
        double v;
        if (j < K) {
            v = 0.0;
            for (int i = 0; i < K; ++i) v += qg[r][nd[i]] * uu[i][j];
        } else {
            v = qg[r][nd[j]];
        }
        g.zw[(a + r) + (int64_t)(a + j) * n] = v;
    }
}

// Final order: eigenvalues ascending (ties by column), one workgroup.
__global__ __launch_bounds__(1024) void dc_sort_kernel(DcArgs g, double* __restrict__ w) {
    const int n = g.n, tid = threadIdx.x;
    __shared__ double sd[DC_MAXN];
    __shared__ int sc[DC_MAXN];
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int p = tid; p < P2; p += 1024) {
        sd[p] = p < n ? g.lam[p] : __builtin_inf();
        sc[p] = p < n ? p : INT_MAX;
    }
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = tid; p < P2; p += 1024) {
                const int q = p ^ j;
                if (q > p) {
                    const bool up = (p & k) == 0;
                    const bool gt = sd[p] > sd[q] || (sd[p] == sd[q] && sc[p] > sc[q]);
                    if (gt == up) {
                        const double td = sd[p];
                        const int tc = sc[p];
                        sd[p] = sd[q]; sc[p] = sc[q];
                        sd[q] = td; sc[q] = tc;
                    }
                }
            }
            __syncthreads();
        }
    for (int p = tid; p < n; p += 1024) {
        w[p] = sd[p];
        g.perm[p] = sc[p];
    }
}

__global__ __launch_bounds__(256) void dc_out_kernel(DcArgs g, double* __restrict__ z, int ldz) {
    const int n = g.n, p = blockIdx.x;
    const double* src = g.zw + (int64_t)g.perm[p] * n;
    double* dst = z + (int64_t)p * ldz;
    for (int r = threadIdx.x; r < n; r += 256) dst[r] = src[r];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int stedc_dc_max_n() { return DC_MAXN; }

size_t stedc_dc_workspace_bytes(int n) {
    if (n < 1) return 0;
    return 3 * align256(sizeof(double) * (size_t)n * n) + 10 * align256(sizeof(double) * n) +
           10 * align256(sizeof(int) * n);
}

hipError_t stedc_dc(int n, double* d, const double* e, double* z, int ldz, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
    if (n < 1 || n > DC_MAXN || ldz < n || ws_bytes < stedc_dc_workspace_bytes(n)) return hipErrorInvalidValue;
    char* p = (char*)ws;
    auto take = [&](size_t bytes) {
        char* q = p;
        p += align256(bytes);
        return q;
    };
    DcArgs g;
    g.n = n;
    g.e = e;
    g.zw = (double*)take(sizeof(double) * (size_t)n * n);
    g.qg = (double*)take(sizeof(double) * (size_t)n * n);
    g.u = (double*)take(sizeof(double) * (size_t)n * n);
    g.lam = (double*)take(sizeof(double) * n);
    g.dsrt = (double*)take(sizeof(double) * n);
    g.zsrt = (double*)take(sizeof(double) * n);
    g.zhat = (double*)take(sizeof(double) * n);
    g.rtau = (double*)take(sizeof(double) * n);
    g.rot_c = (double*)take(sizeof(double) * n);
    g.rot_s = (double*)take(sizeof(double) * n);
    g.rho = (double*)take(sizeof(double) * n);
    take(sizeof(double) * n);
    take(sizeof(double) * n);
    g.colsrc = (int*)take(sizeof(int) * n);
    g.posof = (int*)take(sizeof(int) * n);
    g.rorig = (int*)take(sizeof(int) * n);
    g.rot_p = (int*)take(sizeof(int) * n);
    g.rot_q = (int*)take(sizeof(int) * n);
    g.kof = (int*)take(sizeof(int) * n);
    g.rof = (int*)take(sizeof(int) * n);
    g.perm = (int*)take(sizeof(int) * n);
    hipLaunchKernelGGL(dc_init_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, d, e, g.lam, g.zw);
    int L = 0;
    while ((1 << L) < n) ++L;
    for (int t = L - 1; t >= 0; --t) {
        const int merges = 1 << t;
        const int mmax = (n + merges - 1) / merges;
        const int tiles = (mmax + GT - 1) / GT;
        if (mmax <= SMALL_M) {
            hipLaunchKernelGGL(dc_small_merge_kernel, dim3(merges), dim3(256), 0, stream, g, t);
            continue;
        }
        hipLaunchKernelGGL(dc_scan_kernel, dim3(merges), dim3(256), 0, stream, g, t);
        hipLaunchKernelGGL(dc_gather_kernel, dim3(n), dim3(256), 0, stream, g, t);
        hipLaunchKernelGGL(dc_rotate_kernel, dim3(merges, (mmax + 63) / 64), dim3(64), 0, stream, g, t);
        hipLaunchKernelGGL(dc_secular_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, g, t);
        hipLaunchKernelGGL(dc_zhat_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, g, t);
        hipLaunchKernelGGL(dc_ucols_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, g, t);
        hipLaunchKernelGGL(dc_gemm_kernel, dim3(tiles, tiles, merges), dim3(256), 0, stream, g, t);
    }
    hipLaunchKernelGGL(dc_sort_kernel, dim3(1), dim3(1024), 0, stream, g, d);
    hipLaunchKernelGGL(dc_out_kernel, dim3(n), dim3(256), 0, stream, g, z, ldz);
    return hipGetLastError();
}

}  // namespace mpsk
