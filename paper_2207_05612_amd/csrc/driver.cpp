// Host driver of the DMRG compression step: the C ABI of include/mps_dmrg.h.
//
// One compression step (Sec. IV.B of Ayral et al.) on one GPU:
//   1. the layer becomes a structured MPO on the host (one-qubit gates
//      absorbed, two-qubit gates split by a 4x4 SVD, eq:SVD / App. A.1);
//   2. zip-up initial guess (the TEBD-like start of Sec. V.D.1) from the end
//      of the chain that holds the orthogonality centre;
//   3. n_sweeps two-site sweeps in alternating directions; each step builds
//      the local tensor F of the pair in the vertical contraction order of
//      Sec. IV.B.2, keeps the chi largest singular values (Sec. VI.A) and
//      normalises (eq:optimization);
//   4. f_delta, the f of the last step, multiplies into F~ (eq:Ftilde-sup).
//
// Every pass is executed as a left-to-right pass over a "view" of the chain:
// view 0 is the chain itself, view 1 the mirrored chain (site j of view 1 is
// site n-1-j, and its tensors have their two virtual legs swapped).  The
// environments are stored per bond of the chain, so the left environments
// written by a pass in one view are exactly the right environments read by
// the next pass in the other view.  Only one kernel pipeline is needed.
//
// Contractions run in the state's working precision (FP32 or FP64 complex
// MFMA GEMMs).  The truncation is FP64: the Gram matrix of the local tensor
// (FP64 MFMA), rocSOLVER's Hermitian eigensolver, and the kept-weight sums.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <array>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mps_dmrg.h"
#include "internal.h"

using namespace mpsk;
typedef std::complex<double> cd;

namespace {

thread_local std::string g_last_error;

struct MpsFail {
    mps_status code;
    std::string msg;
};

[[noreturn]] void fail(mps_status code, const std::string& msg) { throw MpsFail{code, msg}; }

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            fail(e_ == hipErrorOutOfMemory ? MPS_ERR_OOM : MPS_ERR_DEVICE,                    \
                 std::string(#expr) + ": " + hipGetErrorString(e_));                          \
    } while (0)

constexpr double EPS_TRUNC = 1e-12;        // kept: S^2 > EPS_TRUNC * sum S^2
constexpr double GATE_RANK_CUTOFF = 1e-14; // operator-Schmidt terms kept: sigma > cutoff * sigma_0

// ------------------------------------------------------------ device memory
// Allocator of the state the current call works on (NULL: hipMallocAsync on the
// call's stream).  Set by check_state() and mps_create(), reset by run_guarded().
thread_local const mps_allocator* g_alloc = nullptr;

void* dalloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (g_alloc) {
        p = g_alloc->alloc(bytes, (void*)s, g_alloc->user);
        if (!p) fail(MPS_ERR_OOM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
        if ((uintptr_t)p % 256 != 0) {
            g_alloc->free(p, (void*)s, g_alloc->user);
            fail(MPS_ERR_ARG, "allocator callback returned memory that is not 256-byte aligned");
        }
        return p;
    }
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        fail(MPS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}
void dfree(void* p, hipStream_t s, const mps_allocator* al) {
    if (!p) return;
    if (al)
        al->free(p, (void*)s, al->user);
    else
        (void)hipFreeAsync(p, s);
}

// Planar complex buffer: re = p, im = p + cap.  It is released through the
// allocator it was obtained from.
template <typename T>
struct Planar {
    T* p = nullptr;
    int64_t cap = 0;
    const mps_allocator* al = nullptr;
    T* re() const { return p; }
    T* im() const { return p + cap; }
    void ensure(int64_t n, hipStream_t s) {
        if (n <= cap && p) return;
        release(s);
        // capacity rounded to 64 elements keeps the imaginary plane 256-byte aligned
        const int64_t c = (std::max<int64_t>(n, 1) + 63) / 64 * 64;
        p = (T*)dalloc(sizeof(T) * 2 * (size_t)c, s);
        al = g_alloc;
        cap = c;
    }
    void release(hipStream_t s) {
        dfree(p, s, al);
        p = nullptr;
        cap = 0;
        al = nullptr;
    }
};

template <typename T>
struct Raw {
    T* p = nullptr;
    int64_t cap = 0;
    const mps_allocator* al = nullptr;
    void ensure(int64_t n, hipStream_t s) {
        if (n <= cap && p) return;
        release(s);
        p = (T*)dalloc(sizeof(T) * (size_t)std::max<int64_t>(n, 1), s);
        al = g_alloc;
        cap = std::max<int64_t>(n, 1);
    }
    void release(hipStream_t s) {
        dfree(p, s, al);
        p = nullptr;
        cap = 0;
        al = nullptr;
    }
};

// ------------------------------------------------------------ profiling ----
struct KStat {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
};
struct PendingTiming {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
};

// ------------------------------------------------------- 4x4 complex SVD ---
// One-sided Jacobi (Hestenes): rotate the columns of m until they are
// mutually orthogonal; singular values are the column norms.
void svd4(const cd m_in[4][4], double sigma[4], cd u[4][4], cd v[4][4]) {
    cd a[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            a[i][j] = m_in[i][j];
            v[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                double al = 0, be = 0;
                cd ga = 0;
                for (int i = 0; i < 4; ++i) {
                    al += std::norm(a[i][p]);
                    be += std::norm(a[i][q]);
                    ga += std::conj(a[i][p]) * a[i][q];
                }
                const double ag = std::abs(ga);
                if (ag == 0.0 || ag <= 1e-17 * std::sqrt(al * be)) continue;
                off = std::max(off, ag / std::sqrt(al * be));
                const cd ph = ga / ag;  // e^{i phi}
                const double zeta = (be - al) / (2.0 * ag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                const cd phc = std::conj(ph);
                for (int i = 0; i < 4; ++i) {
                    const cd xp = a[i][p], xq = a[i][q];
                    a[i][p] = c * xp - s * phc * xq;
                    a[i][q] = s * xp + c * phc * xq;
                    const cd vp = v[i][p], vq = v[i][q];
                    v[i][p] = c * vp - s * phc * vq;
                    v[i][q] = s * vp + c * phc * vq;
                }
            }
        if (off < 1e-16) break;
    }
    double nrm[4];
    int order[4] = {0, 1, 2, 3};
    for (int j = 0; j < 4; ++j) {
        nrm[j] = 0;
        for (int i = 0; i < 4; ++i) nrm[j] += std::norm(a[i][j]);
        nrm[j] = std::sqrt(nrm[j]);
    }
    std::sort(order, order + 4, [&](int x, int y) { return nrm[x] > nrm[y]; });
    cd vv[4][4];
    for (int jj = 0; jj < 4; ++jj) {
        const int j = order[jj];
        sigma[jj] = nrm[j];
        for (int i = 0; i < 4; ++i) {
            u[i][jj] = nrm[j] > 0 ? a[i][j] / nrm[j] : cd(0);
            vv[i][jj] = v[i][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) v[i][j] = vv[i][j];
}

// ------------------------------------------------------------ layer MPO ----
struct HostGate {
    int i, j, r, layer;
    cd x[4][2][2], y[4][2][2];  // [a][s][t]
};

// The MPO of one compression step: K layers applied in order.  Bond c carries
// the mixed-radix index of the operator-Schmidt indices of every two-qubit gate
// (of any of the K layers) with i < c <= j; the digits are ordered by (i, layer),
// the smallest being the most significant.  At each site the K layers act one
// after the other on the physical leg, each on its own gate's digit; view[o][j]
// lists those factors in the order they are applied (one-qubit factors are
// folded into a neighbouring factor, so a site has max(1, #gates at it) of them).
struct LayerMpo {
    std::vector<int64_t> w;                        // n + 1 bond dims
    std::vector<std::vector<MpoSiteOp>> view[2];   // per view-site
    int n_2q = 0;
};

void mul2(const cd a[2][2], const cd b[2][2], cd out[2][2]) {
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) out[s][t] = a[s][0] * b[0][t] + a[s][1] * b[1][t];
}

void set_op(MpoSiteOp& op, int r_in, int r_out, int lo, int64_t H, const cd (*ops)[2][2]) {
    op.r_in = r_in;
    op.r_out = r_out;
    op.lo = lo;
    op.H = (int)H;
    op.out_ws = 0;
    for (int i = 0; i < 16; ++i) op.re[i] = op.im[i] = 0;
    const int r = std::max(r_in, r_out);
    for (int a = 0; a < r; ++a)
        for (int s = 0; s < 2; ++s)
            for (int t = 0; t < 2; ++t) {
                const int ao = (r_out > 1) ? a : 0, ai = (r_in > 1) ? a : 0;
                const int c = ((ao * r_in + ai) * 2 + s) * 2 + t;
                op.re[c] = ops[a][s][t].real();
                op.im[c] = ops[a][s][t].imag();
            }
}

// One factor before it is folded: the gate's digit goes from r_in to r_out values.
struct ProtoOp {
    int r_in, r_out;
    int64_t lo, H;
    cd m[4][2][2];
};

// Fold the one-qubit factors (r_in = r_out = 1 on an absent digit) into their
// neighbours and turn the rest into MpoSiteOps; all but the last write the
// intermediate layout.
std::vector<MpoSiteOp> fold_site_ops(const std::vector<ProtoOp>& seq, const std::vector<bool>& is_1q, int64_t w_in) {
    std::vector<ProtoOp> out;
    cd pre[2][2] = {{1, 0}, {0, 1}};
    for (size_t q = 0; q < seq.size(); ++q) {
        if (is_1q[q]) {
            cd tmp[2][2];
            if (out.empty()) {                       // acts before the first gate factor
                mul2(seq[q].m[0], pre, tmp);
                std::memcpy(pre, tmp, sizeof(tmp));
            } else {                                 // acts after the last one
                ProtoOp& b = out.back();
                for (int a = 0; a < std::max(b.r_in, b.r_out); ++a) {
                    mul2(seq[q].m[0], b.m[a], tmp);
                    std::memcpy(b.m[a], tmp, sizeof(tmp));
                }
            }
            continue;
        }
        ProtoOp g = seq[q];
        if (out.empty())
            for (int a = 0; a < std::max(g.r_in, g.r_out); ++a) {
                cd tmp[2][2];
                mul2(g.m[a], pre, tmp);
                std::memcpy(g.m[a], tmp, sizeof(tmp));
            }
        out.push_back(g);
    }
    if (out.empty()) {
        ProtoOp g;
        g.r_in = g.r_out = 1;
        g.lo = 1;
        g.H = w_in;
        std::memcpy(g.m[0], pre, sizeof(pre));
        out.push_back(g);
    }
    std::vector<MpoSiteOp> ops(out.size());
    for (size_t q = 0; q < out.size(); ++q) {
        set_op(ops[q], out[q].r_in, out[q].r_out, (int)out[q].lo, out[q].H, out[q].m);
        ops[q].out_ws = q + 1 < out.size() ? 1 : 0;
    }
    return ops;
}

// Gates of K consecutive layers (n_gates[l] records each, concatenated) -> MPO.
LayerMpo build_step_mpo(int n, const mps_gate* gates, const int* n_gates, int K) {
    if (K < 1) fail(MPS_ERR_ARG, "a step needs at least one layer");
    std::vector<cd> g1m(4 * (size_t)n * K);
    auto G1 = [&](int l, int k, int s, int t) -> cd& { return g1m[((size_t)l * n + k) * 4 + s * 2 + t]; };
    std::vector<HostGate> hg;
    std::vector<int> at(static_cast<size_t>(n) * K, -1);   // [layer][site] -> index into hg
    int64_t off = 0;
    for (int l = 0; l < K; ++l) {
        if (n_gates[l] < 0) fail(MPS_ERR_ARG, "negative gate count");
        for (int k = 0; k < n; ++k) {
            G1(l, k, 0, 0) = 1; G1(l, k, 0, 1) = 0; G1(l, k, 1, 0) = 0; G1(l, k, 1, 1) = 1;
        }
        const size_t first = hg.size();
        for (int gi = 0; gi < n_gates[l]; ++gi) {
            const mps_gate& g = gates[off + gi];
            for (int e = 0; e < 32; ++e)
                if (!std::isfinite(g.m[e])) fail(MPS_ERR_ARG, "gate matrix has a non-finite entry");
            if (g.q1 < 0) {
                if (g.q1 != -1 || g.q0 < 0 || g.q0 >= n) fail(MPS_ERR_ARG, "one-qubit gate site out of range");
                cd u[2][2], cur[2][2], out[2][2];
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        u[s][t] = cd(g.m[2 * (s * 2 + t)], g.m[2 * (s * 2 + t) + 1]);
                        cur[s][t] = G1(l, g.q0, s, t);
                    }
                mul2(u, cur, out);
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) G1(l, g.q0, s, t) = out[s][t];
                continue;
            }
            if (g.q0 < 0 || g.q0 >= n || g.q1 >= n || g.q0 == g.q1)
                fail(MPS_ERR_ARG, "two-qubit gate sites out of range or equal");
            if (at[(size_t)l * n + g.q0] >= 0 || at[(size_t)l * n + g.q1] >= 0)
                fail(MPS_ERR_ARG, "two-qubit gates of one layer must be disjoint");
            // U[(s0 s1), (t0 t1)] -> Ut[(s_i t_i), (s_j t_j)] with i = min site
            cd u4[2][2][2][2];
            for (int s0 = 0; s0 < 2; ++s0)
                for (int s1 = 0; s1 < 2; ++s1)
                    for (int t0 = 0; t0 < 2; ++t0)
                        for (int t1 = 0; t1 < 2; ++t1) {
                            const int e = (s0 * 2 + s1) * 4 + (t0 * 2 + t1);
                            u4[s0][s1][t0][t1] = cd(g.m[2 * e], g.m[2 * e + 1]);
                        }
            const bool swapq = g.q0 > g.q1;
            cd mt[4][4];
            for (int si = 0; si < 2; ++si)
                for (int ti = 0; ti < 2; ++ti)
                    for (int sj = 0; sj < 2; ++sj)
                        for (int tj = 0; tj < 2; ++tj)
                            mt[si * 2 + ti][sj * 2 + tj] = swapq ? u4[sj][si][tj][ti] : u4[si][sj][ti][tj];
            double sig[4];
            cd uu[4][4], vv[4][4];
            svd4(mt, sig, uu, vv);
            HostGate h;
            h.i = std::min(g.q0, g.q1);
            h.j = std::max(g.q0, g.q1);
            h.layer = l;
            h.r = 0;
            for (int a = 0; a < 4; ++a)
                if (sig[a] > GATE_RANK_CUTOFF * sig[0]) h.r = a + 1;
            for (int a = 0; a < h.r; ++a) {
                const double rs = std::sqrt(sig[a]);
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        h.x[a][s][t] = rs * uu[s * 2 + t][a];
                        h.y[a][s][t] = rs * std::conj(vv[s * 2 + t][a]);
                    }
            }
            at[(size_t)l * n + h.i] = at[(size_t)l * n + h.j] = (int)hg.size();
            hg.push_back(h);
        }
        // this layer's one-qubit gates act before its two-qubit gates: absorb them on the input leg
        for (size_t q = first; q < hg.size(); ++q) {
            HostGate& h = hg[q];
            for (int a = 0; a < h.r; ++a) {
                cd gi[2][2], gj[2][2], tmp[2][2];
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) { gi[s][t] = G1(l, h.i, s, t); gj[s][t] = G1(l, h.j, s, t); }
                mul2(h.x[a], gi, tmp);
                std::memcpy(h.x[a], tmp, sizeof(tmp));
                mul2(h.y[a], gj, tmp);
                std::memcpy(h.y[a], tmp, sizeof(tmp));
            }
        }
        off += n_gates[l];
    }
    LayerMpo L;
    L.n_2q = (int)hg.size();
    L.w.assign(n + 1, 1);
    for (int c = 0; c <= n; ++c) {
        int64_t w = 1;
        for (auto& h : hg)
            if (h.i < c && c <= h.j) {
                w *= h.r;
                if (w > (int64_t)1 << 24) fail(MPS_ERR_ARG, "MPO bond dimension exceeds 2^24");
            }
        L.w[c] = w;
    }
    // digit a is less significant than digit b
    auto less_sig = [&](int a, int b) {
        return hg[a].i > hg[b].i || (hg[a].i == hg[b].i && hg[a].layer > hg[b].layer);
    };
    auto open_at = [&](int c) {
        std::vector<int> v;
        for (int q = 0; q < (int)hg.size(); ++q)
            if (hg[q].i < c && c <= hg[q].j) v.push_back(q);
        return v;
    };
    auto prod = [&](const std::vector<int>& v) {
        int64_t p = 1;
        for (int q : v) p *= hg[q].r;
        return p;
    };
    auto below = [&](const std::vector<int>& v, int g) {
        int64_t p = 1;
        for (int q : v)
            if (q != g && less_sig(q, g)) p *= hg[q].r;
        return p;
    };
    L.view[0].resize(n);
    L.view[1].resize(n);
    for (int k = 0; k < n; ++k) {
        // view 0 runs site k from bond k to bond k+1, view 1 from bond k+1 to bond k
        for (int o = 0; o < 2; ++o) {
            std::vector<int> present = open_at(o == 0 ? k : k + 1);
            const int64_t w_in = prod(present);
            std::vector<ProtoOp> seq;
            std::vector<bool> is_1q;
            for (int l = 0; l < K; ++l) {
                ProtoOp p;
                const int g = at[(size_t)l * n + k];
                if (g < 0) {
                    p.r_in = p.r_out = 1;
                    p.lo = 1;
                    p.H = prod(present);
                    for (int s = 0; s < 2; ++s)
                        for (int t = 0; t < 2; ++t) p.m[0][s][t] = G1(l, k, s, t);
                    seq.push_back(p);
                    is_1q.push_back(true);
                    continue;
                }
                const HostGate& h = hg[g];
                const bool opens = (h.i == k) == (o == 0);   // the digit appears in this view's direction
                const int64_t lo = below(present, g);
                p.lo = lo;
                if (opens) {
                    p.r_in = 1;
                    p.r_out = h.r;
                    p.H = prod(present) / lo;
                    present.push_back(g);
                } else {
                    p.r_in = h.r;
                    p.r_out = 1;
                    p.H = prod(present) / (h.r * lo);
                    present.erase(std::find(present.begin(), present.end(), g));
                }
                std::memcpy(p.m, h.i == k ? h.x : h.y, sizeof(p.m));
                seq.push_back(p);
                is_1q.push_back(false);
            }
            L.view[o][o == 0 ? k : n - 1 - k] = fold_site_ops(seq, is_1q, w_in);
        }
    }
    return L;
}

LayerMpo build_layer_mpo(int n, const mps_gate* gates, int n_gates) { return build_step_mpo(n, gates, &n_gates, 1); }

}  // namespace

// ================================================================ state ====
struct mps_state {
    int n = 0, max_chi = 1, prec = MPS_FP64;
    hipStream_t stream = nullptr;
    int orient = 0;               // stored tensor layout: 0 = [D_k][2][D_k+1], 1 = legs swapped
    int center = 0;               // site holding the norm: 0 or n-1
    std::vector<int> bond;        // n + 1 bond dimensions
    std::vector<Planar<double>> ten;  // per site, FP64 planar
    double log_f = 0;
    int n_layers = 0;
    int64_t n_2q = 0;
    std::vector<double> log_step_f, log_step_s2;
    std::vector<int> log_step_chi;
    // per applied step: the smallest separation (lambda_k - lambda_k+1) / lambda_1 of the Gram
    // eigenvalues at a cut where chi limited the kept count (inf: no such cut)
    std::vector<double> log_step_sep;
    double cur_min_sep = HUGE_VAL;
    bool invalid = false;
    rocblas_handle blas = nullptr;
    // scratch
    Planar<float> splitws;         // partial sums of split-K FP32 / split-precision GEMMs
    Raw<unsigned short> planes;    // BF16 terms of the operands of split-precision GEMMs
    Planar<double> splitws64;      // partial sums of split-K FP64 Gram matrices
    // second stream: with overlap_right, the right block of the next two-site
    // step runs on it while the current step's truncation runs on the state's stream
    hipStream_t stream2 = nullptr;
    Planar<float> splitws2;
    Raw<unsigned short> planes2;
    hipEvent_t ev_order[4] = {nullptr, nullptr, nullptr, nullptr};
    int eigh_method = 1;           // EIGH_PERSISTENT, or EIGH_ROCSOLVER
    // right blocks on the second stream (MPS_OVERLAP=1); off by default: on the benchmark the
    // overlap saved no time, and concurrent products stretch each other's launches
    bool overlap_right = false;
    Raw<double> dscal;             // small device scalars
    Raw<double> partial;           // reduction partials
    bool prof = false;
    bool has_alloc = false;
    mps_allocator alloc{};         // device-memory callbacks (used when has_alloc)
    int64_t eig_count[4] = {0, 0, 0, 0};   // see mps_eigensolver_counts
    KStat stats[MPS_KCLASS_COUNT];
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> event_pool;
};

namespace {

hipEvent_t get_event(mps_state* st) {
    if (!st->event_pool.empty()) {
        hipEvent_t e = st->event_pool.back();
        st->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

struct Timer {
    mps_state* st;
    int cls;
    double flops, bytes;
    hipStream_t strm;
    hipEvent_t a = nullptr;
    Timer(mps_state* s, int c, double f, double b, hipStream_t on = nullptr)
        : st(s), cls(c), flops(f), bytes(b), strm(on ? on : s->stream) {
        if (st->prof) {
            a = get_event(st);
            HIPCHK(hipEventRecord(a, strm));
        }
    }
    void done() {
        if (!st->prof) return;
        hipEvent_t b = get_event(st);
        HIPCHK(hipEventRecord(b, strm));
        st->pending.push_back({cls, a, b, flops, bytes});
    }
};

void flush_timings(mps_state* st) {
    if (st->pending.empty()) return;
    HIPCHK(hipStreamSynchronize(st->stream));
    if (st->stream2) HIPCHK(hipStreamSynchronize(st->stream2));
    for (auto& p : st->pending) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
        KStat& k = st->stats[p.cls];
        k.launches += 1;
        k.ms += ms;
        k.flops += p.flops;
        k.bytes += p.bytes;
        st->event_pool.push_back(p.a);
        st->event_pool.push_back(p.b);
    }
    st->pending.clear();
}

// ---------------------------------------------------------- GEMM helpers ---
// A stream and the split-K workspace that only work on that stream may use.
struct Lane {
    hipStream_t s;
    Planar<float>* ws;
    Raw<unsigned short>* pl;
};
Lane main_lane(mps_state* st) { return Lane{st->stream, &st->splitws, &st->planes}; }

template <typename R>
hipError_t gemm_raw(int opa, int opb, int M, int N, int K, const R* ar, const R* ai, int64_t lda,
                    const R* br, const R* bi, int64_t ldb, R* cr, R* ci, int64_t ldc, hipStream_t s);
template <>
hipError_t gemm_raw<float>(int opa, int opb, int M, int N, int K, const float* ar, const float* ai,
                           int64_t lda, const float* br, const float* bi, int64_t ldb, float* cr,
                           float* ci, int64_t ldc, hipStream_t s) {
    return cgemm_f32(opa, opb, M, N, K, {ar, ai, lda}, {br, bi, ldb}, {cr, ci, ldc}, s);
}
template <>
hipError_t gemm_raw<double>(int opa, int opb, int M, int N, int K, const double* ar, const double* ai,
                            int64_t lda, const double* br, const double* bi, int64_t ldb, double* cr,
                            double* ci, int64_t ldc, hipStream_t s) {
    return cgemm_f64(opa, opb, M, N, K, {ar, ai, lda}, {br, bi, ldb}, {cr, ci, ldc}, s);
}

// FP32 accumulation over a long k range loses accuracy like sqrt(K) eps (one
// accumulator per output).  Long contractions are cut into chunks of about
// 4096 terms whose partial sums are added in FP64; short ones with few output
// tiles are cut too, to occupy all CUs.  Returns the requested chunk count.
int splitk_for(int64_t M, int64_t N, int64_t K) {
    int64_t ks = 1;
    if (K >= 8192) ks = std::min<int64_t>(64, K / 4096);
    const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
    if (tiles < 256 && K >= 2048) ks = std::max<int64_t>(ks, std::min<int64_t>((512 + tiles - 1) / tiles, K / 1024));
    return (int)std::max<int64_t>(1, ks);
}

// The same for the split-precision kernel: 256 x 128 output tiles and one
// workgroup per compute unit, so an output of fewer than 256 tiles is split
// until it fills the 256 units (chunks of at least 512 terms).
int splitk_for_split(int64_t M, int64_t N, int64_t K) {
    int64_t ks = 1;
    if (K >= 8192) ks = std::min<int64_t>(64, K / 4096);
    const int64_t tiles = ((M + 255) / 256) * ((N + 127) / 128);
    if (tiles < 256 && K >= 1024) ks = std::max<int64_t>(ks, std::min<int64_t>((256 + tiles - 1) / tiles, K / 512));
    return (int)std::max<int64_t>(1, ks);
}

// Each launch is timed on its own; the split-K reduction counts as OTHER.
template <typename R>
void gemm(mps_state* st, int cls, int opa, int opb, int64_t M, int64_t N, int64_t K, const R* ar,
          const R* ai, int64_t lda, const R* br, const R* bi, int64_t ldb, R* cr, R* ci, int64_t ldc,
          const Lane* lane = nullptr) {
    if (M > 0x7fffffff || N > 0x7fffffff || K > 0x7fffffff) fail(MPS_ERR_ARG, "GEMM dimension too large");
    const Lane ln = lane ? *lane : main_lane(st);
    const double fl = 8.0 * (double)M * (double)N * (double)K;
    const double by = 2.0 * sizeof(R) * ((double)M * K + (double)K * N + (double)M * N);
    const int ks = sizeof(R) == 4 ? splitk_chunks((int)K, splitk_for(M, N, K), 16) : 1;
    if (ks > 1) {
        ln.ws->ensure(M * N * ks, ln.s);
        {
            Timer t(st, cls, fl, by, ln.s);
            HIPCHK(cgemm_f32_splitk(opa, opb, (int)M, (int)N, (int)K, {(const float*)ar, (const float*)ai, lda},
                                    {(const float*)br, (const float*)bi, ldb}, ln.ws->re(), ln.ws->im(),
                                    splitk_for(M, N, K), ln.s));
            t.done();
        }
        Timer t(st, MPS_KCLASS_OTHER, 0, 8.0 * (double)M * N * (ks + 1), ln.s);
        HIPCHK(splitk_reduce(ln.ws->re(), ln.ws->im(), ks, M, N, (float*)cr, (float*)ci, ldc, ln.s));
        t.done();
    } else {
        Timer t(st, cls, fl, by, ln.s);
        HIPCHK(gemm_raw<R>(opa, opb, (int)M, (int)N, (int)K, ar, ai, lda, br, bi, ldb, cr, ci, ldc, ln.s));
        t.done();
    }
}

// BF16 terms per FP32 operand of a split-precision state.
int split_terms(const mps_state* st) { return st->prec == MPS_BF16X2 ? 2 : 3; }
bool is_split(int prec) { return prec == MPS_BF16X2 || prec == MPS_BF16X3; }

// Split-precision (BF16 x 2 or x 3) complex GEMM, C = A B^T, on operands
// already split into BF16 planes (split_planes / split_planes_t).
void gemm_split_planes(mps_state* st, int cls, int64_t M, int64_t N, int64_t K, const unsigned short* pa,
                       const unsigned short* pb, float* cr, float* ci, int64_t ldc, const Lane& ln) {
    const double fl = 8.0 * (double)M * (double)N * (double)K;
    const double by = 8.0 * ((double)M * K + (double)K * N + (double)M * N);
    const int terms = split_terms(st);
    const int ks = splitk_chunks((int)K, splitk_for_split(M, N, K), 16);
    if (ks > 1) {
        ln.ws->ensure(M * N * ks, ln.s);
        {
            Timer t(st, cls, fl, by, ln.s);
            HIPCHK(cgemm_bf16_planes_splitk(terms, (int)M, (int)N, (int)K, pa, pb, ln.ws->re(), ln.ws->im(),
                                            splitk_for_split(M, N, K), ln.s));
            t.done();
        }
        Timer t(st, MPS_KCLASS_OTHER, 0, 8.0 * (double)M * N * (ks + 1), ln.s);
        HIPCHK(splitk_reduce(ln.ws->re(), ln.ws->im(), ks, M, N, cr, ci, ldc, ln.s));
        t.done();
    } else {
        Timer t(st, cls, fl, by, ln.s);
        HIPCHK(cgemm_bf16_planes(terms, (int)M, (int)N, (int)K, pa, pb, {cr, ci, ldc}, ln.s));
        t.done();
    }
}

// The lane's plane buffer for an A operand of M rows and a B operand of N rows over K.
void lane_planes(mps_state* st, const Lane& ln, int64_t M, int64_t N, int64_t K, unsigned short*& pa,
                 unsigned short*& pb) {
    const int terms = split_terms(st);
    const int64_t ea = split_planes_elems(terms, (int)M, (int)K, true);
    const int64_t eb = split_planes_elems(terms, (int)N, (int)K, false);
    ln.pl->ensure(ea + eb, ln.s);
    pa = ln.pl->p;
    pb = pa + ea;
}

// Split-precision complex GEMM, C = A B^T with both operands FP32 and
// k-contiguous: both are split once into BF16 planes (counted as OTHER, like
// the split-K sum), then multiplied.
void gemm_split(mps_state* st, int cls, int64_t M, int64_t N, int64_t K, const float* ar, const float* ai,
                int64_t lda, const float* br, const float* bi, int64_t ldb, float* cr, float* ci, int64_t ldc,
                const Lane* lane = nullptr) {
    if (M > 0x7fffffff || N > 0x7fffffff || K > 0x7fffffff) fail(MPS_ERR_ARG, "GEMM dimension too large");
    const Lane ln = lane ? *lane : main_lane(st);
    const int terms = split_terms(st);
    unsigned short *pa, *pb;
    lane_planes(st, ln, M, N, K, pa, pb);
    {
        // 8 bytes read and 4 terms bytes written per complex element
        Timer t(st, MPS_KCLASS_OTHER, 0, (8.0 + 4.0 * terms) * ((double)M + N) * K, ln.s);
        HIPCHK(split_planes(terms, (int)M, (int)K, true, {ar, ai, lda}, pa, ln.s));
        HIPCHK(split_planes(terms, (int)N, (int)K, false, {br, bi, ldb}, pb, ln.s));
        t.done();
    }
    gemm_split_planes(st, cls, M, N, K, pa, pb, cr, ci, ldc, ln);
}

// Split count for a GEMM with `active` output tiles over k range K: fill whole
// rounds of `slots` resident workgroups (256 CUs x workgroups per CU) with
// chunks of at least min_chunk terms; among equally full schedules the
// smallest count wins.
int fill_split(int64_t active, int64_t K, int64_t slots, int64_t min_chunk, int max_split) {
    int best = 1;
    double best_eff = 0;
    for (int ks = 1; ks <= max_split; ++ks) {
        if (ks > 1 && K / ks < min_chunk) break;
        const int64_t work = active * ks;
        const int64_t rounds = (work + slots - 1) / slots;
        // rounds shorter than a few slots' worth waste the machine at the tail
        const double eff = (double)work / (double)(rounds * slots);
        if (eff > best_eff + 1e-3) {
            best_eff = eff;
            best = ks;
        }
    }
    return best;
}

// Hermitian Gram product (lower tiles only) with FP64 accumulation; long k
// ranges are split so that whole rounds of workgroups run, and partial sums
// add in FP64.
template <typename TIn>
void gram_product(mps_state* st, int opa, int opb, int dim, int64_t K, const TIn* re, const TIn* im, int64_t ld,
                  double* out_re, double* out_im) {
    // non-empty lower tiles of the 128 x 64 FP64 tiling: row tile i holds columns up to 2i + 1
    const int64_t gm = (dim + 127) / 128, gn = (dim + 63) / 64;
    int64_t active = 0;
    for (int64_t i = 0; i < gm; ++i) active += std::min<int64_t>(gn, 2 * i + 2);
    const int ks = K >= 4096 ? fill_split(active, K, 512, 1024, 32) : 1;
    const int chunks = splitk_chunks((int)K, ks, 8);
    if (chunks > 1) {
        st->splitws64.ensure((int64_t)dim * dim * chunks, st->stream);
        if (sizeof(TIn) == 4)
            HIPCHK(cgemm_f32in_f64_splitk(opa, opb, dim, dim, (int)K, {(const float*)re, (const float*)im, ld},
                                          {(const float*)re, (const float*)im, ld}, st->splitws64.re(),
                                          st->splitws64.im(), ks, 1, st->stream));
        else
            HIPCHK(cgemm_f64_splitk(opa, opb, dim, dim, (int)K, {(const double*)re, (const double*)im, ld},
                                    {(const double*)re, (const double*)im, ld}, st->splitws64.re(),
                                    st->splitws64.im(), ks, 1, st->stream));
        HIPCHK(splitk_reduce64(st->splitws64.re(), st->splitws64.im(), chunks, dim, dim, out_re, out_im, dim,
                               st->stream));
    } else if (sizeof(TIn) == 4) {
        HIPCHK(cgemm_f32in_f64(opa, opb, dim, dim, (int)K, {(const float*)re, (const float*)im, ld},
                               {(const float*)re, (const float*)im, ld}, {out_re, out_im, dim}, st->stream, 1));
    } else {
        HIPCHK(cgemm_f64(opa, opb, dim, dim, (int)K, {(const double*)re, (const double*)im, ld},
                         {(const double*)re, (const double*)im, ld}, {out_re, out_im, dim}, st->stream, 1));
    }
}

// ===================================== batched tridiagonal reductions ====
// Inside apply_layer_dmrg_batched, instances run on several host threads and
// streams.  The persistent tridiagonal reduction of an order-n truncation is
// latency-bound and occupies n / 8 workgroups, one per compute unit, in a
// cooperative launch that no other cooperative launch can overlap; so the
// reductions that the threads reach at about the same time are gathered and
// run in one cooperative launch (at most hetrd_batch_max() instances and 256
// workgroups).  The first thread to arrive leads: it waits until every worker
// thread of the call has submitted, the launch is full, or a window of 1 ms has
// passed, then makes its stream wait for the others' ready events, launches on
// its stream, and records each member's done event there; every member's stream
// then waits on its done event.
struct TridiagBatcher {
    struct Item {
        TrRequest req;
        hipStream_t s;
        hipEvent_t ready, done;
        int P;
        bool launched = false;
        hipError_t err = hipSuccess;
    };
    std::mutex mu;
    std::condition_variable cv;
    std::vector<Item*> pending;
    int active = 0;                                   // worker threads that may still submit
    std::chrono::microseconds window{1000};
    int64_t launches = 0, reductions = 0;

    void worker_done() {
        std::lock_guard<std::mutex> lk(mu);
        --active;
        cv.notify_all();
    }

    // Launch a prefix of the pending items that fits (the front one always does).  Lock held.
    void launch_front() {
        std::vector<Item*> take, rest;
        int sumP = 0;
        for (Item* p : pending) {
            if ((int)take.size() < hetrd_batch_max() && sumP + p->P <= 256) {
                take.push_back(p);
                sumP += p->P;
            } else {
                rest.push_back(p);
            }
        }
        pending.swap(rest);
        const hipStream_t ls = take[0]->s;
        hipError_t err = hipSuccess;
        for (Item* p : take)
            if (err == hipSuccess && p->s != ls) err = hipStreamWaitEvent(ls, p->ready, 0);
        std::vector<TrRequest> reqs;
        for (Item* p : take) reqs.push_back(p->req);
        if (err == hipSuccess) err = hetrd_persistent_multi(reqs.data(), (int)reqs.size(), ls);
        if (err != hipSuccess) (void)hipGetLastError();
        for (Item* p : take) {
            if (err == hipSuccess) {
                const hipError_t e2 = hipEventRecord(p->done, ls);
                p->err = e2;
            } else {
                p->err = err;
            }
            p->launched = true;
        }
        ++launches;
        reductions += (int64_t)take.size();
        cv.notify_all();
    }

    hipError_t run(Item& it) {
        std::unique_lock<std::mutex> lk(mu);
        pending.push_back(&it);
        cv.notify_all();
        const auto t0 = std::chrono::steady_clock::now();
        while (!it.launched) {
            if (pending.front() == &it) {
                int sumP = 0;
                for (Item* p : pending) sumP += p->P;
                const bool full = sumP >= 256 || (int)pending.size() >= hetrd_batch_max();
                const bool all_here = (int)pending.size() >= active;
                if (full || all_here || std::chrono::steady_clock::now() - t0 >= window) {
                    launch_front();
                    break;
                }
                cv.wait_until(lk, t0 + window);
            } else {
                cv.wait(lk);
            }
        }
        return it.err;
    }
};

// The batcher of the batched call this thread works for (NULL outside such calls).
thread_local TridiagBatcher* g_batcher = nullptr;

// Shared launches and the reductions they carried, over all batched calls (mps_batch_stats).
struct BatchStats {
    std::atomic<int64_t> launches{0}, reductions{0};
} g_batch_stats;

// ================================================== FP64 eigensolver ====
enum { EIGH_ROCSOLVER = 0, EIGH_PERSISTENT = 1 };

struct EighWork {
    Raw<double> Z, evals, evwork, tau;   // Z: eigenvectors (complex for the library solver, real of T otherwise)
    Planar<double> vh, S, T, Y, W, ws;   // reflectors (conjugated rows) and back-transformation scratch
    Raw<char> trws, dcws;                // tridiagonal reduction and divide-and-conquer workspaces
    Raw<int> info;
    Raw<double> nrm;                     // partial sums and result of the eigenvector check
    int method_used = EIGH_ROCSOLVER;
    void release(hipStream_t s) {
        Z.release(s); evals.release(s); evwork.release(s); tau.release(s);
        vh.release(s); S.release(s); T.release(s); Y.release(s); W.release(s); ws.release(s);
        trws.release(s); dcws.release(s); info.release(s); nrm.release(s);
    }
};

// C = op(A) op(B) in FP64 with the k range split for short, wide products.
void gemm64_long_k(mps_state* st, EighWork& wk, int opa, int opb, int M, int N, int K, CView<double> A,
                   CView<double> B, CViewMut<double> C) {
    const int64_t tiles = (int64_t)((M + 127) / 128) * ((N + 63) / 64);
    int ks = 1;
    if (K >= 128 && tiles < 256) ks = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)32, K / 64, (512 + tiles - 1) / tiles}));
    const int chunks = splitk_chunks(K, ks, 8);
    if (chunks > 1) {
        wk.ws.ensure((int64_t)M * N * chunks, st->stream);
        HIPCHK(cgemm_f64_splitk(opa, opb, M, N, K, A, B, wk.ws.re(), wk.ws.im(), ks, 0, st->stream));
        HIPCHK(splitk_reduce64(wk.ws.re(), wk.ws.im(), chunks, M, N, C.re, C.im, C.ld, st->stream));
    } else {
        HIPCHK(cgemm_f64(opa, opb, M, N, K, A, B, C, st->stream));
    }
}

// Eigen-decomposition of the Hermitian dim x dim matrix given by the lower
// triangle (row >= column) of the row-major planar array (re, im).  On
// return wk.evals holds the eigenvalues in ascending order; top_eigvecs()
// then forms the eigenvectors of the largest ones.
// EIGH_PERSISTENT: tridiagonal reduction by the persistent kernel, the
// library's own divide and conquer on the real tridiagonal matrix
// (stedc_dc), and (in top_eigvecs) the blocked back-transformation by the
// reflectors on the kept columns only.
// It falls back to rocSOLVER's dense solver when the cooperative launch is
// refused or gives up waiting.
// after_reduce (may be null) is called once the reduction no longer needs
// the whole device: work that the caller queues on other streams from it
// does not compete with the cooperative launch.
void eigh_gram(mps_state* st, EighWork& wk, const double* re, const double* im, int dim, int method,
               const std::function<void()>* after_reduce = nullptr) {
    const hipStream_t s = st->stream;
    wk.evals.ensure(dim, s);
    wk.evwork.ensure(dim, s);
    wk.info.ensure(1, s);
    if (method == EIGH_PERSISTENT && dim >= 2 && dim <= hetrd_max_n()) {
        wk.Z.ensure(2 * (int64_t)dim * dim, s);      // full matrix first, real eigenvectors after
        // reflectors padded to whole blocks of the back-transformation with zero rows (tau = 0)
        const int nb = wy_block(dim), nblk = (dim - 1 + nb - 1) / nb, npad = nblk * nb - (dim - 1);
        wk.tau.ensure(2 * (int64_t)nblk * nb, s);
        wk.vh.ensure((int64_t)nblk * nb * dim, s);
        if (npad > 0) {
            HIPCHK(hipMemsetAsync(wk.tau.p + 2 * (int64_t)(dim - 1), 0, sizeof(double) * 2 * npad, s));
            HIPCHK(hipMemsetAsync(wk.vh.re() + (int64_t)(dim - 1) * dim, 0, sizeof(double) * npad * dim, s));
            HIPCHK(hipMemsetAsync(wk.vh.im() + (int64_t)(dim - 1) * dim, 0, sizeof(double) * npad * dim, s));
        }
        const size_t wsb = hetrd_workspace_bytes(dim);
        wk.trws.ensure((int64_t)wsb, s);
        {
            Timer t(st, MPS_KCLASS_OTHER, 0, 32.0 * dim * dim);
            HIPCHK(hermitian_full_colmajor(re, im, dim, wk.Z.p, s));
            t.done();
        }
        int* abort_dev = nullptr;
        int aborted = 1;
        {
            Timer tr(st, MPS_KCLASS_TRIDIAG, 16.0 / 3.0 * dim * (double)dim * dim, 16.0 * dim * (double)dim);
            hipError_t le;
            if (g_batcher && hetrd_workgroups(dim) > 1) {
                // gathered with the reductions of the other instances of the batched call
                TridiagBatcher::Item it;
                it.req = TrRequest{wk.Z.p, dim, wk.evals.p, wk.evwork.p, wk.tau.p, wk.vh.re(), wk.vh.im(),
                                   wk.trws.p, wsb, &abort_dev};
                it.s = s;
                it.P = hetrd_workgroups(dim);
                it.ready = get_event(st);
                it.done = get_event(st);
                HIPCHK(hipEventRecord(it.ready, s));
                le = g_batcher->run(it);
                if (le == hipSuccess) le = hipStreamWaitEvent(s, it.done, 0);
                st->event_pool.push_back(it.ready);
                st->event_pool.push_back(it.done);
            } else {
                le = hetrd_persistent(wk.Z.p, dim, wk.evals.p, wk.evwork.p, wk.tau.p, wk.vh.re(), wk.vh.im(),
                                      wk.trws.p, wsb, &abort_dev, s);
            }
            tr.done();
            if (le == hipSuccess) {
                HIPCHK(hipMemcpyAsync(&aborted, abort_dev, sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            } else {
                (void)hipGetLastError();
            }
        }
        Timer t(st, MPS_KCLASS_EIGH, 0, 0);
        if (!aborted) {
            if (after_reduce) (*after_reduce)();
            const size_t dcb = stedc_dc_workspace_bytes(dim);
            wk.dcws.ensure((int64_t)dcb, s);
            HIPCHK(stedc_dc(dim, wk.evals.p, wk.evwork.p, wk.Z.p, dim, wk.dcws.p, dcb, s));
            HIPCHK(hipMemsetAsync(wk.info.p, 0, sizeof(int), s));
            t.done();
            wk.method_used = EIGH_PERSISTENT;
            st->eig_count[dim <= 128 ? 1 : 0] += 1;
            return;
        }
        t.done();
        st->eig_count[2] += 1;                       // the persistent reduction was refused or gave up
    } else {
        st->eig_count[3] += 1;
    }
    wk.Z.ensure(2 * (int64_t)dim * dim, s);
    {
        Timer t(st, MPS_KCLASS_OTHER, 0, 32.0 * dim * dim);
        HIPCHK(pack_hermitian(re, im, dim, wk.Z.p, s));
        t.done();
    }
    Timer t(st, MPS_KCLASS_EIGH, 0, 0);
    rocblas_status rs = rocsolver_zheevd(st->blas, rocblas_evect_original, rocblas_fill_upper, dim,
                                         (rocblas_double_complex*)wk.Z.p, dim, wk.evals.p, wk.evwork.p, wk.info.p);
    t.done();
    if (rs != rocblas_status_success) fail(MPS_ERR_DEVICE, "rocsolver_zheevd failed: status " + std::to_string((int)rs));
    wk.method_used = EIGH_ROCSOLVER;
    if (after_reduce) (*after_reduce)();
}

// Eigenvectors of the k largest eigenvalues after eigh_gram(), as planar
// row-major dim x k (largest first).  For the persistent path this applies
// Q = H_0 H_1 ... H_{dim-2} to the eigenvectors of T in blocks b of nb
// reflectors, Q_b = I - V_b T_b V_b^H, last block first.  The factors of all
// blocks are formed up front (S_b = V_b^H V_b, T_b, Y_b = T_b V_b^H, three
// batched launches); each block then costs two products on the rows below it:
//   W = Y_b U,  U -= V_b W.
void top_eigvecs(mps_state* st, EighWork& wk, int dim, int k, double* out_re, double* out_im) {
    const hipStream_t s = st->stream;
    if (wk.method_used == EIGH_ROCSOLVER) {
        HIPCHK(take_top_eigvecs(wk.Z.p, dim, k, nullptr, out_re, out_im, s));
        // the dense library solver has returned non-finite eigenvectors for some inputs
        // (diagonal matrices of order >= 100): check the kept ones
        // (the work buffers are the eigensolver's own: callers such as the self-test pass a
        // state without reduction buffers)
        double nrm = 0;
        wk.nrm.ensure(1024 + 1, s);
        HIPCHK(norm2<double>(out_re, out_im, (int64_t)dim * k, wk.nrm.p, wk.nrm.p + 1024, s));
        HIPCHK(hipMemcpyAsync(&nrm, wk.nrm.p + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!std::isfinite(nrm)) fail(MPS_ERR_NUMERIC, "eigensolver returned non-finite eigenvectors");
        return;
    }
    HIPCHK(take_top_real_eigvecs(wk.Z.p, dim, k, out_re, out_im, s));
    Timer t(st, MPS_KCLASS_EIGH, 0, 0);
    const int nb = wy_block(dim), nblk = (dim - 1 + nb - 1) / nb;
    const int64_t nbb = (int64_t)nb * nb, nbd = (int64_t)nb * dim;
    wk.S.ensure(nblk * nbb, s);
    wk.T.ensure(nblk * nbb, s);
    wk.Y.ensure(nblk * nbd, s);
    wk.W.ensure((int64_t)nb * k, s);
    const int ks = std::max(1, std::min(32, dim / 64));
    const int chunks = splitk_chunks(dim, ks, 8);
    wk.ws.ensure(chunks * nblk * nbb, s);
    HIPCHK(cgemm_f64_batched_splitk(OP_N, OP_C, nb, nb, dim, {wk.vh.re(), wk.vh.im(), dim}, nbd,
                                    {wk.vh.re(), wk.vh.im(), dim}, nbd, wk.ws.re(), wk.ws.im(), ks, nblk, s));
    HIPCHK(splitk_reduce64(wk.ws.re(), wk.ws.im(), chunks, (int64_t)nblk * nb, nb, wk.S.re(), wk.S.im(), nb, s));
    // T factors: the 64 x 64 diagonal sub-blocks from the recurrence, then pairs of
    // h-blocks merged into 2h-blocks, I - [V1 V2] [[T1, -T1 (V1^H V2) T2], [0, T2]] [V1 V2]^H
    // being the product of the two compact WY forms (the blocks below the diagonal stay zero)
    if (nb > 64) {
        HIPCHK(hipMemsetAsync(wk.T.re(), 0, sizeof(double) * nblk * nbb, s));
        HIPCHK(hipMemsetAsync(wk.T.im(), 0, sizeof(double) * nblk * nbb, s));
    }
    HIPCHK(wy_t_diag_factors(wk.S.re(), wk.S.im(), nblk, nb, wk.tau.p, wk.T.re(), wk.T.im(), s));
    for (int h = 64; h < nb; h *= 2)
        for (int o = 0; o < nb; o += 2 * h) {
            const int64_t d1 = (int64_t)o * nb + o, d2 = (int64_t)(o + h) * nb + (o + h), up = (int64_t)o * nb + o + h;
            // X = S12 T2 (h x h per block, in the split-K workspace), then T12 -= T1 X
            HIPCHK(cgemm_f64_batched(OP_N, OP_N, h, h, h, {wk.S.re() + up, wk.S.im() + up, nb}, nbb,
                                     {wk.T.re() + d2, wk.T.im() + d2, nb}, nbb, {wk.ws.re(), wk.ws.im(), h},
                                     (int64_t)h * h, nblk, s));
            HIPCHK(cgemm_f64_batched_sub(h, h, h, {wk.T.re() + d1, wk.T.im() + d1, nb}, nbb,
                                         {wk.ws.re(), wk.ws.im(), h}, (int64_t)h * h,
                                         {wk.T.re() + up, wk.T.im() + up, nb}, nbb, nblk, s));
        }
    HIPCHK(cgemm_f64_batched(OP_N, OP_N, nb, dim, nb, {wk.T.re(), wk.T.im(), nb}, nbb, {wk.vh.re(), wk.vh.im(), dim},
                             nbd, {wk.Y.re(), wk.Y.im(), dim}, nbd, nblk, s));
    for (int b = nblk - 1; b >= 0; --b) {
        const int r0 = b * nb + 1, rows = dim - r0;          // v_j[r] = 0 for r <= j
        if (rows <= 0) continue;
        const CView<double> Yb{wk.Y.re() + b * nbd + r0, wk.Y.im() + b * nbd + r0, dim};
        const CView<double> Vb{wk.vh.re() + b * nbd + r0, wk.vh.im() + b * nbd + r0, dim};
        gemm64_long_k(st, wk, OP_N, OP_N, nb, k, rows, Yb, {out_re + (int64_t)r0 * k, out_im + (int64_t)r0 * k, k},
                      {wk.W.re(), wk.W.im(), k});
        HIPCHK(cgemm_f64_sub(OP_C, OP_N, rows, k, nb, Vb, {wk.W.re(), wk.W.im(), k},
                             {out_re + (int64_t)r0 * k, out_im + (int64_t)r0 * k, k}, s));
    }
    t.done();
}

// =========================================================== the engine ====
template <typename R>
struct Engine {
    mps_state* st;
    hipStream_t s;
    int n, chi;
    LayerMpo mpo;
    std::vector<int> cb;              // bond dims of phi (being built)
    std::vector<Planar<R>> env;       // per bond
    std::vector<Planar<R>> psi[2];    // per view-site, view layout
    std::vector<Planar<double>> phi;  // per site, layout of the pass that wrote it
    Planar<R> X, T2, TH, UR;
    Planar<R> XR, T2R[2];             // right blocks (written on the second stream with overlap_right)
    Planar<R> MT[2][2];               // per lane: intermediates of multi-layer MPO factors
    bool split = false;   // split-precision BF16 contractions (R = float only): operands kept k-contiguous
    Planar<double> TH64, GR, U64, V64, M64;
    Planar<double> LX, LY, LQ, LR, LP, LT, LU;   // factors of a low-rank two-site truncation
    EighWork ew;
    Raw<double> svec, QZ, QG, QT;
    Raw<int> QI;
    std::vector<double> hvals;

    std::vector<int> chi_bond;        // per-bond caps (n + 1 entries); empty: chi everywhere

    Engine(mps_state* state, int chi_) : st(state), s(state->stream), n(state->n), chi(chi_) {}

    int chi_at(int b) const { return chi_bond.empty() ? chi : chi_bond[b]; }

    ~Engine() {
        if (st->stream2) (void)hipStreamSynchronize(st->stream2);   // right blocks in flight
        XR.release(s); T2R[0].release(s); T2R[1].release(s);
        for (auto& l : MT) { l[0].release(s); l[1].release(s); }
        for (auto& e : env) e.release(s);
        for (int o = 0; o < 2; ++o)
            for (auto& e : psi[o]) e.release(s);
        X.release(s); T2.release(s); TH.release(s); UR.release(s);
        TH64.release(s); GR.release(s); U64.release(s); V64.release(s); M64.release(s);
        LX.release(s); LY.release(s); LQ.release(s); LR.release(s); LP.release(s); LT.release(s); LU.release(s);
        ew.release(s); svec.release(s); QZ.release(s); QG.release(s); QT.release(s); QI.release(s);
        for (auto& p : phi) p.release(s);
    }

    int site(int o, int j) const { return o == 0 ? j : n - 1 - j; }
    int bnd(int o, int j) const { return o == 0 ? j : n - j; }

    // ---------------------------------------------------------- truncation
    struct Trunc {
        int k;
        double f, total;
        bool caseA;
    };

    // FP64 eigen-decomposition of the Hermitian dim x dim Gram matrix in GR.
    const std::function<void()>* after_reduce = nullptr;
    void eigh(int dim) { eigh_gram(st, ew, GR.re(), GR.im(), dim, st->eigh_method, after_reduce); }

    // Kept count and weights from the eigenvalues of the Gram matrix.
    Trunc select(int dim, int chi_) {
        hvals.resize(dim);
        int hinfo = 0;
        HIPCHK(hipMemcpyAsync(hvals.data(), ew.evals.p, sizeof(double) * dim, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hinfo, ew.info.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hinfo != 0) fail(MPS_ERR_NUMERIC, "eigensolver did not converge (info " + std::to_string(hinfo) + ")");
        for (int i = 0; i < dim; ++i)
            if (!std::isfinite(hvals[i])) fail(MPS_ERR_NUMERIC, "eigensolver returned a non-finite eigenvalue");
        double total = 0;
        for (int i = dim - 1; i >= 0; --i) total += hvals[i];
        if (!(total > 0) || !std::isfinite(total)) fail(MPS_ERR_NUMERIC, "local tensor has zero or non-finite norm");
        int keep = 0;
        for (int i = dim - 1; i >= 0; --i)
            if (hvals[i] > EPS_TRUNC * total) ++keep;
        const int k = std::max(1, std::min(chi_, keep));
        double f = 0;
        for (int i = 0; i < k; ++i) f += hvals[dim - 1 - i];
        if (keep > chi_ && hvals[dim - 1] > 0)          // the cut at chi discarded weight above the threshold
            st->cur_min_sep = std::min(st->cur_min_sep, (hvals[dim - k] - hvals[dim - 1 - k]) / hvals[dim - 1]);
        return Trunc{k, f, total, true};
    }

    // Truncated SVD of the rows x cols matrix M (working precision, planar,
    // row-major).  On return U64 holds U (rows x k).  When want_right is set,
    // V64 holds the right factor S V^H / sqrt(f) (k x cols).
    Trunc truncate(const R* m_re, const R* m_im, int64_t rows, int64_t cols, bool want_right,
                   const double* m64_re, const double* m64_im, int bond) {
        const int chi = chi_at(bond);
        if (rows <= cols) {
            const int dim = (int)rows;
            GR.ensure((int64_t)dim * dim, s);
            {
                // Hermitian product: rows (rows + 1) / 2 distinct entries of cols MACs each
                Timer t(st, MPS_KCLASS_GRAM, 4.0 * rows * (rows + 1) * cols, 2.0 * sizeof(R) * rows * cols + 8.0 * rows * (rows + 1));
                if (m64_re)
                    gram_product<double>(st, OP_N, OP_C, dim, cols, m64_re, m64_im, cols, GR.re(), GR.im());
                else
                    gram_product<R>(st, OP_N, OP_C, dim, cols, m_re, m_im, cols, GR.re(), GR.im());
                t.done();
            }
            eigh(dim);
            Trunc tr = select(dim, chi);
            U64.ensure(rows * tr.k, s);
            top_eigvecs(st, ew, dim, tr.k, U64.re(), U64.im());
            if (want_right) {
                if (!m64_re) fail(MPS_ERR_ARG, "internal: right factor needs FP64 input");
                V64.ensure((int64_t)tr.k * cols, s);
                gemm<double>(st, MPS_KCLASS_OTHER, OP_C, OP_N, tr.k, cols, rows, U64.re(), U64.im(), tr.k,
                             m64_re, m64_im, cols, V64.re(), V64.im(), cols);
                set_scalar(0, 1.0 / std::sqrt(tr.f));
                HIPCHK(scale_by_device_scalar<double>(V64.re(), V64.im(), (int64_t)tr.k * cols, st->dscal.p, s));
            }
            tr.caseA = true;
            return tr;
        }
        // rows > cols: eigen-decompose M^H M, U = M V S^{-1}
        const int dim = (int)cols;
        if (!m64_re) {
            M64.ensure(rows * cols, s);
            HIPCHK((convert_planar<R, double>(m_re, m_im, rows * cols, M64.re(), M64.im(), s)));
            m64_re = M64.re();
            m64_im = M64.im();
        }
        GR.ensure((int64_t)dim * dim, s);
        {
            Timer t(st, MPS_KCLASS_GRAM, 4.0 * cols * (cols + 1) * rows, 16.0 * rows * cols + 8.0 * cols * (cols + 1));
            gram_product<double>(st, OP_C, OP_N, dim, rows, m64_re, m64_im, cols, GR.re(), GR.im());
            t.done();
        }
        eigh(dim);
        Trunc tr = select(dim, chi);
        V64.ensure((int64_t)dim * tr.k, s);
        top_eigvecs(st, ew, dim, tr.k, V64.re(), V64.im());
        std::vector<double> inv_s(tr.k), s_over(tr.k);
        for (int i = 0; i < tr.k; ++i) {
            const double sv = std::sqrt(std::max(hvals[dim - 1 - i], 0.0));
            inv_s[i] = sv > 0 ? 1.0 / sv : 0.0;
            s_over[i] = sv / std::sqrt(tr.f);
        }
        svec.ensure(2 * tr.k, s);
        HIPCHK(hipMemcpyAsync(svec.p, inv_s.data(), sizeof(double) * tr.k, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(svec.p + tr.k, s_over.data(), sizeof(double) * tr.k, hipMemcpyHostToDevice, s));
        U64.ensure(rows * tr.k, s);
        gemm<double>(st, MPS_KCLASS_OTHER, OP_N, OP_N, rows, tr.k, cols, m64_re, m64_im, cols, V64.re(), V64.im(),
                     tr.k, U64.re(), U64.im(), tr.k);
        HIPCHK(scale_columns(U64.re(), U64.im(), rows, tr.k, svec.p, s));
        if (want_right) {
            // S V^H / sqrt(f): (k x cols) from V (cols x k)
            Planar<double> tmp;
            tmp.ensure((int64_t)tr.k * cols, s);
            HIPCHK(scaled_adjoint(V64.re(), V64.im(), dim, tr.k, svec.p + tr.k, tmp.re(), tmp.im(), s));
            std::swap(tmp, V64);
            tmp.release(s);
        }
        HIPCHK(hipStreamSynchronize(s));  // host vectors above must outlive their copies
        tr.caseA = false;
        return tr;
    }

    // Truncation of Theta = X Y^T (X: rows x r, Y: cols x r, planar row-major, working
    // precision, r < rows and r < cols), without forming Theta: the Gram matrix
    // Theta Theta^H = X (Y^T conj(Y)) X^H has rank <= r, and with X = Q R (Q orthonormal,
    // rows x r) its non-zero eigen-pairs are those of the order-r Hermitian matrix
    // H = R conj(Y^H Y) R^H = R (Y^H Y)^T R^H, whose eigenvectors Q maps back.  The kept
    // values, the total weight (trace H = |Theta|^2) and U64 are those truncate() returns, up
    // to rounding (H carries errors of order eps |X|^2 |Y|^2 where the Gram matrix of Theta
    // carries eps |Theta|^2; the two agree when the factors are not much larger than Theta,
    // as in the sweep); the eigen-decomposition has order r instead of min(rows, cols).
    Trunc truncate_lowrank(const R* x_re, const R* x_im, const R* y_re, const R* y_im, int64_t rows, int64_t cols,
                           int64_t r, int bond) {
        const int chi = chi_at(bond);
        LX.ensure(rows * r, s);
        LY.ensure(cols * r, s);
        HIPCHK((convert_planar<R, double>(x_re, x_im, rows * r, LX.re(), LX.im(), s)));
        HIPCHK((convert_planar<R, double>(y_re, y_im, cols * r, LY.re(), LY.im(), s)));
        const int64_t kq = qr_orth(rows, r, LX.re(), LX.im());        // Q (rows x r) in U64
        std::swap(U64, LQ);
        LR.ensure(kq * r, s);
        LP.ensure(r * r, s);
        LT.ensure(kq * r, s);
        GR.ensure(kq * kq, s);
        gemm<double>(st, MPS_KCLASS_GRAM, OP_C, OP_N, kq, r, rows, LQ.re(), LQ.im(), kq, LX.re(), LX.im(), r,
                     LR.re(), LR.im(), r);                                   // R = Q^H X
        gemm<double>(st, MPS_KCLASS_GRAM, OP_C, OP_N, r, r, cols, LY.re(), LY.im(), r, LY.re(), LY.im(), r,
                     LP.re(), LP.im(), r);                                   // P = Y^H Y
        gemm<double>(st, MPS_KCLASS_GRAM, OP_N, OP_T, kq, r, r, LR.re(), LR.im(), r, LP.re(), LP.im(), r,
                     LT.re(), LT.im(), r);                                   // R P^T
        gemm<double>(st, MPS_KCLASS_GRAM, OP_N, OP_C, kq, kq, r, LT.re(), LT.im(), r, LR.re(), LR.im(), r,
                     GR.re(), GR.im(), kq);                                  // H = R P^T R^H
        eigh((int)kq);
        Trunc tr = select((int)kq, chi);
        LU.ensure(kq * tr.k, s);
        top_eigvecs(st, ew, (int)kq, tr.k, LU.re(), LU.im());
        U64.ensure(rows * tr.k, s);
        gemm<double>(st, MPS_KCLASS_EIGH, OP_N, OP_N, rows, tr.k, kq, LQ.re(), LQ.im(), kq, LU.re(), LU.im(), tr.k,
                     U64.re(), U64.im(), tr.k);                              // U = Q U_H
        tr.caseA = true;
        return tr;
    }

    // FP64 QR of the planar row-major rows x cols matrix (re, im): U64 <- Q
    // (rows x k, k = min(rows, cols)), an orthonormal basis of its column space
    // with the order of the columns kept (M = Q R, R upper triangular).
    // Cholesky QR twice when rows >= cols: each pass G = X^H X (rocBLAS herk),
    // R = chol(G) (rocSOLVER potrf), X <- X R^{-1} (rocBLAS trsm); the second
    // pass restores orthogonality to rounding for condition numbers up to
    // ~1e7.  Householder QR (rocSOLVER geqrf + ungqr) when rows < cols or when
    // a Cholesky factorisation fails.
    int qr_orth(int64_t rows, int64_t cols, const double* re, const double* im) {
        const int64_t k = std::min(rows, cols);
        QZ.ensure(2 * rows * cols, s);
        HIPCHK(rm_planar_to_cm(re, im, rows, cols, QZ.p, s));
        rocblas_double_complex* X = (rocblas_double_complex*)QZ.p;
        const rocblas_double_complex one(1.0, 0.0);
        const double one_r = 1.0, zero_r = 0.0;
        bool ok = false;
        {
            Timer t(st, MPS_KCLASS_EIGH, 0, 0);
            if (rows >= cols) {
                QG.ensure(2 * cols * cols, s);
                QI.ensure(2, s);
                rocblas_double_complex* G = (rocblas_double_complex*)QG.p;
                bool st_ok = true;
                for (int pass = 0; pass < 2 && st_ok; ++pass) {
                    st_ok = rocblas_zherk(st->blas, rocblas_fill_upper, rocblas_operation_conjugate_transpose, (int)cols,
                                          (int)rows, &one_r, X, (int)rows, &zero_r, G, (int)cols) == rocblas_status_success;
                    st_ok = st_ok && rocsolver_zpotrf(st->blas, rocblas_fill_upper, (int)cols, G, (int)cols,
                                                      QI.p + pass) == rocblas_status_success;
                    st_ok = st_ok && rocblas_ztrsm(st->blas, rocblas_side_right, rocblas_fill_upper,
                                                   rocblas_operation_none, rocblas_diagonal_non_unit, (int)rows,
                                                   (int)cols, &one, G, (int)cols, X, (int)rows) == rocblas_status_success;
                }
                int hinfo[2] = {1, 1};
                if (st_ok) {
                    HIPCHK(hipMemcpyAsync(hinfo, QI.p, sizeof(hinfo), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                }
                ok = st_ok && hinfo[0] == 0 && hinfo[1] == 0;
                if (!ok) HIPCHK(rm_planar_to_cm(re, im, rows, cols, QZ.p, s));   // restart from M
            }
            if (!ok) {
                QT.ensure(2 * k, s);
                rocblas_double_complex* tau = (rocblas_double_complex*)QT.p;
                if (rocsolver_zgeqrf(st->blas, (int)rows, (int)cols, X, (int)rows, tau) != rocblas_status_success ||
                    rocsolver_zungqr(st->blas, (int)rows, (int)k, (int)k, X, (int)rows, tau) != rocblas_status_success)
                    fail(MPS_ERR_DEVICE, "rocsolver QR failed");
            }
            t.done();
        }
        U64.ensure(rows * k, s);
        HIPCHK(cm_to_rm_planar(QZ.p, rows, k, U64.re(), U64.im(), s));
        return (int)k;
    }

    void set_scalar(int idx, double v) {
        HIPCHK(hipMemcpyAsync(st->dscal.p + idx, &v, sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }

    // ------------------------------------------------------------ layer
    // Buffers grow when written: the zip-up may keep more singular values
    // than 2^min(c, n-c) at bond c (its right factor carries the MPO bond),
    // so no static cap is used.
    void setup() {
        env.resize(n + 1);
        env[0].ensure(1, s);
        env[n].ensure(1, s);
        HIPCHK(fill_planar<R>(env[0].re(), env[0].im(), 1, 1.0, s));
        HIPCHK(fill_planar<R>(env[n].re(), env[n].im(), 1, 1.0, s));
        // psi in both views
        for (int o = 0; o < 2; ++o) {
            psi[o].resize(n);
            for (int j = 0; j < n; ++j) {
                const int k = site(o, j);
                const int64_t sz = (int64_t)st->bond[k] * 2 * st->bond[k + 1];
                psi[o][j].ensure(sz, s);
                const int Dl = st->orient == 0 ? st->bond[k] : st->bond[k + 1];
                const int Dr = st->orient == 0 ? st->bond[k + 1] : st->bond[k];
                Timer t(st, MPS_KCLASS_OTHER, 0, (8.0 + sizeof(R) * 2) * sz);
                if (split) {
                    // k-major copy: (2 D_right) x D_left with the view's legs
                    const int Dlv = st->orient != o ? Dr : Dl, Drv = st->orient != o ? Dl : Dr;
                    HIPCHK(site_to_kmajor(st->ten[k].re(), st->ten[k].im(), Dlv, Drv, st->orient != o ? 1 : 0,
                                          (float*)psi[o][j].re(), (float*)psi[o][j].im(), s));
                } else {
                    HIPCHK(site_to_view<R>(st->ten[k].re(), st->ten[k].im(), Dl, Dr, st->orient != o ? 1 : 0,
                                           psi[o][j].re(), psi[o][j].im(), s));
                }
                t.done();
            }
        }
        phi.resize(n);
        cb.assign(n + 1, 1);
    }

    // L_j A_j W_j for view o, view-site j, into out ([cL][2][wM][DM]); xb holds
    // the intermediate L_j A_j.  Applied in the mirrored view this is the right
    // block A W R of a pair, with the pair's right site as view-site j.
    void block(int o, int j, Planar<R>& xb, Planar<R>& out, const Lane& ln) {
        const int bL = bnd(o, j), bM = bnd(o, j + 1);
        const int64_t cL = cb[bL], wL = mpo.w[bL], wM = mpo.w[bM];
        const int64_t DL = st->bond[bL], DM = st->bond[bM];
        xb.ensure(cL * wL * 2 * DM, ln.s);
        out.ensure(cL * 2 * wM * DM, ln.s);
        if (split)
            gemm_split(st, MPS_KCLASS_CONTRACT, cL * wL, 2 * DM, DL, (const float*)env[bL].re(),
                       (const float*)env[bL].im(), DL, (const float*)psi[o][j].re(), (const float*)psi[o][j].im(), DL,
                       (float*)xb.re(), (float*)xb.im(), 2 * DM, &ln);
        else
            gemm<R>(st, MPS_KCLASS_CONTRACT, OP_N, OP_N, cL * wL, 2 * DM, DL, env[bL].re(), env[bL].im(), DL,
                    psi[o][j].re(), psi[o][j].im(), 2 * DM, xb.re(), xb.im(), 2 * DM, &ln);
        const std::vector<MpoSiteOp>& ops = mpo.view[o][j];
        // several layers acting at this site: one factor after the other, through
        // two temporaries of the lane
        Planar<R>* tmp = MT[ln.s == s ? 0 : 1];
        const R* in_re = xb.re();
        const R* in_im = xb.im();
        int64_t w_in = wL;
        for (size_t q = 0; q < ops.size(); ++q) {
            const MpoSiteOp& op = ops[q];
            const int64_t w_out = (int64_t)op.H * op.r_out * op.lo;
            Planar<R>& dst = q + 1 == ops.size() ? out : tmp[q & 1];
            dst.ensure(cL * 2 * w_out * DM, ln.s);
            Timer t(st, MPS_KCLASS_MPO, 0, 2.0 * sizeof(R) * (cL * w_in * 2 * DM + cL * 2 * w_out * DM), ln.s);
            HIPCHK(mpo_apply<R>(op, cL, DM, in_re, in_im, dst.re(), dst.im(), ln.s));
            t.done();
            in_re = dst.re();
            in_im = dst.im();
            w_in = w_out;
        }
        if (w_in != wM) fail(MPS_ERR_DEVICE, "MPO factors do not end on the bond dimension");
    }

    void left_block(int o, int j) { block(o, j, X, T2, main_lane(st)); }

    // Store U64 (rows x k) as the phi tensor of site k0 and update the left
    // environment of bond bM from T2: env = U^H T2 (k x (wM DM)).
    void finish_left(int o, int j, const Trunc& tr, bool update_env) {
        const int k0 = site(o, j);
        const int bL = bnd(o, j), bM = bnd(o, j + 1);
        const int64_t cL = cb[bL], wM = mpo.w[bM], DM = st->bond[bM];
        const int64_t rows = 2 * cL;
        phi[k0].ensure(rows * tr.k, s);
        HIPCHK((convert_planar<double, double>(U64.re(), U64.im(), rows * tr.k, phi[k0].re(), phi[k0].im(), s)));
        cb[bM] = tr.k;
        if (!update_env) return;
        env[bM].ensure(tr.k * wM * DM, s);
        UR.ensure(rows * tr.k, s);
        if (split) {
            // env = U^H T2 = (U^H) (T2^T)^T: U^H is k-contiguous as it stands, and T2^T is
            // split into planes straight from T2 (never formed in FP32)
            HIPCHK(adjoint_to_f32(U64.re(), U64.im(), rows, tr.k, (float*)UR.re(), (float*)UR.im(), s));
            const Lane ln = main_lane(st);
            const int terms = split_terms(st);
            const int64_t N = wM * DM;
            if (N > 0x7fffffff) fail(MPS_ERR_ARG, "GEMM dimension too large");
            unsigned short *pa, *pb;
            lane_planes(st, ln, tr.k, N, rows, pa, pb);
            {
                Timer t(st, MPS_KCLASS_OTHER, 0, (8.0 + 4.0 * terms) * ((double)tr.k + N) * rows, s);
                HIPCHK(split_planes(terms, tr.k, (int)rows, true, {(const float*)UR.re(), (const float*)UR.im(), rows},
                                    pa, s));
                HIPCHK(split_planes_t(terms, (int)N, (int)rows, false, {(const float*)T2.re(), (const float*)T2.im(), N},
                                      pb, s));
                t.done();
            }
            gemm_split_planes(st, MPS_KCLASS_CONTRACT, tr.k, N, rows, pa, pb, (float*)env[bM].re(),
                              (float*)env[bM].im(), N, ln);
            return;
        }
        HIPCHK((convert_planar<double, R>(U64.re(), U64.im(), rows * tr.k, UR.re(), UR.im(), s)));
        gemm<R>(st, MPS_KCLASS_CONTRACT, OP_C, OP_N, tr.k, wM * DM, rows, UR.re(), UR.im(), tr.k, T2.re(), T2.im(),
                wM * DM, env[bM].re(), env[bM].im(), wM * DM);
    }

    double zipup(int o) {
        double f0 = 0;
        for (int j = 0; j < n; ++j) {
            left_block(o, j);
            const int bL = bnd(o, j), bM = bnd(o, j + 1);
            const int64_t cL = cb[bL], wM = mpo.w[bM], DM = st->bond[bM];
            if (j == n - 1) {
                const int64_t sz = cL * 2;  // wM = DM = 1
                HIPCHK(norm2<R>(T2.re(), T2.im(), sz, st->partial.p, st->dscal.p + 1, s));
                HIPCHK(hipMemcpyAsync(&f0, st->dscal.p + 1, sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                if (!(f0 > 0) || !std::isfinite(f0)) fail(MPS_ERR_NUMERIC, "zip-up produced a zero or non-finite state");
                const int k0 = site(o, j);
                phi[k0].ensure(sz, s);
                HIPCHK((convert_planar<R, double>(T2.re(), T2.im(), sz, phi[k0].re(), phi[k0].im(), s)));
                set_scalar(0, 1.0 / std::sqrt(f0));
                HIPCHK(scale_by_device_scalar<double>(phi[k0].re(), phi[k0].im(), sz, st->dscal.p, s));
                cb[bM] = 1;
                log_step(f0, f0, (int)cL);
                break;
            }
            Trunc tr = truncate(T2.re(), T2.im(), 2 * cL, wM * DM, false, nullptr, nullptr, bM);
            finish_left(o, j, tr, true);
        }
        return f0;
    }

    void ensure_stream2() {
        if (st->stream2) return;
        HIPCHK(hipStreamCreateWithFlags(&st->stream2, hipStreamNonBlocking));
        for (auto& e : st->ev_order) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }

    // One directional pass in view o.  The local tensor of the pair (j, j+1)
    // is met in the middle: Theta = (L_j A_j W_j) . (A_{j+1} W_{j+1} R_{j+2})^T
    // contracted over the MPO bond and the psi bond between the pair
    // (rows (cL, s1), columns (cR, s2)).  The right block depends only on psi
    // and on right environments that this pass has not yet overwritten, so
    // the block of the next pair can be built on the second stream while the
    // current pair is truncated (overlap_right).
    double sweep(int o) {
        if (n < 2) return 0;
        ensure_stream2();
        const Lane l2 = st->overlap_right ? Lane{st->stream2, &st->splitws2, &st->planes2} : main_lane(st);
        hipEvent_t ev_start = st->ev_order[0], ev_used = st->ev_order[1];
        hipEvent_t ev_right[2] = {st->ev_order[2], st->ev_order[3]};
        HIPCHK(hipEventRecord(ev_start, s));
        HIPCHK(hipStreamWaitEvent(st->stream2, ev_start, 0));
        block(1 - o, n - 2, XR, T2R[0], l2);
        HIPCHK(hipEventRecord(ev_right[0], st->stream2));
        double f = 0;
        for (int j = 0; j + 1 < n; ++j) {
            const bool last = (j + 2 == n);
            left_block(o, j);
            const int bL = bnd(o, j), bM = bnd(o, j + 1), bR = bnd(o, j + 2);
            const int64_t cL = cb[bL], cR = cb[bR], wM = mpo.w[bM];
            const int64_t DM = st->bond[bM];
            const int64_t rows = 2 * cL, cols = 2 * cR, K = wM * DM;
            const Planar<R>& rb = T2R[j & 1];
            HIPCHK(hipStreamWaitEvent(s, ev_right[j & 1], 0));
            // Theta = T2 rb^T has rank <= K: when K < rows, cols (a bond that no gate of the layer
            // crosses, wM = 1, below saturation of the outer bonds) the truncation works on the
            // factors and Theta is never formed (the last pair needs Theta for its right factor)
            const bool lowrank = !last && K < rows && K < cols;
            if (!lowrank) {
                TH.ensure(rows * cols, s);
                TH64.ensure(rows * cols, s);
                if (split)
                    gemm_split(st, MPS_KCLASS_CONTRACT, rows, cols, K, (const float*)T2.re(), (const float*)T2.im(), K,
                               (const float*)rb.re(), (const float*)rb.im(), K, (float*)TH.re(), (float*)TH.im(), cols);
                else
                    gemm<R>(st, MPS_KCLASS_CONTRACT, OP_N, OP_T, rows, cols, K, T2.re(), T2.im(), K, rb.re(), rb.im(),
                            K, TH.re(), TH.im(), cols);
            }
            // The right block of the next pair is queued once this pair's tridiagonal
            // reduction (a whole-device cooperative launch) has finished: on the second
            // stream (overlap_right) it overlaps the rest of the truncation.
            bool queued = last;
            const std::function<void()> queue_right = [&, j]() {
                if (queued) return;
                queued = true;
                // buffer (j+1)&1 was last read by the previous pair's product
                HIPCHK(hipEventRecord(ev_used, s));
                HIPCHK(hipStreamWaitEvent(st->stream2, ev_used, 0));
                block(1 - o, n - 3 - j, XR, T2R[(j + 1) & 1], l2);
                HIPCHK(hipEventRecord(ev_right[(j + 1) & 1], st->stream2));
            };
            after_reduce = &queue_right;
            Trunc tr;
            if (lowrank) {
                tr = truncate_lowrank(T2.re(), T2.im(), rb.re(), rb.im(), rows, cols, K, bM);
            } else {
                HIPCHK((convert_planar<R, double>(TH.re(), TH.im(), rows * cols, TH64.re(), TH64.im(), s)));
                tr = truncate(TH.re(), TH.im(), rows, cols, last, TH64.re(), TH64.im(), bM);
            }
            after_reduce = nullptr;
            queue_right();          // no-op when the truncation already queued it
            f = tr.f;
            if (f > 1.0 + 1e-3) fail(MPS_ERR_NUMERIC, "partial fidelity above 1: " + std::to_string(f));
            finish_left(o, j, tr, !last);
            if (last) {
                // cR = 1 at the end of the chain: the column order (cR, s2) is the site layout [k][s2]
                const int k1 = site(o, j + 1);
                phi[k1].ensure((int64_t)tr.k * cols, s);
                HIPCHK((convert_planar<double, double>(V64.re(), V64.im(), (int64_t)tr.k * cols, phi[k1].re(),
                                                       phi[k1].im(), s)));
            }
            log_step(tr.f, tr.total, tr.k);
        }
        return f;
    }

    // Single-site pass in view o (the paper's update with one free tensor):
    // F_j = (L_j A_j W_j) R_{j+1}^T over the MPO bond and the psi bond right of
    // site j (rows (cL, s), columns cR), f = |F|^2, M = F / sqrt(f); the centre
    // moves right by an FP64 QR of M.  Bond dimensions can only shrink (when
    // 2 cL < cR).  The last site keeps M.
    double sweep_single(int o) {
        double f = 0;
        for (int j = 0; j < n; ++j) {
            left_block(o, j);
            const int bL = bnd(o, j), bM = bnd(o, j + 1);
            const int64_t cL = cb[bL], cM = cb[bM], wM = mpo.w[bM], DM = st->bond[bM];
            const int64_t rows = 2 * cL, K = wM * DM;
            TH.ensure(rows * cM, s);
            TH64.ensure(rows * cM, s);
            if (split)
                gemm_split(st, MPS_KCLASS_CONTRACT, rows, cM, K, (const float*)T2.re(), (const float*)T2.im(), K,
                           (const float*)env[bM].re(), (const float*)env[bM].im(), K, (float*)TH.re(),
                           (float*)TH.im(), cM);
            else
                gemm<R>(st, MPS_KCLASS_CONTRACT, OP_N, OP_T, rows, cM, K, T2.re(), T2.im(), K, env[bM].re(),
                        env[bM].im(), K, TH.re(), TH.im(), cM);
            HIPCHK((convert_planar<R, double>(TH.re(), TH.im(), rows * cM, TH64.re(), TH64.im(), s)));
            HIPCHK(norm2<double>(TH64.re(), TH64.im(), rows * cM, st->partial.p, st->dscal.p + 1, s));
            HIPCHK(hipMemcpyAsync(&f, st->dscal.p + 1, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (!(f > 0) || !std::isfinite(f)) fail(MPS_ERR_NUMERIC, "local tensor has zero or non-finite norm");
            if (f > 1.0 + 1e-3) fail(MPS_ERR_NUMERIC, "partial fidelity above 1: " + std::to_string(f));
            if (j == n - 1) {
                const int k0 = site(o, j);
                phi[k0].ensure(rows * cM, s);
                HIPCHK((convert_planar<double, double>(TH64.re(), TH64.im(), rows * cM, phi[k0].re(), phi[k0].im(), s)));
                set_scalar(0, 1.0 / std::sqrt(f));
                HIPCHK(scale_by_device_scalar<double>(phi[k0].re(), phi[k0].im(), rows * cM, st->dscal.p, s));
                log_step(f, f, (int)cM);
                break;
            }
            const int k = qr_orth(rows, cM, TH64.re(), TH64.im());
            finish_left(o, j, Trunc{k, f, f, true}, true);
            log_step(f, f, k);
        }
        return f;
    }

    void log_step(double f, double s2, int k) {
        st->log_step_f.push_back(f);
        st->log_step_s2.push_back(s2);
        st->log_step_chi.push_back(k);
    }

    bool single_site = false;

    double run(const mps_gate* gates, const int* n_gates, int n_layers, int n_sweeps) {
        mpo = build_step_mpo(n, gates, n_gates, n_layers);
        setup();
        const int oz = st->center == 0 ? 0 : 1;
        double f = zipup(oz);
        int last = oz;
        if (n >= 2) {
            int o = 1 - oz;
            for (int sw = 0; sw < n_sweeps; ++sw) {
                f = single_site ? sweep_single(o) : sweep(o);
                last = o;
                o = 1 - o;
            }
        }
        HIPCHK(hipStreamSynchronize(s));
        // commit
        for (auto& t : st->ten) t.release(s);
        st->ten.swap(phi);
        phi.clear();
        st->bond = cb;
        st->orient = last;
        st->center = last == 0 ? n - 1 : 0;
        st->n_2q += mpo.n_2q;
        return f;
    }
};

// Forward-layout FP64 copy of site k into dst ([D_k][2][D_k+1]), on `on`
// (default: the state's stream).
void forward_tensor(const mps_state* st, int k, Planar<double>& dst, hipStream_t on = nullptr) {
    const hipStream_t s = on ? on : st->stream;
    const int64_t sz = (int64_t)st->bond[k] * 2 * st->bond[k + 1];
    dst.ensure(sz, s);
    const int Dl = st->orient == 0 ? st->bond[k] : st->bond[k + 1];
    const int Dr = st->orient == 0 ? st->bond[k + 1] : st->bond[k];
    HIPCHK(site_to_view<double>(st->ten[k].re(), st->ten[k].im(), Dl, Dr, st->orient, dst.re(), dst.im(), s));
}

mps_status run_guarded(const std::function<void()>& fn) {
    mps_status code = MPS_OK;
    try {
        fn();
        g_last_error.clear();
    } catch (const MpsFail& e) {
        g_last_error = e.msg;
        code = e.code;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        code = MPS_ERR_DEVICE;
    }
    g_alloc = nullptr;
    return code;
}

// Argument check of a state; device memory of the call comes from its allocator.
void check_state(const mps_state* st) {
    if (!st) fail(MPS_ERR_ARG, "state is NULL");
    if (st->invalid) fail(MPS_ERR_STATE, "state was invalidated by an earlier failure");
    g_alloc = st->has_alloc ? &st->alloc : nullptr;
}


// One compression step over n_layers consecutive layers (n_gates[l] records each).
void apply_step_impl(mps_state* st, const mps_gate* gates, const int* n_gates, int n_layers, int chi, int n_sweeps,
                     double* f_layer, bool single_site, const int* chi_bond = nullptr) {
    check_state(st);
    if (chi_bond) {
        chi = 1;
        for (int c = 1; c < st->n; ++c) {
            if (chi_bond[c] < 1 || chi_bond[c] > st->max_chi) fail(MPS_ERR_ARG, "chi_bond entries must be in [1, max_chi]");
            chi = std::max(chi, chi_bond[c]);
        }
    }
    if (n_layers < 1 || n_layers > 64) fail(MPS_ERR_ARG, "n_layers must be in [1, 64]");
    if (!n_gates) fail(MPS_ERR_ARG, "n_gates is NULL");
    int64_t total = 0;
    for (int l = 0; l < n_layers; ++l) {
        if (n_gates[l] < 0) fail(MPS_ERR_ARG, "negative gate count");
        total += n_gates[l];
    }
    if (total > 0 && !gates) fail(MPS_ERR_ARG, "gates is NULL");
    if (chi < 1 || chi > st->max_chi) fail(MPS_ERR_ARG, "chi must be in [1, max_chi]");
    if (n_sweeps < 0) fail(MPS_ERR_ARG, "n_sweeps must be >= 0");
    // argument validation happens in the MPO build, before any device work
    (void)build_step_mpo(st->n, gates, n_gates, n_layers);
    const size_t log_mark = st->log_step_f.size();
    st->cur_min_sep = HUGE_VAL;
    double f = 0;
    try {
        if (st->prec == MPS_FP32 || is_split(st->prec)) {
            Engine<float> e(st, chi);
            e.split = is_split(st->prec);
            e.single_site = single_site;
            if (chi_bond) e.chi_bond.assign(chi_bond, chi_bond + st->n + 1);
            f = e.run(gates, n_gates, n_layers, n_sweeps);
        } else {
            Engine<double> e(st, chi);
            e.single_site = single_site;
            if (chi_bond) e.chi_bond.assign(chi_bond, chi_bond + st->n + 1);
            f = e.run(gates, n_gates, n_layers, n_sweeps);
        }
        HIPCHK(hipStreamSynchronize(st->stream));
        if (!(f > 0) || !std::isfinite(f)) fail(MPS_ERR_NUMERIC, "non-positive layer fidelity");
    } catch (const MpsFail& e) {
        st->invalid = true;
        st->log_step_f.resize(log_mark);
        st->log_step_s2.resize(log_mark);
        st->log_step_chi.resize(log_mark);
        (void)hipStreamSynchronize(st->stream);
        throw;
    }
    flush_timings(st);
    st->log_f += std::log(f);
    st->log_step_sep.push_back(st->cur_min_sep);
    st->n_layers += n_layers;
    if (f_layer) *f_layer = f;
}

void apply_layer_impl(mps_state* st, const mps_gate* gates, int n_gates, int chi, int n_sweeps, double* f_layer,
                      bool single_site = false) {
    apply_step_impl(st, gates, &n_gates, 1, chi, n_sweeps, f_layer, single_site);
}

}  // namespace

// ================================================================= C ABI ===
extern "C" {

const char* mps_last_error(void) { return g_last_error.c_str(); }

mps_status mps_create(int n_sites, const uint8_t* init_bits, int max_chi, int precision, void* hip_stream,
                      const mps_allocator* alloc, mps_state** out) {
    return run_guarded([&] {
        if (!out) fail(MPS_ERR_ARG, "out is NULL");
        *out = nullptr;
        if (n_sites < 1 || n_sites > 4096) fail(MPS_ERR_ARG, "n_sites must be in [1, 4096]");
        if (max_chi < 1) fail(MPS_ERR_ARG, "max_chi must be >= 1");
        if (precision != MPS_FP64 && precision != MPS_FP32 && !is_split(precision))
            fail(MPS_ERR_ARG, "unknown precision");
        if (alloc && (!alloc->alloc || !alloc->free)) fail(MPS_ERR_ARG, "allocator callbacks must be non-NULL");
        if (init_bits)
            for (int k = 0; k < n_sites; ++k)
                if (init_bits[k] > 1) fail(MPS_ERR_ARG, "init_bits must be 0 or 1");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(MPS_ERR_DEVICE, "no HIP device available");
        mps_state* st = new mps_state();
        st->n = n_sites;
        st->max_chi = max_chi;
        st->prec = precision;
        st->stream = (hipStream_t)hip_stream;
        if (alloc) {
            st->alloc = *alloc;
            st->has_alloc = true;
            g_alloc = &st->alloc;
        }
        if (const char* em = std::getenv("MPS_EIGENSOLVER"))
            st->eigh_method = std::strcmp(em, "rocsolver") == 0 ? EIGH_ROCSOLVER : EIGH_PERSISTENT;
        if (const char* ov = std::getenv("MPS_OVERLAP")) st->overlap_right = std::strcmp(ov, "0") != 0;
        try {
            if (rocblas_create_handle(&st->blas) != rocblas_status_success) fail(MPS_ERR_DEVICE, "rocblas_create_handle failed");
            rocblas_set_stream(st->blas, st->stream);
            st->dscal.ensure(16, st->stream);
            st->partial.ensure(1024, st->stream);
            st->bond.assign(n_sites + 1, 1);
            st->ten.resize(n_sites);
            for (int k = 0; k < n_sites; ++k) {
                st->ten[k].ensure(2, st->stream);
                const int b = init_bits ? init_bits[k] : 0;
                const double re[2] = {b == 0 ? 1.0 : 0.0, b == 1 ? 1.0 : 0.0}, im[2] = {0.0, 0.0};
                HIPCHK(hipMemcpyAsync(st->ten[k].re(), re, sizeof(re), hipMemcpyHostToDevice, st->stream));
                HIPCHK(hipMemcpyAsync(st->ten[k].im(), im, sizeof(im), hipMemcpyHostToDevice, st->stream));
                HIPCHK(hipStreamSynchronize(st->stream));
            }
        } catch (...) {
            mps_destroy(st);
            throw;
        }
        *out = st;
    });
}

mps_status mps_destroy(mps_state* st) {
    if (!st) return MPS_OK;
    g_alloc = st->has_alloc ? &st->alloc : nullptr;
    (void)hipStreamSynchronize(st->stream);
    if (st->stream2) (void)hipStreamSynchronize(st->stream2);
    for (auto& t : st->ten) t.release(st->stream);
    st->dscal.release(st->stream);
    st->partial.release(st->stream);
    st->splitws.release(st->stream);
    st->planes.release(st->stream);
    st->splitws64.release(st->stream);
    if (st->stream2) {
        st->splitws2.release(st->stream2);
        st->planes2.release(st->stream2);
        (void)hipStreamSynchronize(st->stream2);
        (void)hipStreamDestroy(st->stream2);
        st->stream2 = nullptr;
    }
    for (auto& e : st->ev_order)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    for (auto& p : st->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    st->pending.clear();
    for (auto e : st->event_pool) (void)hipEventDestroy(e);
    st->event_pool.clear();
    if (st->blas) rocblas_destroy_handle(st->blas);
    st->blas = nullptr;
    (void)hipStreamSynchronize(st->stream);
    if (!st->has_alloc) {
        // return what the default pool cached for this state's frees to the device
        int dev = 0;
        hipMemPool_t pool = nullptr;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool)
            (void)hipMemPoolTrimTo(pool, 0);
    }
    (void)hipGetLastError();
    g_alloc = nullptr;
    delete st;
    return MPS_OK;
}

mps_status apply_layer_dmrg(mps_state* st, const mps_gate* gates, int n_gates, int chi, int n_sweeps,
                            double* f_layer) {
    return run_guarded([&] { apply_layer_impl(st, gates, n_gates, chi, n_sweeps, f_layer); });
}

mps_status apply_layer_dmrg_single_site(mps_state* st, const mps_gate* gates, int n_gates, int chi, int n_sweeps,
                            double* f_layer) {
    return run_guarded([&] { apply_layer_impl(st, gates, n_gates, chi, n_sweeps, f_layer, true); });
}

mps_status apply_layers_dmrg(mps_state* st, const mps_gate* gates, const int* n_gates, int n_layers, int chi,
                             int n_sweeps, int update, double* f_step) {
    return run_guarded([&] {
        if (update != MPS_UPDATE_TWO_SITE && update != MPS_UPDATE_SINGLE_SITE) fail(MPS_ERR_ARG, "unknown update rule");
        apply_step_impl(st, gates, n_gates, n_layers, chi, n_sweeps, f_step, update == MPS_UPDATE_SINGLE_SITE);
    });
}

mps_status apply_layers_dmrg_bonds(mps_state* st, const mps_gate* gates, const int* n_gates, int n_layers,
                                   const int* chi_bond, int n_sweeps, int update, double* f_step) {
    return run_guarded([&] {
        if (update != MPS_UPDATE_TWO_SITE && update != MPS_UPDATE_SINGLE_SITE) fail(MPS_ERR_ARG, "unknown update rule");
        if (!chi_bond) fail(MPS_ERR_ARG, "chi_bond is NULL");
        apply_step_impl(st, gates, n_gates, n_layers, 1, n_sweeps, f_step, update == MPS_UPDATE_SINGLE_SITE, chi_bond);
    });
}

mps_status apply_layer_dmrg_batched(mps_state* const* states, int batch, const mps_gate* const* gates,
                                    const int* n_gates, const int* chi, int n_sweeps, double* f_layers) {
    return run_guarded([&] {
        if (batch < 0) fail(MPS_ERR_ARG, "batch must be >= 0");
        if (batch == 0) return;
        if (!states || !gates || !n_gates || !chi) fail(MPS_ERR_ARG, "NULL batched argument");
        for (int i = 0; i < batch; ++i) {
            if (!states[i]) fail(MPS_ERR_ARG, "states[" + std::to_string(i) + "] is NULL");
            for (int j = 0; j < i; ++j)
                if (states[j] == states[i]) fail(MPS_ERR_ARG, "a state appears twice in the batch");
        }
        // argument checks of every instance before any device work
        for (int i = 0; i < batch; ++i) {
            check_state(states[i]);
            if (n_gates[i] < 0 || (n_gates[i] > 0 && !gates[i])) fail(MPS_ERR_ARG, "bad gates of instance " + std::to_string(i));
            if (chi[i] < 1 || chi[i] > states[i]->max_chi) fail(MPS_ERR_ARG, "bad chi of instance " + std::to_string(i));
            (void)build_layer_mpo(states[i]->n, gates[i], n_gates[i]);
        }
        if (n_sweeps < 0) fail(MPS_ERR_ARG, "n_sweeps must be >= 0");
        // one host thread per concurrently driven instance; each instance runs on its own
        // stream, and their persistent tridiagonal reductions are gathered into shared launches
        const int n_threads = std::max(1, std::min(batch, 8));
        std::vector<mps_status> status(batch, MPS_OK);
        std::vector<std::string> msg(batch);
        std::vector<std::thread> pool;
        std::atomic<int> next(0);
        TridiagBatcher batcher;
        batcher.active = n_threads;
        for (int t = 0; t < n_threads; ++t)
            pool.emplace_back([&] {
                g_batcher = &batcher;
                for (int i = next.fetch_add(1); i < batch; i = next.fetch_add(1)) {
                    double f = 0;
                    status[i] = run_guarded([&] { apply_layer_impl(states[i], gates[i], n_gates[i], chi[i], n_sweeps, &f); });
                    if (status[i] != MPS_OK) msg[i] = g_last_error;
                    if (f_layers) f_layers[i] = f;
                }
                g_batcher = nullptr;
                batcher.worker_done();
            });
        for (auto& th : pool) th.join();
        g_batch_stats.launches += batcher.launches;
        g_batch_stats.reductions += batcher.reductions;
        for (int i = 0; i < batch; ++i)
            if (status[i] != MPS_OK) fail(status[i], "instance " + std::to_string(i) + ": " + msg[i]);
    });
}

mps_status fidelity(const mps_state* st, double* F_tilde, double* log_F_tilde, int* n_layers, int64_t* n_2q) {
    return run_guarded([&] {
        check_state(st);
        if (F_tilde) *F_tilde = std::exp(st->log_f);
        if (log_F_tilde) *log_F_tilde = st->log_f;
        if (n_layers) *n_layers = st->n_layers;
        if (n_2q) *n_2q = st->n_2q;
    });
}

mps_status mps_bond_dims(const mps_state* st, int* dims) {
    return run_guarded([&] {
        check_state(st);
        if (!dims) fail(MPS_ERR_ARG, "dims is NULL");
        for (int c = 0; c <= st->n; ++c) dims[c] = st->bond[c];
    });
}

mps_status mps_get_tensor(const mps_state* st, int site, double* re_im) {
    return run_guarded([&] {
        check_state(st);
        if (site < 0 || site >= st->n || !re_im) fail(MPS_ERR_ARG, "bad site or NULL output");
        Planar<double> tmp;
        forward_tensor(st, site, tmp);
        const int64_t sz = (int64_t)st->bond[site] * 2 * st->bond[site + 1];
        std::vector<double> h(2 * sz);
        HIPCHK(hipMemcpyAsync(h.data(), tmp.p, sizeof(double) * sz, hipMemcpyDeviceToHost, st->stream));
        HIPCHK(hipMemcpyAsync(h.data() + sz, tmp.p + tmp.cap, sizeof(double) * sz, hipMemcpyDeviceToHost, st->stream));
        HIPCHK(hipStreamSynchronize(st->stream));
        tmp.release(st->stream);
        for (int64_t i = 0; i < sz; ++i) {
            re_im[2 * i] = h[i];
            re_im[2 * i + 1] = h[sz + i];
        }
    });
}

mps_status mps_step_log(const mps_state* st, double* f, double* sum_s2, int* chi_kept, int cap, int* n) {
    return run_guarded([&] {
        if (!st) fail(MPS_ERR_ARG, "state is NULL");
        const int total = (int)st->log_step_f.size();
        if (n) *n = total;
        const int m = std::min(cap, total);
        for (int i = 0; i < m; ++i) {
            if (f) f[i] = st->log_step_f[i];
            if (sum_s2) sum_s2[i] = st->log_step_s2[i];
            if (chi_kept) chi_kept[i] = st->log_step_chi[i];
        }
    });
}

mps_status mps_cut_separations(const mps_state* st, double* sep, int cap, int* n) {
    return run_guarded([&] {
        if (!st) fail(MPS_ERR_ARG, "state is NULL");
        const int total = (int)st->log_step_sep.size();
        if (n) *n = total;
        for (int i = 0; i < std::min(cap, total); ++i)
            if (sep) sep[i] = st->log_step_sep[i];
    });
}

mps_status mps_to_statevector(const mps_state* st_c, double* re_im) {
    return run_guarded([&] {
        check_state(st_c);
        mps_state* st = const_cast<mps_state*>(st_c);
        if (!re_im) fail(MPS_ERR_ARG, "output is NULL");
        if (st->n > 26) fail(MPS_ERR_ARG, "statevector limited to n <= 26");
        const hipStream_t s = st->stream;
        // rows x (2 D_{k+1}) intermediate; bonds may exceed 2^min(c, n-c) after a zip-up-only layer
        int64_t need = (int64_t)1 << st->n;
        for (int k = 0; k < st->n; ++k) need = std::max<int64_t>(need, ((int64_t)2 << k) * st->bond[k + 1]);
        if (need > ((int64_t)1 << 31)) fail(MPS_ERR_ARG, "statevector intermediate too large");
        Planar<double> v, w, a;
        v.ensure(need, s);
        w.ensure(need, s);
        HIPCHK(fill_planar<double>(v.re(), v.im(), 1, 1.0, s));
        int64_t rows = 1;
        for (int k = 0; k < st->n; ++k) {
            forward_tensor(st, k, a);
            const int64_t Dk = st->bond[k], Dn = st->bond[k + 1];
            gemm<double>(st, MPS_KCLASS_OTHER, OP_N, OP_N, rows, 2 * Dn, Dk, v.re(), v.im(), Dk, a.re(), a.im(),
                         2 * Dn, w.re(), w.im(), 2 * Dn);
            std::swap(v, w);
            rows *= 2;
        }
        const int64_t N = (int64_t)1 << st->n;
        std::vector<double> h(2 * N);
        HIPCHK(hipMemcpyAsync(h.data(), v.re(), sizeof(double) * N, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h.data() + N, v.im(), sizeof(double) * N, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int64_t i = 0; i < N; ++i) {
            re_im[2 * i] = h[i];
            re_im[2 * i + 1] = h[N + i];
        }
        v.release(s); w.release(s); a.release(s);
        flush_timings(st);
    });
}

mps_status mps_amplitude(const mps_state* st_c, int n_strings, const uint8_t* bits, double* re_im) {
    return run_guarded([&] {
        check_state(st_c);
        mps_state* st = const_cast<mps_state*>(st_c);
        if (n_strings < 0 || (n_strings > 0 && (!bits || !re_im))) fail(MPS_ERR_ARG, "bad amplitude arguments");
        if (n_strings == 0) return;
        const int n = st->n;
        for (int64_t i = 0; i < (int64_t)n_strings * n; ++i)
            if (bits[i] > 1) fail(MPS_ERR_ARG, "bits must be 0 or 1");
        const hipStream_t s = st->stream;
        int maxD = 1;
        for (int c = 0; c <= n; ++c) maxD = std::max(maxD, st->bond[c]);
        // strings are evaluated in chunks that keep the two row buffers under ~1.5 GiB
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_strings, ((int64_t)1 << 26) / maxD));
        Planar<double> v, u, a;
        v.ensure(chunk * maxD, s);
        u.ensure(chunk * 2 * maxD, s);
        Raw<uint8_t> bdev;
        bdev.ensure(chunk, s);
        std::vector<uint8_t> col(chunk);
        std::vector<double> h(2 * chunk);
        for (int64_t s0 = 0; s0 < n_strings; s0 += chunk) {
            const int64_t S = std::min<int64_t>(chunk, n_strings - s0);
            HIPCHK(fill_planar<double>(v.re(), v.im(), S, 1.0, s));
            for (int k = 0; k < n; ++k) {
                forward_tensor(st, k, a);
                const int64_t Dk = st->bond[k], Dn = st->bond[k + 1];
                gemm<double>(st, MPS_KCLASS_OTHER, OP_N, OP_N, S, 2 * Dn, Dk, v.re(), v.im(), Dk, a.re(), a.im(),
                             2 * Dn, u.re(), u.im(), 2 * Dn);
                for (int64_t r = 0; r < S; ++r) col[r] = bits[(s0 + r) * n + k];
                HIPCHK(hipMemcpyAsync(bdev.p, col.data(), S, hipMemcpyHostToDevice, s));
                HIPCHK(select_rows<double>(u.re(), u.im(), S, (int)Dn, 0, bdev.p, 0, 0, k, v.re(), v.im(), nullptr, s));
                HIPCHK(hipStreamSynchronize(s));
            }
            HIPCHK(hipMemcpyAsync(h.data(), v.re(), sizeof(double) * S, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(h.data() + S, v.im(), sizeof(double) * S, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int64_t r = 0; r < S; ++r) {
                re_im[2 * (s0 + r)] = h[r];
                re_im[2 * (s0 + r) + 1] = h[S + r];
            }
        }
        v.release(s); u.release(s); a.release(s); bdev.release(s);
        flush_timings(st);
    });
}

}  // extern "C"

namespace {

template <typename R>
void sample_impl(mps_state* st, int64_t n_samples, uint64_t seed, uint64_t* out, bool split = false) {
    const int n = st->n;
    const hipStream_t s = st->stream;
    const int words = (n + 63) / 64;
    std::memset(out, 0, sizeof(uint64_t) * words * n_samples);
    // the view whose site 0 is the orthogonality centre: tensors there are right isometries
    const int oc = st->center == 0 ? 0 : 1;
    int maxD = 1;
    for (int c = 0; c <= n; ++c) maxD = std::max(maxD, st->bond[c]);
    const int64_t chunk = std::min<int64_t>(n_samples, std::max<int64_t>(1024, (int64_t)(1 << 26) / (2 * maxD)));
    std::vector<Planar<R>> views(n);
    for (int j = 0; j < n; ++j) {
        const int k = oc == 0 ? j : n - 1 - j;
        views[j].ensure((int64_t)st->bond[k] * 2 * st->bond[k + 1], s);
        const int Dl = st->orient == 0 ? st->bond[k] : st->bond[k + 1];
        const int Dr = st->orient == 0 ? st->bond[k + 1] : st->bond[k];
        if (split) {
            const int Dlv = st->orient != oc ? Dr : Dl, Drv = st->orient != oc ? Dl : Dr;
            HIPCHK(site_to_kmajor(st->ten[k].re(), st->ten[k].im(), Dlv, Drv, st->orient != oc ? 1 : 0,
                                  (float*)views[j].re(), (float*)views[j].im(), s));
        } else {
            HIPCHK(site_to_view<R>(st->ten[k].re(), st->ten[k].im(), Dl, Dr, st->orient != oc ? 1 : 0,
                                   views[j].re(), views[j].im(), s));
        }
    }
    Planar<R> v, u;
    v.ensure(chunk * maxD, s);
    u.ensure(chunk * 2 * maxD, s);
    Raw<uint8_t> bdev;
    bdev.ensure(chunk * n, s);
    std::vector<uint8_t> hb(chunk * n);
    for (int64_t s0 = 0; s0 < n_samples; s0 += chunk) {
        const int64_t S = std::min(chunk, n_samples - s0);
        HIPCHK(fill_planar<R>(v.re(), v.im(), S, 1.0, s));
        for (int j = 0; j < n; ++j) {
            const int k = oc == 0 ? j : n - 1 - j;
            const int64_t Dv = oc == 0 ? st->bond[k] : st->bond[k + 1];
            const int64_t Dn = oc == 0 ? st->bond[k + 1] : st->bond[k];
            if (split)
                gemm_split(st, MPS_KCLASS_CONTRACT, S, 2 * Dn, Dv, (const float*)v.re(), (const float*)v.im(), Dv,
                           (const float*)views[j].re(), (const float*)views[j].im(), Dv, (float*)u.re(),
                           (float*)u.im(), 2 * Dn);
            else
                gemm<R>(st, MPS_KCLASS_CONTRACT, OP_N, OP_N, S, 2 * Dn, Dv, v.re(), v.im(), Dv, views[j].re(),
                        views[j].im(), 2 * Dn, u.re(), u.im(), 2 * Dn);
            Timer t(st, MPS_KCLASS_OTHER, 0, 3.0 * sizeof(R) * S * 2 * Dn);
            HIPCHK(select_rows<R>(u.re(), u.im(), S, (int)Dn, 1, nullptr, seed, s0, k, v.re(), v.im(),
                                  bdev.p + (int64_t)k * S, s));
            t.done();
        }
        HIPCHK(hipMemcpyAsync(hb.data(), bdev.p, (size_t)S * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < n; ++k)
            for (int64_t r = 0; r < S; ++r)
                if (hb[(size_t)k * S + r]) out[(s0 + r) * words + k / 64] |= (uint64_t)1 << (k % 64);
    }
    for (auto& vv : views) vv.release(s);
    v.release(s); u.release(s); bdev.release(s);
    flush_timings(st);
}

}  // namespace

extern "C" {

mps_status sample(mps_state* st, int64_t n_samples, uint64_t seed, uint64_t* bits) {
    return run_guarded([&] {
        check_state(st);
        if (n_samples < 0 || (n_samples > 0 && !bits)) fail(MPS_ERR_ARG, "bad sample arguments");
        if (n_samples == 0) return;
        if (st->prec == MPS_FP32) sample_impl<float>(st, n_samples, seed, bits);
        else if (is_split(st->prec)) sample_impl<float>(st, n_samples, seed, bits, true);
        else sample_impl<double>(st, n_samples, seed, bits);
    });
}

mps_status mps_batch_stats(int64_t* launches, int64_t* reductions) {
    return run_guarded([&] {
        if (launches) *launches = g_batch_stats.launches.load();
        if (reductions) *reductions = g_batch_stats.reductions.load();
    });
}

mps_status mps_eigensolver_counts(const mps_state* st, int64_t* counts) {
    return run_guarded([&] {
        if (!st) fail(MPS_ERR_ARG, "state is NULL");
        if (!counts) fail(MPS_ERR_ARG, "counts is NULL");
        for (int i = 0; i < 4; ++i) counts[i] = st->eig_count[i];
    });
}

mps_status mps_expect_zz(const mps_state* st_c, int i, int j, double* value) {
    return run_guarded([&] {
        check_state(st_c);
        mps_state* st = const_cast<mps_state*>(st_c);
        if (i < 0 || j < 0 || i >= st->n || j >= st->n || !value) fail(MPS_ERR_ARG, "bad site or NULL output");
        const hipStream_t s = st->stream;
        int maxD = 1;
        for (int c = 0; c <= st->n; ++c) maxD = std::max(maxD, st->bond[c]);
        Planar<double> e, x, a, az;
        e.ensure((int64_t)maxD * maxD, s);
        x.ensure((int64_t)maxD * 2 * maxD, s);
        az.ensure((int64_t)maxD * 2 * maxD, s);
        HIPCHK(fill_planar<double>(e.re(), e.im(), 1, 1.0, s));
        for (int k = 0; k < st->n; ++k) {
            forward_tensor(st, k, a);
            const int64_t Dk = st->bond[k], Dn = st->bond[k + 1];
            gemm<double>(st, MPS_KCLASS_OTHER, OP_N, OP_N, Dk, 2 * Dn, Dk, e.re(), e.im(), Dk, a.re(), a.im(), 2 * Dn,
                         x.re(), x.im(), 2 * Dn);
            const double* xr = x.re();
            const double* xi = x.im();
            if (k == i || k == j) {
                HIPCHK(apply_z_phys(x.re(), x.im(), (int)Dk, (int)Dn, az.re(), az.im(), s));
                xr = az.re();
                xi = az.im();
            }
            gemm<double>(st, MPS_KCLASS_OTHER, OP_C, OP_N, Dn, Dn, 2 * Dk, a.re(), a.im(), Dn, xr, xi, Dn, e.re(),
                         e.im(), Dn);
        }
        double v = 0;
        HIPCHK(hipMemcpyAsync(&v, e.re(), sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *value = v;
        e.release(s); x.release(s); a.release(s); az.release(s);
        flush_timings(st);
    });
}

mps_status mps_overlap(const mps_state* bra_c, const mps_state* ket_c, double* re, double* im) {
    return run_guarded([&] {
        check_state(bra_c);
        check_state(ket_c);
        if (!re || !im) fail(MPS_ERR_ARG, "NULL output");
        if (bra_c->n != ket_c->n) fail(MPS_ERR_ARG, "the states have different numbers of sites");
        mps_state* ket = const_cast<mps_state*>(ket_c);
        const mps_state* bra = bra_c;
        // transfer matrices E_{k+1} = sum_s B_k[:, s, :]^H E_k A_k[:, s, :] on the ket's stream
        HIPCHK(hipStreamSynchronize(bra->stream));
        const hipStream_t s = ket->stream;
        int maxB = 1, maxK = 1;
        for (int c = 0; c <= ket->n; ++c) {
            maxB = std::max(maxB, bra->bond[c]);
            maxK = std::max(maxK, ket->bond[c]);
        }
        Planar<double> e, x, a, b;
        e.ensure((int64_t)maxB * maxK, s);
        x.ensure((int64_t)maxB * 2 * maxK, s);
        HIPCHK(fill_planar<double>(e.re(), e.im(), 1, 1.0, s));
        for (int k = 0; k < ket->n; ++k) {
            forward_tensor(ket, k, a, s);
            forward_tensor(bra, k, b, s);
            const int64_t Bk = bra->bond[k], Bn = bra->bond[k + 1], Kk = ket->bond[k], Kn = ket->bond[k + 1];
            gemm<double>(ket, MPS_KCLASS_OTHER, OP_N, OP_N, Bk, 2 * Kn, Kk, e.re(), e.im(), Kk, a.re(), a.im(), 2 * Kn,
                         x.re(), x.im(), 2 * Kn);
            gemm<double>(ket, MPS_KCLASS_OTHER, OP_C, OP_N, Bn, Kn, 2 * Bk, b.re(), b.im(), Bn, x.re(), x.im(), Kn,
                         e.re(), e.im(), Kn);
        }
        double v[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(&v[0], e.re(), sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&v[1], e.im(), sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *re = v[0];
        *im = v[1];
        e.release(s); x.release(s); a.release(s); b.release(s);
        HIPCHK(hipStreamSynchronize(s));
        flush_timings(ket);
    });
}

mps_status mps_overlap_layers(const mps_state* bra_c, mps_state* ket, const mps_gate* gates, const int* n_gates,
                              int n_layers, double* re, double* im) {
    if (n_layers == 0) return mps_overlap(bra_c, ket, re, im);
    return run_guarded([&] {
        check_state(bra_c);
        check_state(ket);
        if (!re || !im) fail(MPS_ERR_ARG, "NULL output");
        if (bra_c->n != ket->n) fail(MPS_ERR_ARG, "the states have different numbers of sites");
        if (n_layers < 0 || n_layers > 64) fail(MPS_ERR_ARG, "n_layers must be in [0, 64]");
        if (!n_gates) fail(MPS_ERR_ARG, "n_gates is NULL");
        int64_t total = 0;
        for (int l = 0; l < n_layers; ++l) {
            if (n_gates[l] < 0) fail(MPS_ERR_ARG, "negative gate count");
            total += n_gates[l];
        }
        if (total > 0 && !gates) fail(MPS_ERR_ARG, "gates is NULL");
        const mps_state* bra = bra_c;
        const int n = ket->n;
        LayerMpo mpo = build_step_mpo(n, gates, n_gates, n_layers);      // validates the gates
        for (int c = 0; c <= n; ++c) {
            const double env = (double)bra->bond[c] * (double)mpo.w[c] * (double)ket->bond[c];
            if (env > (double)(1LL << 31))
                fail(MPS_ERR_ARG, "the middle layers are too wide: an environment of " + std::to_string(env) +
                                      " complex values at bond " + std::to_string(c));
        }
        HIPCHK(hipStreamSynchronize(bra->stream));
        const hipStream_t s = ket->stream;
        {
            // the left-environment recursion of the compression step with the bra as the
            // fitted state: E_{j+1} = B_j^H (E_j A_j W_j), FP64 contractions
            Engine<double> e(ket, 1);
            e.mpo = std::move(mpo);
            e.setup();
            for (int c = 0; c <= n; ++c) e.cb[c] = bra->bond[c];
            for (int j = 0; j < n; ++j) {
                e.left_block(0, j);
                forward_tensor(bra, j, e.U64, s);
                e.finish_left(0, j, typename Engine<double>::Trunc{bra->bond[j + 1], 0.0, 0.0, true}, true);
            }
            double v[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(&v[0], e.env[n].re(), sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&v[1], e.env[n].im(), sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            *re = v[0];
            *im = v[1];
        }
        HIPCHK(hipStreamSynchronize(s));
        flush_timings(ket);
    });
}

mps_status mps_set_profiling(mps_state* st, int on) {
    return run_guarded([&] {
        if (!st) fail(MPS_ERR_ARG, "state is NULL");
        flush_timings(st);
        st->prof = on != 0;
        for (auto& k : st->stats) k = KStat();
    });
}

mps_status mps_kernel_stats(const mps_state* st, int cls, int64_t* launches, double* total_ms, double* flops,
                            double* bytes) {
    return run_guarded([&] {
        if (!st) fail(MPS_ERR_ARG, "state is NULL");
        if (cls < 0 || cls >= MPS_KCLASS_COUNT) fail(MPS_ERR_ARG, "bad kernel class");
        const KStat& k = st->stats[cls];
        if (launches) *launches = k.launches;
        if (total_ms) *total_ms = k.ms;
        if (flops) *flops = k.flops;
        if (bytes) *bytes = k.bytes;
    });
}

}  // extern "C"

namespace {
template <typename R>
void selftest_cgemm_impl(int opa, int opb, int M, int N, int K, const double* a, const double* b, double* c,
                         int split_terms_ = 0) {
    const bool split = split_terms_ > 0;
    hipStream_t s = nullptr;
    const int64_t na = (int64_t)M * K, nb = (int64_t)K * N, nc = (int64_t)M * N;
    std::vector<R> ha(2 * na), hb(2 * nb), hc(2 * nc);
    for (int64_t i = 0; i < na; ++i) { ha[i] = (R)a[2 * i]; ha[na + i] = (R)a[2 * i + 1]; }
    for (int64_t i = 0; i < nb; ++i) { hb[i] = (R)b[2 * i]; hb[nb + i] = (R)b[2 * i + 1]; }
    R* da = (R*)dalloc(sizeof(R) * 2 * std::max<int64_t>(na, 1), s);
    R* db = (R*)dalloc(sizeof(R) * 2 * std::max<int64_t>(nb, 1), s);
    R* dc = (R*)dalloc(sizeof(R) * 2 * std::max<int64_t>(nc, 1), s);
    HIPCHK(hipMemcpyAsync(da, ha.data(), sizeof(R) * 2 * na, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(db, hb.data(), sizeof(R) * 2 * nb, hipMemcpyHostToDevice, s));
    const int64_t lda = (opa == OP_N) ? K : M;
    const int64_t ldb = (opb == OP_N) ? N : K;
    // the same split-K policy as the compression step (FP32 and split-precision kernels)
    const int req = split ? splitk_for_split(M, N, K) : splitk_for(M, N, K);
    const int ks = sizeof(R) == 4 ? splitk_chunks(K, req, 16) : 1;
    float* ws = nullptr;
    if (ks > 1) ws = (float*)dalloc(sizeof(float) * 2 * (size_t)nc * ks, s);
    // split precision: operands split once into BF16 planes, as in the compression step
    unsigned short* pl = nullptr;
    int64_t ea = 0;
    if (split) {
        ea = split_planes_elems(split_terms_, M, K, true);
        const int64_t eb = split_planes_elems(split_terms_, N, K, false);
        pl = (unsigned short*)dalloc(sizeof(unsigned short) * (size_t)std::max<int64_t>(ea + eb, 1), s);
        HIPCHK(split_planes(split_terms_, M, K, true, {(const float*)da, (const float*)(da + na), lda}, pl, s));
        if (opb == OP_T)
            HIPCHK(split_planes(split_terms_, N, K, false, {(const float*)db, (const float*)(db + nb), ldb}, pl + ea, s));
        else   // b is K x N: the planes of b^T straight from b, as in the environment update
            HIPCHK(split_planes_t(split_terms_, N, K, false, {(const float*)db, (const float*)(db + nb), ldb}, pl + ea,
                                  s));
    }
    if (split && ks > 1)
        HIPCHK(cgemm_bf16_planes_splitk(split_terms_, M, N, K, pl, pl + ea, ws, ws + nc * ks, req, s));
    else if (split)
        HIPCHK(cgemm_bf16_planes(split_terms_, M, N, K, pl, pl + ea, {(float*)dc, (float*)(dc + nc), N}, s));
    else if (ks > 1)
        HIPCHK(cgemm_f32_splitk(opa, opb, M, N, K, {(const float*)da, (const float*)(da + na), lda},
                                {(const float*)db, (const float*)(db + nb), ldb}, ws, ws + nc * ks, req, s));
    else
        HIPCHK(gemm_raw<R>(opa, opb, M, N, K, da, da + na, lda, db, db + nb, ldb, dc, dc + nc, N, s));
    if (ks > 1) {
        HIPCHK(splitk_reduce(ws, ws + nc * ks, ks, M, N, (float*)dc, (float*)(dc + nc), N, s));
        dfree(ws, s, nullptr);
    }
    HIPCHK(hipMemcpyAsync(hc.data(), dc, sizeof(R) * 2 * nc, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (pl) dfree(pl, s, nullptr);
    dfree(da, s, nullptr); dfree(db, s, nullptr); dfree(dc, s, nullptr);
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nc; ++i) { c[2 * i] = hc[i]; c[2 * i + 1] = hc[nc + i]; }
}
}  // namespace

namespace {
void selftest_eigh_impl(int n, const double* a, int method, double* w, double* z, int* used) {
    mps_state tmp;
    tmp.stream = nullptr;
    if (rocblas_create_handle(&tmp.blas) != rocblas_status_success) fail(MPS_ERR_DEVICE, "rocblas_create_handle failed");
    EighWork wk;
    Planar<double> g;
    try {
        const int64_t nn = (int64_t)n * n;
        std::vector<double> h(2 * nn);
        for (int64_t i = 0; i < nn; ++i) { h[i] = a[2 * i]; h[nn + i] = a[2 * i + 1]; }
        g.ensure(nn, nullptr);
        HIPCHK(hipMemcpyAsync(g.re(), h.data(), sizeof(double) * nn, hipMemcpyHostToDevice, nullptr));
        HIPCHK(hipMemcpyAsync(g.im(), h.data() + nn, sizeof(double) * nn, hipMemcpyHostToDevice, nullptr));
        eigh_gram(&tmp, wk, g.re(), g.im(), n, method);
        Planar<double> u;
        u.ensure(nn, nullptr);
        top_eigvecs(&tmp, wk, n, n, u.re(), u.im());      // row-major n x n, largest first
        int info = 0;
        std::vector<double> hu(2 * nn);
        HIPCHK(hipMemcpyAsync(w, wk.evals.p, sizeof(double) * n, hipMemcpyDeviceToHost, nullptr));
        HIPCHK(hipMemcpyAsync(hu.data(), u.re(), sizeof(double) * nn, hipMemcpyDeviceToHost, nullptr));
        HIPCHK(hipMemcpyAsync(hu.data() + nn, u.im(), sizeof(double) * nn, hipMemcpyDeviceToHost, nullptr));
        HIPCHK(hipMemcpyAsync(&info, wk.info.p, sizeof(int), hipMemcpyDeviceToHost, nullptr));
        HIPCHK(hipStreamSynchronize(nullptr));
        u.release(nullptr);
        // eigenvector j (ascending order) is column n - 1 - j of u
        for (int64_t r = 0; r < n; ++r)
            for (int64_t j = 0; j < n; ++j) {
                z[2 * (r + j * n)] = hu[r * n + (n - 1 - j)];
                z[2 * (r + j * n) + 1] = hu[nn + r * n + (n - 1 - j)];
            }
        if (info != 0) fail(MPS_ERR_NUMERIC, "eigensolver did not converge (info " + std::to_string(info) + ")");
        if (used) *used = wk.method_used;
    } catch (...) {
        (void)hipStreamSynchronize(nullptr);
        wk.release(nullptr);
        g.release(nullptr);
        rocblas_destroy_handle(tmp.blas);
        throw;
    }
    wk.release(nullptr);
    g.release(nullptr);
    HIPCHK(hipStreamSynchronize(nullptr));
    rocblas_destroy_handle(tmp.blas);
}
}  // namespace

extern "C" mps_status mps_kernel_selftest_eigh(int n, const double* a, int method, double* w, double* z, int* used) {
    return run_guarded([&] {
        if (n < 1 || n > 8192 || !a || !w || !z) fail(MPS_ERR_ARG, "bad eigensolver self-test arguments");
        if (method != EIGH_ROCSOLVER && method != EIGH_PERSISTENT) fail(MPS_ERR_ARG, "method must be 0 or 1");
        selftest_eigh_impl(n, a, method, w, z, used);
    });
}

extern "C" mps_status mps_kernel_selftest_stedc(int n, const double* d, const double* e, double* w, double* z) {
    return run_guarded([&] {
        if (n < 1 || n > stedc_dc_max_n() || !d || (n > 1 && !e) || !w || !z)
            fail(MPS_ERR_ARG, "bad tridiagonal self-test arguments");
        Raw<double> dd, ee, zz;
        Raw<char> ws;
        try {
            const size_t wsb = stedc_dc_workspace_bytes(n);
            dd.ensure(n, nullptr);
            ee.ensure(std::max(1, n - 1), nullptr);
            zz.ensure((int64_t)n * n, nullptr);
            ws.ensure((int64_t)wsb, nullptr);
            HIPCHK(hipMemcpyAsync(dd.p, d, sizeof(double) * n, hipMemcpyHostToDevice, nullptr));
            if (n > 1) HIPCHK(hipMemcpyAsync(ee.p, e, sizeof(double) * (n - 1), hipMemcpyHostToDevice, nullptr));
            HIPCHK(stedc_dc(n, dd.p, ee.p, zz.p, n, ws.p, wsb, nullptr));
            HIPCHK(hipMemcpyAsync(w, dd.p, sizeof(double) * n, hipMemcpyDeviceToHost, nullptr));
            HIPCHK(hipMemcpyAsync(z, zz.p, sizeof(double) * n * n, hipMemcpyDeviceToHost, nullptr));
            HIPCHK(hipStreamSynchronize(nullptr));
        } catch (...) {
            (void)hipStreamSynchronize(nullptr);
            dd.release(nullptr); ee.release(nullptr); zz.release(nullptr); ws.release(nullptr);
            throw;
        }
        dd.release(nullptr); ee.release(nullptr); zz.release(nullptr); ws.release(nullptr);
    });
}

extern "C" mps_status mps_kernel_selftest_cgemm(int precision, int opa, int opb, int M, int N, int K,
                                                const double* a, const double* b, double* c) {
    return run_guarded([&] {
        if (M < 1 || N < 1 || K < 1 || !a || !b || !c) fail(MPS_ERR_ARG, "bad GEMM self-test arguments");
        if (opa != OP_N && opa != OP_C) fail(MPS_ERR_ARG, "opa must be 0 (N) or 2 (C)");
        if (opb != OP_N && opb != OP_T && opb != OP_C) fail(MPS_ERR_ARG, "opb must be 0, 1 or 2");
        if ((int64_t)M * K > (1 << 28) || (int64_t)K * N > (1 << 28) || (int64_t)M * N > (1 << 28))
            fail(MPS_ERR_ARG, "self-test operands too large");
        if (is_split(precision)) {
            if (opa != OP_N || (opb != OP_T && opb != OP_N))
                fail(MPS_ERR_ARG, "the split-precision kernel takes opa = 0, opb = 1 (or 0: B split transposed)");
            selftest_cgemm_impl<float>(opa, opb, M, N, K, a, b, c, precision == MPS_BF16X2 ? 2 : 3);
        } else if (precision == MPS_FP32) selftest_cgemm_impl<float>(opa, opb, M, N, K, a, b, c);
        else if (precision == MPS_FP64) selftest_cgemm_impl<double>(opa, opb, M, N, K, a, b, c);
        else fail(MPS_ERR_ARG, "unknown precision");
    });
}

// ============================================== allocation-free GEMM ====
// Split-K partial sums of mps_cgemm_noalloc live in this file-scope device
// array (one copy per GPU, held until the process ends).  Host code never
// passes its name to a kernel: the address is taken once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t SCRATCH_FLOATS = (size_t)16 << 20;            // 64 MiB
static __device__ __align__(256) float scratch[SCRATCH_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

// The scratch array of the current device (its address is resolved on first use).
float* scratch_of_current_device() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(MPS_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(MPS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (float*)ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" mps_status mps_cgemm_noalloc(int precision, int opa, int opb, int M, int N, int K, const void* a_re,
                                        const void* a_im, int64_t lda, const void* b_re, const void* b_im,
                                        int64_t ldb, void* c_re, void* c_im, int64_t ldc, void* hip_stream) {
    return run_guarded([&] {
        if (M < 1 || N < 1 || K < 1) fail(MPS_ERR_ARG, "M, N and K must be >= 1");
        if (!a_re || !a_im || !b_re || !b_im || !c_re || !c_im) fail(MPS_ERR_ARG, "NULL operand");
        if (opa != OP_N && opa != OP_C) fail(MPS_ERR_ARG, "opa must be 0 (N) or 2 (C)");
        if (opb != OP_N && opb != OP_T && opb != OP_C) fail(MPS_ERR_ARG, "opb must be 0, 1 or 2");
        if (lda < (opa == OP_N ? K : M) || ldb < (opb == OP_N ? N : K) || ldc < N)
            fail(MPS_ERR_ARG, "leading dimension smaller than the row length");
        if (precision != MPS_FP64 && precision != MPS_FP32 && !is_split(precision))
            fail(MPS_ERR_ARG, "unknown precision");
        if (is_split(precision) && (opa != OP_N || opb != OP_T))
            fail(MPS_ERR_ARG, "the split-precision kernel takes opa = 0, opb = 1");
        const hipStream_t s = (hipStream_t)hip_stream;
        if (precision == MPS_FP64) {
            HIPCHK(cgemm_f64(opa, opb, M, N, K, {(const double*)a_re, (const double*)a_im, lda},
                             {(const double*)b_re, (const double*)b_im, ldb}, {(double*)c_re, (double*)c_im, ldc}, s));
            return;
        }
        // the split-K policy of the compression step and of mps_kernel_selftest_cgemm
        const int req = is_split(precision) ? splitk_for_split(M, N, K) : splitk_for(M, N, K);
        const int ks = splitk_chunks(K, req, 16);
        const CView<float> A{(const float*)a_re, (const float*)a_im, lda};
        const CView<float> B{(const float*)b_re, (const float*)b_im, ldb};
        const int terms = precision == MPS_BF16X2 ? 2 : 3;
        if (ks <= 1) {
            const CViewMut<float> C{(float*)c_re, (float*)c_im, ldc};
            if (is_split(precision))
                HIPCHK(cgemm_bf16_nt(terms, M, N, K, A, B, C, s));
            else
                HIPCHK(cgemm_f32(opa, opb, M, N, K, A, B, C, s));
            return;
        }
        const size_t need = 2 * (size_t)M * (size_t)N * (size_t)ks;
        if (need > SCRATCH_FLOATS)
            fail(MPS_ERR_ARG, "split-K partial sums need " + std::to_string(need * sizeof(float)) +
                                  " bytes, more than the " + std::to_string(SCRATCH_FLOATS * sizeof(float)) +
                                  "-byte scratch array");
        float* ws = scratch_of_current_device();
        float* ws_re = ws;
        float* ws_im = ws + (size_t)M * N * ks;
        if (is_split(precision))
            HIPCHK(cgemm_bf16_nt_splitk(terms, M, N, K, A, B, ws_re, ws_im, req, s));
        else
            HIPCHK(cgemm_f32_splitk(opa, opb, M, N, K, A, B, ws_re, ws_im, req, s));
        HIPCHK(splitk_reduce(ws_re, ws_im, ks, M, N, (float*)c_re, (float*)c_im, ldc, s));
    });
}

// ======================================================= exact statevector ===
// The brute-force state U|0> kept in HBM, against which an MPS is measured
// (F of eq:F-sup, F_B of eq:FB-sup).
struct sv_state {
    int n = 0;
    hipStream_t stream = nullptr;
    double* re = nullptr;   // one allocation: re block of 2^n, then im block
    double* im = nullptr;
};

namespace {

constexpr int SV_MAX_QUBITS = 34;

struct SvTwo {
    int q0, q1;
    cd u[4][4];   // row 2 s_q0 + s_q1
};

// One layer under the rules of mps_gate: per-qubit products of the one-qubit gates (list
// order) and the two-qubit gates, checked for range, finiteness and disjointness.
void parse_sv_layer(int n, const mps_gate* gates, int n_gates, std::vector<cd>& g1, std::vector<SvTwo>& two) {
    if (n_gates < 0 || (n_gates > 0 && !gates)) fail(MPS_ERR_ARG, "gates is NULL");
    g1.assign(4 * (size_t)n, cd(0));
    for (int q = 0; q < n; ++q) g1[4 * q] = g1[4 * q + 3] = 1.0;
    std::vector<int> used(n, 0);
    two.clear();
    for (int gi = 0; gi < n_gates; ++gi) {
        const mps_gate& g = gates[gi];
        for (int e = 0; e < 32; ++e)
            if (!std::isfinite(g.m[e])) fail(MPS_ERR_ARG, "gate matrix has a non-finite entry");
        if (g.q1 < 0) {
            if (g.q1 != -1 || g.q0 < 0 || g.q0 >= n) fail(MPS_ERR_ARG, "one-qubit gate site out of range");
            cd u[2][2], cur[2][2], out[2][2];
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t) {
                    u[s][t] = cd(g.m[2 * (s * 2 + t)], g.m[2 * (s * 2 + t) + 1]);
                    cur[s][t] = g1[4 * (size_t)g.q0 + s * 2 + t];
                }
            mul2(u, cur, out);
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t) g1[4 * (size_t)g.q0 + s * 2 + t] = out[s][t];
            continue;
        }
        if (g.q0 < 0 || g.q0 >= n || g.q1 >= n || g.q0 == g.q1)
            fail(MPS_ERR_ARG, "two-qubit gate sites out of range or equal");
        if (used[g.q0] || used[g.q1]) fail(MPS_ERR_ARG, "two-qubit gates of one layer must be disjoint");
        used[g.q0] = used[g.q1] = 1;
        SvTwo t;
        t.q0 = g.q0;
        t.q1 = g.q1;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) t.u[r][c] = cd(g.m[2 * (r * 4 + c)], g.m[2 * (r * 4 + c) + 1]);
        two.push_back(t);
    }
}

// (G_a x G_b)[(s_a s_b), (t_a t_b)] = G_a[s_a][t_a] G_b[s_b][t_b]
void kron2(const cd* ga, const cd* gb, cd out[4][4]) {
    for (int sa = 0; sa < 2; ++sa)
        for (int sb = 0; sb < 2; ++sb)
            for (int ta = 0; ta < 2; ++ta)
                for (int tb = 0; tb < 2; ++tb) out[sa * 2 + sb][ta * 2 + tb] = ga[sa * 2 + ta] * gb[sb * 2 + tb];
}

SvGate2 to_gate2(const cd u[4][4]) {
    SvGate2 g;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            g.re[r * 4 + c] = u[r][c].real();
            g.im[r * 4 + c] = u[r][c].imag();
        }
    return g;
}

void sv_apply_layer_impl(sv_state* sv, const mps_gate* gates, int n_gates) {
    const int n = sv->n;
    std::vector<cd> g1;
    std::vector<SvTwo> two;
    parse_sv_layer(n, gates, n_gates, g1, two);
    std::vector<int> in_two(n, 0);
    // each two-qubit gate with the one-qubit gates of its qubits folded in: U (G_q0 x G_q1)
    for (const SvTwo& t : two) {
        in_two[t.q0] = in_two[t.q1] = 1;
        cd k[4][4], u[4][4];
        kron2(&g1[4 * (size_t)t.q0], &g1[4 * (size_t)t.q1], k);
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                u[r][c] = 0;
                for (int m = 0; m < 4; ++m) u[r][c] += t.u[r][m] * k[m][c];
            }
        HIPCHK(sv_apply_2q(sv->re, sv->im, n, n - 1 - t.q0, n - 1 - t.q1, to_gate2(u), sv->stream));
    }
    // the remaining one-qubit gates, two per pass
    std::vector<int> lone;
    for (int q = 0; q < n; ++q) {
        const cd* g = &g1[4 * (size_t)q];
        if (!in_two[q] && !(g[0] == cd(1) && g[1] == cd(0) && g[2] == cd(0) && g[3] == cd(1))) lone.push_back(q);
    }
    size_t i = 0;
    for (; i + 1 < lone.size(); i += 2) {
        cd k[4][4];
        kron2(&g1[4 * (size_t)lone[i]], &g1[4 * (size_t)lone[i + 1]], k);
        HIPCHK(sv_apply_2q(sv->re, sv->im, n, n - 1 - lone[i], n - 1 - lone[i + 1], to_gate2(k), sv->stream));
    }
    if (i < lone.size()) {
        SvGate1 g;
        for (int e = 0; e < 4; ++e) {
            g.re[e] = g1[4 * (size_t)lone[i] + e].real();
            g.im[e] = g1[4 * (size_t)lone[i] + e].imag();
        }
        HIPCHK(sv_apply_1q(sv->re, sv->im, n, n - 1 - lone[i], g, sv->stream));
    }
}

// The MPS as a statevector on the device: contract the sites in chain order,
// cur (2^k x D_k) * A_k (D_k x 2 D_{k+1}) read as (2^(k+1) x D_{k+1}); then the
// fixed-order reductions of sv_compare against the exact state.
void sv_compare_impl(const sv_state* sv, mps_state* st, double* out5) {
    if (st->n != sv->n) fail(MPS_ERR_ARG, "the MPS and the statevector have different numbers of qubits");
    const int n = sv->n;
    HIPCHK(hipStreamSynchronize(sv->stream));
    const hipStream_t s = st->stream;
    int64_t need = 1;
    for (int k = 0; k < n; ++k) need = std::max<int64_t>(need, ((int64_t)1 << k) * 2 * st->bond[k + 1]);
    if (need > ((int64_t)2 << n)) fail(MPS_ERR_ARG, "MPS bond dimensions exceed the state space");
    Planar<double> cur, nxt, t;
    cur.ensure(need, s);
    nxt.ensure(need, s);
    HIPCHK(fill_planar<double>(cur.re(), cur.im(), 1, 1.0, s));
    int64_t rows = 1;
    constexpr int64_t CH = (int64_t)1 << 24;
    for (int k = 0; k < n; ++k) {
        forward_tensor(st, k, t, s);
        const int64_t Dk = st->bond[k], Dn = st->bond[k + 1];
        for (int64_t r0 = 0; r0 < rows; r0 += CH) {
            const int64_t m = std::min(CH, rows - r0);
            gemm<double>(st, MPS_KCLASS_OTHER, OP_N, OP_N, m, 2 * Dn, Dk, cur.re() + r0 * Dk, cur.im() + r0 * Dk, Dk,
                         t.re(), t.im(), 2 * Dn, nxt.re() + r0 * 2 * Dn, nxt.im() + r0 * 2 * Dn, 2 * Dn);
        }
        rows *= 2;
        std::swap(cur, nxt);
    }
    const int nb = sv_compare_blocks();
    Raw<double> part;
    part.ensure((int64_t)nb * 5, s);
    HIPCHK(sv_compare(cur.re(), cur.im(), sv->re, sv->im, (uint64_t)1 << n, part.p, s));
    std::vector<double> h((size_t)nb * 5);
    HIPCHK(hipMemcpyAsync(h.data(), part.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < 5; ++k) out5[k] = 0;
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 5; ++k) out5[k] += h[(size_t)b * 5 + k];
    cur.release(s); nxt.release(s); t.release(s); part.release(s);
    HIPCHK(hipStreamSynchronize(s));
    flush_timings(st);
}

// Eigenvalues (ascending) of the Gram matrix of psi split after `cut` sites: the squared
// Schmidt values of the cut (the best-MPS reference of Sec. VI).  The smaller side sets the
// order of the Gram matrix (at most SV_MAX_SCHMIDT_DIM); it is formed by the FP64 Gram GEMM
// and diagonalised by rocSOLVER (values only).
constexpr int SV_MAX_SCHMIDT_DIM = 16384;

std::vector<double> sv_schmidt_impl(const sv_state* sv, int cut) {
    const int n = sv->n;
    if (cut < 1 || cut >= n) fail(MPS_ERR_ARG, "cut must be in [1, n_qubits - 1]");
    const int64_t rows = (int64_t)1 << cut, cols = (int64_t)1 << (n - cut);
    const int64_t dim = std::min(rows, cols);
    if (dim > SV_MAX_SCHMIDT_DIM) fail(MPS_ERR_ARG, "the smaller side of the cut exceeds 14 qubits");
    mps_state tmp;
    tmp.stream = sv->stream;
    if (rocblas_create_handle(&tmp.blas) != rocblas_status_success) fail(MPS_ERR_DEVICE, "rocblas_create_handle failed");
    rocblas_set_stream(tmp.blas, tmp.stream);
    const hipStream_t s = tmp.stream;
    Planar<double> g;
    Raw<double> z, ev, ework;
    Raw<int> info;
    std::vector<double> w(dim);
    try {
        g.ensure(dim * dim, s);
        if (rows <= cols)
            gram_product<double>(&tmp, OP_N, OP_C, (int)dim, cols, sv->re, sv->im, cols, g.re(), g.im());
        else
            gram_product<double>(&tmp, OP_C, OP_N, (int)dim, rows, sv->re, sv->im, cols, g.re(), g.im());
        z.ensure(2 * dim * dim, s);
        HIPCHK(pack_hermitian(g.re(), g.im(), (int)dim, z.p, s));
        g.release(s);
        ev.ensure(dim, s);
        ework.ensure(dim, s);
        info.ensure(1, s);
        const rocblas_status rs = rocsolver_zheevd(tmp.blas, rocblas_evect_none, rocblas_fill_upper, (int)dim,
                                                   (rocblas_double_complex*)z.p, (int)dim, ev.p, ework.p, info.p);
        if (rs != rocblas_status_success) fail(MPS_ERR_DEVICE, "rocsolver_zheevd failed: status " + std::to_string((int)rs));
        int hinfo = 0;
        HIPCHK(hipMemcpyAsync(w.data(), ev.p, sizeof(double) * dim, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hinfo != 0) fail(MPS_ERR_NUMERIC, "eigensolver did not converge");
    } catch (...) {
        (void)hipStreamSynchronize(s);
        g.release(s); z.release(s); ev.release(s); ework.release(s); info.release(s); tmp.splitws64.release(s);
        (void)hipStreamSynchronize(s);
        rocblas_destroy_handle(tmp.blas);
        throw;
    }
    z.release(s); ev.release(s); ework.release(s); info.release(s); tmp.splitws64.release(s);
    HIPCHK(hipStreamSynchronize(s));
    rocblas_destroy_handle(tmp.blas);
    return w;
}

}  // namespace

extern "C" {

mps_status sv_create(int n_qubits, const uint8_t* init_bits, void* hip_stream, sv_state** out) {
    return run_guarded([&] {
        if (!out) fail(MPS_ERR_ARG, "out is NULL");
        *out = nullptr;
        if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) fail(MPS_ERR_ARG, "n_qubits must be in [1, 34]");
        uint64_t one_at = 0;
        if (init_bits)
            for (int k = 0; k < n_qubits; ++k) {
                if (init_bits[k] > 1) fail(MPS_ERR_ARG, "init_bits must be 0 or 1");
                one_at = (one_at << 1) | init_bits[k];
            }
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(MPS_ERR_DEVICE, "no HIP device available");
        const uint64_t dim = (uint64_t)1 << n_qubits;
        void* p = nullptr;
        if (hipMalloc(&p, sizeof(double) * 2 * dim) != hipSuccess) {
            (void)hipGetLastError();
            fail(MPS_ERR_OOM, "cannot allocate the statevector");
        }
        sv_state* sv = new sv_state();
        sv->n = n_qubits;
        sv->stream = (hipStream_t)hip_stream;
        sv->re = (double*)p;
        sv->im = sv->re + dim;
        const hipError_t e = sv_fill(sv->re, sv->im, dim, one_at, sv->stream);
        if (e != hipSuccess || hipStreamSynchronize(sv->stream) != hipSuccess) {
            (void)hipFree(p);
            delete sv;
            fail(MPS_ERR_DEVICE, "statevector initialisation failed");
        }
        *out = sv;
    });
}

mps_status sv_destroy(sv_state* sv) {
    return run_guarded([&] {
        if (!sv) return;
        (void)hipStreamSynchronize(sv->stream);
        (void)hipFree(sv->re);
        delete sv;
    });
}

mps_status sv_apply_layer(sv_state* sv, const mps_gate* gates, int n_gates) {
    return run_guarded([&] {
        if (!sv) fail(MPS_ERR_ARG, "statevector is NULL");
        sv_apply_layer_impl(sv, gates, n_gates);
        HIPCHK(hipStreamSynchronize(sv->stream));
    });
}

mps_status sv_amplitudes(const sv_state* sv, int64_t count, const int64_t* indices, double* out) {
    return run_guarded([&] {
        if (!sv) fail(MPS_ERR_ARG, "statevector is NULL");
        if (count < 0 || (count > 0 && (!indices || !out))) fail(MPS_ERR_ARG, "bad amplitude arguments");
        const int64_t dim = (int64_t)1 << sv->n;
        for (int64_t t = 0; t < count; ++t)
            if (indices[t] < 0 || indices[t] >= dim) fail(MPS_ERR_ARG, "index out of range");
        if (count == 0) return;
        const hipStream_t s = sv->stream;
        Raw<int64_t> di;
        Raw<double> dout;
        di.ensure(count, s);
        dout.ensure(2 * count, s);
        HIPCHK(hipMemcpyAsync(di.p, indices, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
        HIPCHK(sv_gather(sv->re, sv->im, di.p, count, dout.p, s));
        HIPCHK(hipMemcpyAsync(out, dout.p, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        di.release(s);
        dout.release(s);
        HIPCHK(hipStreamSynchronize(s));
    });
}

mps_status sv_compare_mps(const sv_state* sv, mps_state* mps, double* overlap, double* F, double* F_B,
                          double* norms) {
    return run_guarded([&] {
        if (!sv) fail(MPS_ERR_ARG, "statevector is NULL");
        check_state(mps);
        double r[5];
        sv_compare_impl(sv, mps, r);
        const double dim = std::ldexp(1.0, sv->n);
        if (overlap) { overlap[0] = r[0]; overlap[1] = r[1]; }
        if (F) *F = r[0] * r[0] + r[1] * r[1];
        if (F_B) *F_B = dim * r[2] - 1.0;
        if (norms) { norms[0] = r[3]; norms[1] = r[4]; }
    });
}

mps_status sv_schmidt_weights(const sv_state* sv, int cut, int chi, double* kept, double* total, double* s2) {
    return run_guarded([&] {
        if (!sv) fail(MPS_ERR_ARG, "statevector is NULL");
        if (chi < 1) fail(MPS_ERR_ARG, "chi must be >= 1");
        const std::vector<double> w = sv_schmidt_impl(sv, cut);
        const int64_t dim = (int64_t)w.size();
        double sum = 0, top = 0;
        for (int64_t i = 0; i < dim; ++i) sum += w[i];
        for (int64_t i = dim - 1; i >= 0 && dim - 1 - i < chi; --i) top += w[i];
        if (kept) *kept = top;
        if (total) *total = sum;
        if (s2)
            for (int64_t i = 0; i < dim; ++i) s2[i] = w[dim - 1 - i];
    });
}

}  // extern "C"
