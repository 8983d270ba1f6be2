// Householder reduction of a Hermitian matrix to real symmetric tridiagonal
// form, T = Q^H A Q with Q = H_0 H_1 ... H_{n-2}, as one persistent kernel.
//
// The FP64 truncation of a two-site step (Sec. VI.A: keep the chi largest
// singular values) diagonalises a Gram matrix of order 2 chi.  Its
// tridiagonal reduction is a chain of n - 1 dependent Householder steps, each
// a matrix-vector product with the trailing block; issued as a few kernels
// per step it is launch-latency bound.  Here one cooperative launch does all
// steps:
//   * workgroup g owns the columns 8g .. 8g + 7, four in registers and four
//     in LDS, for the whole reduction, so the trailing block is never re-read
//     from memory; a workgroup whose columns are all reduced leaves, so the
//     number of workgroups that exchange data shrinks from n / 8 to one
//     (the cost of an exchange grows with the number of participants);
//   * every workgroup holds column i (as updated by steps 0 .. i-1) in its
//     registers and forms the reflector (v, tau) from it redundantly;
//   * it computes y = A v for its own columns (the matrix is Hermitian, so
//     y_c is the dot product of column c with v), publishes y_c and its share
//     of y^H v, and waits for the other workgroups that still hold columns
//     (the only wait of the step);
//   * it applies the rank-2 update A -= v w^H + w v^H,
//     w = tau y - (|tau|^2 y^H v / 2) v, to its columns, and rebuilds column
//     i+1 for the next step from the copy of it that the column's owner
//     published one step earlier plus this step's update (look-ahead), so no
//     second wait is needed;
//   * the owner of column i+2 publishes it after this step's update.
// Reflector convention: H = I - tau v v^H with v_i[0..i] = 0, v_i[i+1] = 1,
// H^H x = (beta, 0, ...) for the column x below the diagonal, beta real.
// The reflectors are written conjugated, one per row, as the planar
// row-major (n - 1) x n matrix V^H, which is the operand layout of the
// blocked back-transformation by GEMMs.
//
// Every wait is bounded: a workgroup that waits too long raises the abort
// flag, every other wait sees it, and all workgroups exit; the host then
// falls back to another eigensolver.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mpsk {
namespace {

constexpr int TT = 512;            // threads per workgroup
constexpr int TQ = 4;              // rows per thread: row = tid + TT * q
constexpr int TC = 8;              // columns per workgroup
constexpr int TCR = 4;             // columns kept in registers (the rest in LDS)
constexpr int TMAXN = TT * TQ;     // 2048
constexpr int NWAVE = TT / 64;
constexpr int SPIN_LIMIT = 1 << 21;
constexpr int TR_MAXB = 8;         // instances per launch
constexpr int HG = 4;              // groups of the two-level wait (workgroups wg = g mod HG)
constexpr int GF_STRIDE = 16;      // ints between group flags

struct TrArgs {
    const double2* a;    // n x n column-major, full Hermitian (not modified)
    double* vh_re;       // (n - 1) x n row-major planar: row i = conj(v_i)
    double* vh_im;
    int n, lda, P;
    double* d;           // n
    double* e;           // n - 1
    double2* tau;        // n - 1
    double2* colbuf;     // 2 x n: published column
    double2* ybuf;       // 2 x n: published y
    double2* pdot;       // 2 x P: per-workgroup partial y^H v
    int* col_flag;       // number of published columns
    int* wg_flag;        // P: steps completed by each workgroup
    int* grp_flag;       // HG group flags, 64 bytes apart: steps completed by every member
    int* abort_flag;
};

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
__device__ inline double2 cjmul(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ inline double2 ld_coh(const double2* p) {
    const unsigned long long* q = (const unsigned long long*)p;
    const unsigned long long x = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long y = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_double2(__builtin_bit_cast(double, x), __builtin_bit_cast(double, y));
}
__device__ inline double ld_coh1(const double* p) {
    return __builtin_bit_cast(double, __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline void st_coh1(double* p, double v) {
    __hip_atomic_store((unsigned long long*)p, __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_coh(double2* p, double2 v) {
    unsigned long long* q = (unsigned long long*)p;
    __hip_atomic_store(q, __builtin_bit_cast(unsigned long long, v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, __builtin_bit_cast(unsigned long long, v.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-workgroup protocol (release / acquire at agent scope).  Every value
// another workgroup reads is written with a device-coherent atomic store
// (st_coh) and read with a device-coherent atomic load (ld_coh).  A producer
// joins its workgroup barrier; then its first wavefront issues an agent-scope
// release fence and one thread stores the flag.  A consumer's first wavefront
// waits (wait_step_acquire, below) with relaxed loads, issues an agent-scope
// acquire fence once every producer has the value, and the workgroup barrier
// that follows orders the data loads of every wavefront after it.  The
// barriers carry the ordering inside a workgroup and the fence pair
// (fence-fence synchronisation of the HIP / C++ memory model) carries it
// across workgroups, so the protocol does not rest on hardware ordering.
// One fence of each kind per workgroup and step (two more in a leader): each one
// costs an L2 write-back (release) or invalidation (acquire).  The reflectors
// and the tridiagonal entries are written with coherent stores as well, so
// the L2 holds no dirty lines that a release would have to write back.

// After the workgroup barrier, release this workgroup's earlier stores and set *flag = val.
__device__ void publish(int* flag, int val) {
    __syncthreads();
    if (threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) __hip_atomic_store(flag, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Wait of step i.  The participants are the workgroups g0 .. count - 1 (those that
// still hold an unreduced column).  With many participants, polling all their
// flags from every workgroup contends for the same few cache lines; then they
// form HG groups (g mod HG) and the first participant of each group leads it:
// its first wavefront waits for the flags of its members, acquires, releases
// and sets the group's flag; every participant then waits for the flags of the
// non-empty groups and acquires.  The release -> acquire -> release -> acquire
// chain through the leader makes every member's stores visible to every
// participant (happens-before is transitive), so the protocol stays the
// fence-fence synchronisation described above.  With at most FLAT_MAX (one per
// lane) participants every one polls all their flags directly.  Every wait is
// bounded: on time-out the abort flag is raised; on abort (own or seen) it
// returns false in wavefront 0.
constexpr int FLAT_MAX = 64;
__device__ bool wait_step_acquire(int* flags, int* grp_flags, int g0, int count, int wg, int target, int* abort_flag) {
    bool ok = true;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int spins = 0;
        auto bail = [&]() {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return true;
            }
            __builtin_amdgcn_s_sleep(1);
            return false;
        };
        if (count - g0 <= FLAT_MAX) {
            while (true) {
                const int m = g0 + lane;
                const bool done = m >= count ||
                                  __hip_atomic_load(flags + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
                if (__all(done)) break;
                if (bail()) { ok = false; break; }
            }
        } else {
            if (wg < g0 + HG) {
                // members wg, wg + HG, ... (at most 256 / HG = 64 of them: one per lane)
                while (true) {
                    const int m = wg + HG * lane;
                    const bool done = m >= count ||
                                      __hip_atomic_load(flags + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
                    if (__all(done)) break;
                    if (bail()) { ok = false; break; }
                }
                if (ok) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    if (lane == 0)
                        __hip_atomic_store(grp_flags + GF_STRIDE * (wg % HG), target, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            while (ok) {
                // group lane % HG is led by g0 + lane (count - g0 > HG: every group has members)
                const bool done = lane >= HG ||
                                  __hip_atomic_load(grp_flags + GF_STRIDE * ((g0 + lane) % HG), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT) >= target;
                if (__all(done)) break;
                if (bail()) { ok = false; break; }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    return ok;
}

// The value of lane ^ M.  Partners within a row of 16 lanes (M <= 8) move through DPP
// (quad permutations; row shifts left / right by M, selected by bit M of the lane), which
// stays in the VALU; the row-crossing ones (16, 32) through the LDS crossbar.
template <int CTRL>
__device__ inline double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int M>
__device__ inline double xor_lane(double v, int lane) {
    if constexpr (M == 1) return dpp_mov<0xB1>(v);                    // quad_perm [1, 0, 3, 2]
    else if constexpr (M == 2) return dpp_mov<0x4E>(v);               // quad_perm [2, 3, 0, 1]
    else if constexpr (M == 4 || M == 8) {
        const double up = dpp_mov<0x100 + M>(v);                         // row_shl: from lane + M
        const double dn = dpp_mov<0x110 + M>(v);                         // row_shr: from lane - M
        return (lane & M) ? dn : up;
    } else {
        return __shfl_xor(v, M);
    }
}

__device__ inline double wave_sum(double v) {
    const int lane = threadIdx.x & 63;
    v += xor_lane<32>(v, lane);
    v += xor_lane<16>(v, lane);
    v += xor_lane<8>(v, lane);
    v += xor_lane<4>(v, lane);
    v += xor_lane<2>(v, lane);
    v += xor_lane<1>(v, lane);
    return v;
}

// Sums of 16 values over the 64 lanes of a wave by reduce-scatter: at the
// exchange with lane ^ 32, ^ 16, ^ 8, ^ 4 each lane keeps half of its values
// and adds the partner's copy of that half (8 + 4 + 2 + 1 exchanges), then two
// plain steps finish.  On return every lane holds the total of value
// index (lane >> 2) & 15 in bit-reversed order; see sum16_index().
__device__ inline double wave_sum16(double (&v)[16], int lane) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool hi = lane & 32;
        const double keep = hi ? v[8 + k] : v[k], give = hi ? v[k] : v[8 + k];
        v[k] = keep + xor_lane<32>(give, lane);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool hi = lane & 16;
        const double keep = hi ? v[4 + k] : v[k], give = hi ? v[k] : v[4 + k];
        v[k] = keep + xor_lane<16>(give, lane);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const bool hi = lane & 8;
        const double keep = hi ? v[2 + k] : v[k], give = hi ? v[k] : v[2 + k];
        v[k] = keep + xor_lane<8>(give, lane);
    }
    {
        const bool hi = lane & 4;
        const double keep = hi ? v[1] : v[0], give = hi ? v[0] : v[1];
        v[0] = keep + xor_lane<4>(give, lane);
    }
    double r = v[0];
    r += xor_lane<2>(r, lane);
    r += xor_lane<1>(r, lane);
    return r;
}
// Index (0..15) of the value whose total wave_sum16 leaves in this lane.
__device__ inline int sum16_index(int lane) {
    return ((lane & 32) ? 8 : 0) + ((lane & 16) ? 4 : 0) + ((lane & 8) ? 2 : 0) + ((lane & 4) ? 1 : 0);
}

// Owned column j (a compile-time constant after unrolling), thread row slot q, row r.
#define A_GET(j, q, r) ((j) < TCR ? areg[(j) < TCR ? (j) : 0][q] : alds[(j) < TCR ? 0 : (j) - TCR][r])
#define A_SUB(j, q, r, dx, dy)                                \
    do {                                                      \
        if ((j) < TCR) {                                      \
            areg[(j) < TCR ? (j) : 0][q].x -= (dx);           \
            areg[(j) < TCR ? (j) : 0][q].y -= (dy);           \
        } else {                                              \
            alds[(j) < TCR ? 0 : (j) - TCR][r].x -= (dx);     \
            alds[(j) < TCR ? 0 : (j) - TCR][r].y -= (dy);     \
        }                                                     \
    } while (0)
// A[r, c_j] -= v[r] conj(w_cj) + w[r] conj(v_cj) over the trailing rows
#define UPDATE_COL(j)                                                  \
    do {                                                               \
        const double2 vc_ = vcol[buf][j];                              \
        const double2 ty_ = cmul(tau, ycol[buf][j]);                   \
        const double2 wc_ = make_double2(ty_.x + alw * vc_.x, ty_.y + alw * vc_.y); \
        _Pragma("unroll") for (int q = 0; q < TQ; ++q) {               \
            const int r = tid + TT * q;                                \
            if (r < i + 1 || r >= n) continue;                         \
            const double2 t1 = cjmul(wc_, v[q]);                       \
            const double2 t2 = cjmul(vc_, w[q]);                       \
            A_SUB(j, q, r, t1.x + t2.x, t1.y + t2.y);                  \
        }                                                              \
    } while (0)

// The small shared values of a step are double-buffered by the parity of the step: a
// step's three workgroup barriers (after the partial sums, in the publication, after the
// wait) keep every wavefront within one step of the others, so a buffer is rewritten only
// after every read of it in the step before the previous one.
// Several independent reductions may share one cooperative launch (the reduction is
// latency-bound; an order-n matrix occupies only n / 8 workgroups): instance i owns the
// workgroups [first[i], first[i + 1]) and its own workspace and flags.
struct TrBatch {
    TrArgs a[TR_MAXB];
    int first[TR_MAXB + 1];
    int count;
};

__global__ __launch_bounds__(TT, 1) void hetrd_kernel(TrBatch batch) {
    __shared__ double2 alds[TC - TCR][TMAXN];
    __shared__ double red[2][NWAVE][2 * TC + 1];
    __shared__ double2 vcol[2][TC], ycol[2][TC], xcol[2][TC], a1col[2][TC];
    __shared__ double2 alpha_s[2];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int inst = 0;
    while (inst + 1 < batch.count && (int)blockIdx.x >= batch.first[inst + 1]) ++inst;
    const TrArgs g = batch.a[inst];
    const int wg = (int)blockIdx.x - batch.first[inst], P = g.P, n = g.n;
    const int64_t lda = g.lda;
    double2 areg[TCR][TQ];
    double2 x[TQ];          // column i at this thread's rows

    // load the owned columns and column 0
#pragma unroll
    for (int j = 0; j < TC; ++j) {
        const int c = wg * TC + j;
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const int r = tid + TT * q;
            double2 val = make_double2(0.0, 0.0);
            if (c < n && r < n) val = g.a[r + c * lda];
            if (j < TCR)
                areg[j < TCR ? j : 0][q] = val;
            else
                alds[j < TCR ? 0 : j - TCR][r] = val;
        }
    }
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
        const int r = tid + TT * q;
        x[q] = r < n ? g.a[r] : make_double2(0.0, 0.0);
    }
    if (tid < TC) {
        xcol[0][tid] = xcol[1][tid] = make_double2(0.0, 0.0);
        a1col[0][tid] = a1col[1][tid] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    const int c_first = wg * TC, c_last = min(n, c_first + TC) - 1;   // owned columns
    for (int i = 0; i + 1 < n; ++i) {
        // this workgroup leaves once all its columns are reduced (no column >= i + 1); the
        // participants of step i are the workgroups g0 .. P - 1
        if (c_last < i + 1) break;
        const int g0 = (i + 1) / TC;
        const int buf = i & 1;
        // ---- broadcasts from row i+1 and from the rows of the owned columns
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const int r = tid + TT * q;
            if (r == i + 1) {
                alpha_s[buf] = x[q];
#pragma unroll
                for (int j = 0; j < TC; ++j) a1col[buf][j] = A_GET(j, q, r);
            }
            if (r >= c_first && r <= c_last) xcol[buf][r - c_first] = x[q];
        }
        // ---- one reduction: |x[i+2:]|^2 and z_c = sum_{r >= i+2} conj(A[r, c]) x[r]
        double part = 0.0;
        double zp[2 * TC];
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const int r = tid + TT * q;
            if (r >= i + 2 && r < n) part += x[q].x * x[q].x + x[q].y * x[q].y;
        }
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            double2 sacc = make_double2(0.0, 0.0);
            const int c = c_first + j;
            if (c >= i + 1 && c < n) {
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int r = tid + TT * q;
                    if (r >= i + 2) sacc = cadd(sacc, cjmul(A_GET(j, q, r), x[q]));
                }
            }
            zp[2 * j] = sacc.x;
            zp[2 * j + 1] = sacc.y;
        }
        {
            const double zs = wave_sum16(zp, lane);
            if ((lane & 3) == 0) red[buf][wave][sum16_index(lane)] = zs;
        }
        part = wave_sum(part);
        if (lane == 0) red[buf][wave][2 * TC] = part;
        __syncthreads();
        // ---- reflector: H^H x = (beta, 0, ...), v = (1, x[i+2:] / (alpha - beta));
        //      every thread sums the wavefronts' partial |x|^2 itself
        double xnorm2 = 0.0;
#pragma unroll
        for (int w = 0; w < NWAVE; ++w) xnorm2 += red[buf][w][2 * TC];
        const double2 alpha = alpha_s[buf];
        const double anorm2 = alpha.x * alpha.x + alpha.y * alpha.y + xnorm2;
        // tau = 0 (H = I) when x is already (real alpha, 0, ...) or negligible
        const bool reflect = !(xnorm2 == 0.0 && alpha.y == 0.0) && anorm2 > 1e-300;
        double2 tau = make_double2(0.0, 0.0);
        double beta = alpha.x;
        double2 scale = make_double2(0.0, 0.0);
        if (reflect) {
            beta = -copysign(sqrt(anorm2), alpha.x);
            tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            const double2 am = make_double2(alpha.x - beta, alpha.y);     // scale = 1 / (alpha - beta)
            const double den = am.x * am.x + am.y * am.y;
            scale = make_double2(am.x / den, -am.y / den);
        }
        double2 v[TQ];
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const int r = tid + TT * q;
            v[q] = make_double2(0.0, 0.0);
            if (r == i + 1)
                v[q] = make_double2(1.0, 0.0);
            else if (r >= i + 2 && r < n)
                v[q] = cmul(x[q], scale);
        }
        if (wave == 0) {
            // lanes 0 .. TC-1: y and v of the owned columns, and this workgroup's share of y^H v
            double2 pdt = make_double2(0.0, 0.0);
            if (tid < TC) {
                const int c = c_first + tid;
                double2 vc = make_double2(0.0, 0.0), yc = make_double2(0.0, 0.0);
                if (c >= i + 1 && c < n) {
                    double zr = 0.0, zi = 0.0;
#pragma unroll
                    for (int w = 0; w < NWAVE; ++w) {
                        zr += red[buf][w][2 * tid];
                        zi += red[buf][w][2 * tid + 1];
                    }
                    vc = c == i + 1 ? make_double2(1.0, 0.0) : cmul(xcol[buf][tid], scale);
                    // y_c = conj(A[i+1, c]) + scale z_c
                    const double2 a1 = a1col[buf][tid];
                    yc = cadd(make_double2(a1.x, -a1.y), cmul(scale, make_double2(zr, zi)));
                    st_coh(&g.ybuf[(int64_t)buf * n + c], yc);
                }
                vcol[buf][tid] = vc;
                ycol[buf][tid] = yc;
                pdt = cjmul(yc, vc);
            }
            static_assert(TC == 8, "the y^H v share sums lanes 0..7");
            pdt.x += xor_lane<4>(pdt.x, lane);
            pdt.y += xor_lane<4>(pdt.y, lane);
            pdt.x += xor_lane<2>(pdt.x, lane);
            pdt.y += xor_lane<2>(pdt.y, lane);
            pdt.x += xor_lane<1>(pdt.x, lane);
            pdt.y += xor_lane<1>(pdt.y, lane);
            if (tid == 0) st_coh(&g.pdot[(int64_t)buf * P + wg], pdt);
        }
        // d_i before x is reused
        double d_i = 0.0;
#pragma unroll
        for (int q = 0; q < TQ; ++q)
            if (tid + TT * q == i) d_i = x[q].x;
        publish(g.wg_flag + wg, i + 1);
        // the first participant (the owner of column i + 1) records d_i, e_i, tau_i and the
        // reflector; issued after the flag so that the publication does not wait for them
        if (wg == g0) {
#pragma unroll
            for (int q = 0; q < TQ; ++q) {
                const int r = tid + TT * q;
                if (r < n) {
                    st_coh1(&g.vh_re[(int64_t)i * n + r], v[q].x);
                    st_coh1(&g.vh_im[(int64_t)i * n + r], -v[q].y);
                }
                if (r == i) st_coh1(&g.d[i], d_i);
            }
            if (tid == 0) {
                st_coh1(&g.e[i], beta);
                st_coh(&g.tau[i], tau);
            }
        }
        // ---- wait for every workgroup's y entries and partial y^H v (and the
        //      column published one step earlier)
        const bool ok = wait_step_acquire(g.wg_flag, g.grp_flag, g0, P, wg, i + 1, g.abort_flag);
        if (__syncthreads_or(!ok)) return;
        // every published value of this step is complete now: issue the loads of y and of
        // the partial y^H v together, so that their latencies overlap
        double2 yq[TQ];
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const int r = tid + TT * q;
            yq[q] = (r >= i + 1 && r < n) ? ld_coh(&g.ybuf[(int64_t)buf * n + r]) : make_double2(0.0, 0.0);
        }
        const double2 y1 = ld_coh(&g.ybuf[(int64_t)buf * n + i + 1]);
        // every wavefront sums the participants' (<= 256) shares of y^H v itself (no barrier);
        // the loads are issued together with those of y and of the next column
        double pd[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = g0 + lane + 64 * q;
            pd[q] = k < P ? ld_coh1(&g.pdot[(int64_t)buf * P + k].x) : 0.0;
        }
        // next column x_{i+1} = A[:, i+1] as updated by steps 0 .. i-1: published by its owner
        // in step i-1, before that owner's flag of step i
        double2 cv[TQ];
        {
            const double2* src = g.colbuf + (int64_t)((i + 1) & 1) * n;
#pragma unroll
            for (int q = 0; q < TQ; ++q) {
                const int r = tid + TT * q;
                cv[q] = make_double2(0.0, 0.0);
                if (r >= i + 1 && r < n) cv[q] = (i == 0) ? g.a[r + lda] : ld_coh(&src[r]);
            }
        }
        const double pdr = wave_sum(pd[0] + pd[1] + pd[2] + pd[3]);
        // w = tau y + alpha_w v, alpha_w = -|tau|^2 (y^H v) / 2
        const double alw = -0.5 * (tau.x * tau.x + tau.y * tau.y) * pdr;
        double2 w[TQ];
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const int r = tid + TT * q;
            w[q] = make_double2(0.0, 0.0);
            if (r >= i + 1 && r < n) {
                const double2 ty = cmul(tau, yq[q]);
                w[q] = make_double2(ty.x + alw * v[q].x, ty.y + alw * v[q].y);
            }
        }
        // w at row i+1 (v there is 1): the scalar of the next column's update
        const double2 ty1 = cmul(tau, y1);
        const double2 w1 = make_double2(ty1.x + alw, ty1.y);
        // ---- rank-2 update of the owned columns; column i+2 first, then published
        const int j2 = (i + 2 < n && wg == (i + 2) / TC) ? (i + 2) % TC : -1;
        if (j2 >= 0) {
#pragma unroll
            for (int j = 0; j < TC; ++j) {
                if (j != j2) continue;
                UPDATE_COL(j);
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int r = tid + TT * q;
                    // slot (i+2) & 1 == buf: read after the next step's wait
                    if (r >= i + 1 && r < n) st_coh(&g.colbuf[(int64_t)buf * n + r], A_GET(j, q, r));
                }
            }
        }
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            const int c = c_first + j;
            if (j == j2 || c < i + 1 || c >= n) continue;
            UPDATE_COL(j);
        }
        // ---- next column: x_{i+1} = A[:, i+1] (after step i-1, loaded above) - v conj(w_{i+1}) - w
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const double2 t1 = cjmul(w1, v[q]);
            x[q] = make_double2(cv[q].x - t1.x - w[q].x, cv[q].y - t1.y - w[q].y);
        }
    }
    // last diagonal entry: column n-1 after step n-2 (its owner takes part in every step)
    if (wg == (n - 1) / TC) {
#pragma unroll
        for (int q = 0; q < TQ; ++q)
            if (tid + TT * q == n - 1) g.d[n - 1] = x[q].x;
    }
}
#undef UPDATE_COL
#undef A_SUB
#undef A_GET

// Orders up to 128: the reduction of a small truncation is pure latency, so one workgroup
// holds the whole matrix in registers and the steps are separated by barriers instead of
// cross-workgroup waits.  Thread t keeps column t % 128 at the interleaved rows
// t / 128 + 8 q.  Same reflector convention and outputs as hetrd_kernel.
constexpr int SN = 128;             // largest order
constexpr int ST = 1024;            // threads
constexpr int SRB = ST / SN;        // row blocks
constexpr int SQ = SN / SRB;        // rows per thread

__global__ __launch_bounds__(ST, 1) void hetrd_small_kernel(TrArgs g) {
    __shared__ double2 xs[SN], vs[SN], ys[SN], wsh[SN];
    __shared__ double2 part[SRB][SN];
    __shared__ double red[2];
    __shared__ double xn2_s;
    const int tid = threadIdx.x, n = g.n;
    const int c = tid % SN, rb = tid / SN;
    const int64_t lda = g.lda;
    double2 a[SQ];
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
        const int r = rb + SRB * q;
        a[q] = (r < n && c < n) ? g.a[r + c * lda] : make_double2(0.0, 0.0);
    }
    for (int i = 0; i + 1 < n; ++i) {
        // column i (updated by steps 0 .. i-1)
        if (c == i) {
#pragma unroll
            for (int q = 0; q < SQ; ++q) {
                const int r = rb + SRB * q;
                if (r < n) xs[r] = a[q];
            }
        }
        __syncthreads();
        if (tid < 64) {
            double p = 0.0;
            for (int r = i + 2 + tid; r < n; r += 64) p += xs[r].x * xs[r].x + xs[r].y * xs[r].y;
            p = wave_sum(p);
            if (tid == 0) {
                xn2_s = p;
                g.d[i] = xs[i].x;
            }
        }
        __syncthreads();
        // reflector: H^H x = (beta, 0, ...), v = (1, x[i+2:] / (alpha - beta))
        const double xnorm2 = xn2_s;
        const double2 alpha = xs[i + 1];
        const double anorm2 = alpha.x * alpha.x + alpha.y * alpha.y + xnorm2;
        const bool reflect = !(xnorm2 == 0.0 && alpha.y == 0.0) && anorm2 > 1e-300;
        double2 tau = make_double2(0.0, 0.0);
        double beta = alpha.x;
        double2 scale = make_double2(0.0, 0.0);
        if (reflect) {
            beta = -copysign(sqrt(anorm2), alpha.x);
            tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            const double2 am = make_double2(alpha.x - beta, alpha.y);
            const double den = am.x * am.x + am.y * am.y;
            scale = make_double2(am.x / den, -am.y / den);
        }
        if (tid < SN) {
            const int r = tid;
            double2 vr = make_double2(0.0, 0.0);
            if (r == i + 1)
                vr = make_double2(1.0, 0.0);
            else if (r >= i + 2 && r < n)
                vr = cmul(xs[r], scale);
            vs[r] = vr;
            if (r < n) {
                g.vh_re[(int64_t)i * n + r] = vr.x;
                g.vh_im[(int64_t)i * n + r] = -vr.y;
            }
        }
        if (tid == 0) {
            g.e[i] = beta;
            g.tau[i] = tau;
        }
        __syncthreads();
        // y_c = sum_r conj(A[r, c]) v_r: partial sums over this thread's rows
        double2 sp = make_double2(0.0, 0.0);
        if (c >= i + 1 && c < n) {
#pragma unroll
            for (int q = 0; q < SQ; ++q) {
                const int r = rb + SRB * q;
                if (r >= i + 1 && r < n) sp = cadd(sp, cjmul(a[q], vs[r]));
            }
        }
        part[rb][c] = sp;
        __syncthreads();
        if (tid < SN) {
            double2 y = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < SRB; ++k) y = cadd(y, part[k][tid]);
            ys[tid] = y;
            double pd = wave_sum(cjmul(y, vs[tid]).x);      // Re(y^H v), over two waves
            if ((tid & 63) == 0) red[tid >> 6] = pd;
        }
        __syncthreads();
        // w = tau y - (|tau|^2 Re(y^H v) / 2) v
        const double alw = -0.5 * (tau.x * tau.x + tau.y * tau.y) * (red[0] + red[1]);
        if (tid < SN) {
            const int r = tid;
            double2 w = make_double2(0.0, 0.0);
            if (r >= i + 1 && r < n) {
                const double2 ty = cmul(tau, ys[r]);
                w = make_double2(ty.x + alw * vs[r].x, ty.y + alw * vs[r].y);
            }
            wsh[r] = w;
        }
        __syncthreads();
        // A[r, c] -= v_r conj(w_c) + w_r conj(v_c) on the trailing block
        if (c >= i + 1 && c < n) {
            const double2 wc = wsh[c], vc = vs[c];
#pragma unroll
            for (int q = 0; q < SQ; ++q) {
                const int r = rb + SRB * q;
                if (r >= i + 1 && r < n) {
                    const double2 t1 = cjmul(wc, vs[r]);
                    const double2 t2 = cjmul(vc, wsh[r]);
                    a[q].x -= t1.x + t2.x;
                    a[q].y -= t1.y + t2.y;
                }
            }
        }
    }
    // last diagonal entry, after step n-2
    if (c == n - 1) {
#pragma unroll
        for (int q = 0; q < SQ; ++q)
            if (rb + SRB * q == n - 1) g.d[n - 1] = a[q].x;
    }
}

// Full Hermitian matrix, column-major interleaved, from the row-major planar
// Gram matrix whose lower triangle (row >= column) is valid.
__global__ __launch_bounds__(256) void herm_full_kernel(const double* __restrict__ re, const double* __restrict__ im,
                                                       int n, double2* __restrict__ out) {
    __shared__ double2 lo[64][65];   // lo[a][b] = rho[bi + a][bj + b]  (valid for row >= col)
    __shared__ double2 up[64][65];   // up[a][b] = rho[bj + a][bi + b]
    const int bi = blockIdx.x * 64, bj = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int a = ty; a < 64; a += 4) {
        const int r1 = bi + a, c1 = bj + tx;
        if (r1 < n && c1 < n && r1 >= c1) lo[a][tx] = make_double2(re[(int64_t)r1 * n + c1], im[(int64_t)r1 * n + c1]);
        const int r2 = bj + a, c2 = bi + tx;
        if (r2 < n && c2 < n && r2 >= c2) up[a][tx] = make_double2(re[(int64_t)r2 * n + c2], im[(int64_t)r2 * n + c2]);
    }
    __syncthreads();
    // out(i, j) at i + j n: i = bi + x (fastest), j = bj + y
    for (int y = ty; y < 64; y += 4) {
        const int i = bi + tx, j = bj + y;
        if (i >= n || j >= n) continue;
        double2 v;
        if (i >= j) {
            v = lo[tx][y];                  // rho[i][j]
        } else {
            const double2 u = up[y][tx];    // rho[j][i]
            v = make_double2(u.x, -u.y);
        }
        out[i + (int64_t)j * n] = v;
    }
}

// T of the compact WY form H_0 H_1 ... H_{m-1} = I - V T V^H (T upper
// triangular): T[i][i] = tau_i, T[i][j] = -tau_j sum_{l=i}^{j-1} T[i][l] S[l][j]
// for i < j, with S = V^H V.  Row i depends only on itself: one wave per row,
// lane l holding T[i][l]; one workgroup per block of reflectors.
constexpr int WY_MAX = 64;
constexpr int WY_THREADS = 1024;
// Workgroup z forms the 64 x 64 diagonal sub-block q = z mod (nb / 64) of the
// T factor of block b = z / (nb / 64) (S and T planar row-major nb x nb per
// block, leading dimension nb; tau of the sub-block's reflectors at 64 z).
__global__ __launch_bounds__(WY_THREADS) void wy_t_kernel(const double* __restrict__ s_re, const double* __restrict__ s_im,
                                                        const double2* __restrict__ tau, double* __restrict__ t_re,
                                                        double* __restrict__ t_im, int nb) {
    __shared__ double2 S[WY_MAX][WY_MAX + 1];
    const int sub = nb / WY_MAX;
    const int64_t b = blockIdx.x / sub, q = blockIdx.x % sub;
    const int64_t off = b * nb * nb + q * WY_MAX * (nb + 1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double* sr = s_re + off;
    const double* si = s_im + off;
    for (int idx = threadIdx.x; idx < WY_MAX * WY_MAX; idx += WY_THREADS)
        S[idx / WY_MAX][idx % WY_MAX] = make_double2(sr[(idx / WY_MAX) * nb + idx % WY_MAX],
                                                     si[(idx / WY_MAX) * nb + idx % WY_MAX]);
    __syncthreads();
    const double2* tb = tau + (int64_t)blockIdx.x * WY_MAX;
    for (int i = wave; i < WY_MAX; i += WY_THREADS / 64) {
        double2 t = make_double2(0.0, 0.0);        // T[i][lane]
        if (lane == i) t = tb[i];
        for (int j = i + 1; j < WY_MAX; ++j) {
            double2 p = make_double2(0.0, 0.0);
            if (lane >= i && lane < j) p = cmul(t, S[lane][j]);
            const double sx = wave_sum(p.x), sy = wave_sum(p.y);
            if (lane == j) {
                const double2 tt = cmul(tb[j], make_double2(sx, sy));
                t = make_double2(-tt.x, -tt.y);
            }
        }
        t_re[off + (int64_t)i * nb + lane] = t.x;
        t_im[off + (int64_t)i * nb + lane] = t.y;
    }
}

// The k eigenvectors of the largest eigenvalues (ascending order input, real
// n x n column-major) as planar complex row-major n x k, largest first.
__global__ __launch_bounds__(256) void top_real_kernel(const double* __restrict__ ev, int n, int k,
                                                      double* __restrict__ ore, double* __restrict__ oim) {
    const int64_t total = (int64_t)n * k;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx % k, r = idx / k;
        ore[idx] = ev[r + (int64_t)(n - 1 - c) * n];
        oim[idx] = 0.0;
    }
}

}  // namespace

int wy_block(int n) { return n > 512 ? 4 * WY_MAX : WY_MAX; }

hipError_t wy_t_diag_factors(const double* s_re, const double* s_im, int nblk, int nb, const double* tau_z,
                             double* t_re, double* t_im, hipStream_t stream) {
    if (nblk < 1 || nb < WY_MAX || nb % WY_MAX != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wy_t_kernel, dim3(nblk * (nb / WY_MAX)), dim3(WY_THREADS), 0, stream, s_re, s_im,
                       (const double2*)tau_z, t_re, t_im, nb);
    return hipGetLastError();
}

hipError_t take_top_real_eigvecs(const double* evec, int n, int k, double* out_re, double* out_im, hipStream_t stream) {
    const int64_t total = (int64_t)n * k;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(top_real_kernel, dim3((unsigned)g), dim3(256), 0, stream, evec, n, k, out_re, out_im);
    return hipGetLastError();
}

int hetrd_max_n() { return TMAXN; }

size_t hetrd_workspace_bytes(int n) {
    const int P = (n + TC - 1) / TC;
    return sizeof(double2) * (4 * (size_t)n + 2 * (size_t)P) + sizeof(int) * (size_t)(P + 2 + HG * GF_STRIDE) + 256;
}

hipError_t hermitian_full_colmajor(const double* re, const double* im, int n, double* out_z, hipStream_t stream) {
    const dim3 grid((n + 63) / 64, (n + 63) / 64);
    hipLaunchKernelGGL(herm_full_kernel, grid, dim3(256), 0, stream, re, im, n, (double2*)out_z);
    return hipGetLastError();
}

namespace {
// Arguments of one reduction over its workspace; clears its flags on `stream`.
hipError_t prepare(const TrRequest& r, TrArgs& g, hipStream_t stream) {
    if (r.n < 2 || r.n > TMAXN) return hipErrorInvalidValue;
    if (r.ws_bytes < hetrd_workspace_bytes(r.n)) return hipErrorInvalidValue;
    g.a = (const double2*)r.a_z;
    g.vh_re = r.vh_re;
    g.vh_im = r.vh_im;
    g.n = r.n;
    g.lda = r.n;
    g.P = (r.n + TC - 1) / TC;
    g.d = r.d;
    g.e = r.e;
    g.tau = (double2*)r.tau_z;
    char* p = (char*)r.ws;
    g.colbuf = (double2*)p;
    g.ybuf = g.colbuf + 2 * (size_t)r.n;
    g.pdot = g.ybuf + 2 * (size_t)r.n;
    int* flags = (int*)(g.pdot + 2 * (size_t)g.P);
    g.col_flag = flags;
    g.abort_flag = flags + 1;
    g.wg_flag = flags + 2;
    g.grp_flag = flags + 2 + g.P;
    if (r.abort_flag) *r.abort_flag = g.abort_flag;
    return hipMemsetAsync(flags, 0, sizeof(int) * (size_t)(g.P + 2 + HG * GF_STRIDE), stream);
}
}  // namespace

int hetrd_batch_max() { return TR_MAXB; }
int hetrd_workgroups(int n) { return n <= SN ? 1 : (n + TC - 1) / TC; }

hipError_t hetrd_persistent_multi(const TrRequest* reqs, int count, hipStream_t stream) {
    if (count < 1 || count > TR_MAXB) return hipErrorInvalidValue;
    TrBatch b;
    b.count = count;
    b.first[0] = 0;
    for (int i = 0; i < count; ++i) {
        if (reqs[i].n <= SN) return hipErrorInvalidValue;   // small orders use the one-workgroup kernel
        const hipError_t err = prepare(reqs[i], b.a[i], stream);
        if (err != hipSuccess) return err;
        b.first[i + 1] = b.first[i] + b.a[i].P;
    }
    void* args[] = {&b};
    return hipLaunchCooperativeKernel((const void*)hetrd_kernel, dim3(b.first[count]), dim3(TT), args, 0, stream);
}

hipError_t hetrd_persistent(const double* a_z, int n, double* d, double* e, double* tau_z, double* vh_re,
                            double* vh_im, void* ws, size_t ws_bytes, int** abort_flag, hipStream_t stream) {
    const TrRequest r{a_z, n, d, e, tau_z, vh_re, vh_im, ws, ws_bytes, abort_flag};
    if (n > SN) return hetrd_persistent_multi(&r, 1, stream);
    TrArgs g;
    const hipError_t err = prepare(r, g, stream);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(hetrd_small_kernel, dim3(1), dim3(ST), 0, stream, g);
    return hipGetLastError();
}

}  // namespace mpsk
