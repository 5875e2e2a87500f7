// bed_big.hip -- symmetric matrices of order 64 < n <= 128 in binary32.  The
// divide step of the note applies at any size (Sec. 2.1): one tearing step
// above the n <= 64 solver, whose halves then fit a single team, and the top
// merge (Sec. 2.3) on one 512-thread team per matrix, with the merge code of
// the n <= 64 solver laid out for 128 elements.
//
//   k_big_reduce  Householder tridiagonalization T = Q_H^T A Q_H with binary64
//                 arithmetic (binary32 for eigenvalues alone, as for n <= 64);
//                 T torn at s = floor(n/2) (Eq. (3)) into T1 (s x s) and T2
//                 ((n-s) x (n-s)), written as their diagonals; with
//                 eigenvectors the reflectors go to the workspace
//   k_big_qh      Q_H = H_0 ... H_{n-3} from the reflectors in compact-WY
//                 blocks on binary64 MFMA tiles, staged in the Q output
//   children      the n <= 64 solver on tridiagonal input (no reduction, no
//                 back-transform) solves T1 and T2; for eigenvalues alone it
//                 returns only the end rows of their eigenvector matrices
//   k_big_merge   z = [sgn(beta) Q1(s-1, :), Q2(0, :)] (Eq. (5)), deflation,
//                 secular roots, Loewner vectors and the merge matrix M;
//                 Q = Q_H (diag(Q1, Q2) M) on 16x16x4 MFMA tiles, sign rule
// Every kernel fits two 512-thread teams per CU (at most 128 VGPRs and 80 KB
// of LDS each).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <mutex>
#include <type_traits>

#include "bed_host.hpp"
#include "bed_internal.hpp"
#include "bed_lru.hpp"
#include "bed_syevd.hpp"

namespace bed {
namespace big {

constexpr int BN = NMAX_BIG;  // largest order
constexpr int BT = 512;       // threads per matrix (8 waves)
constexpr int CPL = BN * BN / BT;  // matrix entries per lane (32)

struct Meta {
    float beta;  // coupling b_{s-1} of the torn tridiagonal matrix (scaled)
    int shift;   // the matrix was solved as 2^shift A
    int bad;     // non-finite input
    int pad;
};

// Workspace of one batch: children (tridiagonal input, eigenvectors,
// eigenvalues, info), per-matrix meta data and, with eigenvectors, the
// reflectors.  For even n the two children's arrays are
// contiguous (child 2 of matrix b follows all children 1), so one uniform
// launch solves both.
struct Ws {
    float *c1, *c2;  // children (diagonal, then off-diagonal), 2 n1 and 2 n2 values apart
    float *q1, *q2;  // their eigenvectors
    float *l1, *l2;  // their eigenvalues
    int32_t *i1, *i2;
    Meta *meta;
    float *v;    // with eigenvectors: reflectors v_0 .. v_{n-3} (binary32 rows of n)
    float *tau;  // their tau (zero for a skipped step), n per matrix
    float *e1, *e2;  // eigenvalues only: the children's first and last eigenvector
                     // rows (2 n1 and 2 n2 values apart), in the q1 space
};

// ------------------------------------------------------------------ reduction
// About 66 KB, so that two teams share a CU: the load staging and the
// buffers of the steps share the space.
template <typename H>
struct RedSmem {
    static constexpr int SLD = BN + 1;  // odd stride
    union {
        float st[BN * SLD];  // load staging (binary32)
        struct {
            H xe[2][BN][2];  // pivot column as (x_r, 0) below row k + 1, (0, 1) at it
                             // (v = x rv0 + e), by step parity: the update of step k
                             // reads it while the next owner group writes step k + 1's
            H w[BN];         // w = p - (tau/2)(p^T v) v
            H part[4][BN];   // per column group: partial products
            H red[8];        // per wave: partial sums
            H red2[8];
        } s;
    } u;
    float a[BN], b[BN];
    int badw[BT / 64];
    int expw[BT / 64];
};

// Arithmetic type H: binary64 when Q_H is formed (eigenvectors), binary32
// for eigenvalues alone (as for n <= 64).  Lane (r, g) = (t % 128, t / 128)
// keeps row r of the columns c = g + 4j (j < 32) in registers; the four column groups are whole waves, so
// reads of v and w at a lane's columns are wave-wide broadcasts.  Step k:
// the owner group of column k publishes it with the partial of ||x||^2 (one
// barrier), every lane forms the reflector (Golub-Van Loan 8.3, as for n <=
// 64), its partial of p = tau A v and of v^T A v (second barrier), p and w
// (third barrier), then the rank-2 update A -= v w^T + w v^T of its entries.
// With eigenvectors the reflectors (rounded to binary32) and their tau go to
// the workspace for k_big_qh.  Two teams per CU: at most 128 VGPRs.
template <typename H>
__global__ void __launch_bounds__(BT, 4)
k_big_reduce(const float *__restrict__ A, int n, int64_t batch, Ws ws)
{
    __shared__ RedSmem<H> S;
    const int64_t bi = blockIdx.x;
    if (bi >= batch) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int r = t & (BN - 1), g = t >> 7;
    const int s = n / 2, n1 = s, n2 = n - s;
    const float *Ab = A + bi * n * n;

    // load (coalesced, staged in LDS as binary32 over the reflector buffer)
    float *St = S.u.st;
    constexpr int SLD = RedSmem<H>::SLD;
    {
        // lane (j, i0) = (t % BN, t / BN) reads rows i0, i0 + 4, ... at column
        // j: every load is issued before the first LDS write
        const int j = t & (BN - 1), i0 = t / BN;
        float ld[BN * BN / BT];
#pragma unroll
        for (int q = 0; q < BN * BN / BT; ++q) {
            const int i = i0 + (BT / BN) * q;
            const bool in = i < n && j < n;
            const float v = Ab[in ? i * n + j : 0];  // clamped address: no branch
            ld[q] = in ? v : 0.f;
        }
#pragma unroll
        for (int q = 0; q < BN * BN / BT; ++q) St[(i0 + (BT / BN) * q) * SLD + j] = ld[q];
    }
    __syncthreads();
    H ar[CPL];
    bool bad = false;
    float amax = 0.f;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int c = g + 4 * j;
        float v = 0.f;
        if (r < n && c < n) {
            v = (c <= r) ? St[r * SLD + c] : St[c * SLD + r];  // lower triangle
            bad = bad || !f_finite(v);
            amax = f_max(amax, f_abs(v));
        }
        ar[j] = H(v);
    }
    {
        const bool wb = __ballot(bad) != 0;
        const int we = group_max<64>(exp_field(amax), lane);
        if (lane == 0) {
            S.badw[wave] = wb ? 1 : 0;
            S.expw[wave] = we;
        }
    }
    __syncthreads();
    int anybad = 0, emax = 0;
#pragma unroll
    for (int w = 0; w < BT / 64; ++w) {
        anybad |= S.badw[w];
        emax = max(emax, S.expw[w]);
    }
    // exact power-of-two scaling to max |a_ij| in [1/2, 1), as for n <= 64
    int sh = (emax == 0) ? 0 : fexp<float>::BIAS - 1 - emax;
    sh = min(max(sh, -fexp<float>::SMAX), fexp<float>::SMAX);
    if (anybad) {
        for (int e = t; e < 2 * n1; e += BT) ws.c1[bi * 2 * n1 + e] = 0.f;
        for (int e = t; e < 2 * n2; e += BT) ws.c2[bi * 2 * n2 + e] = 0.f;
        if (t == 0) ws.meta[bi] = Meta{0.f, 0, 1, 0};
        return;
    }
    const H hs = H(fexp<float>::pow2(sh));
#pragma unroll
    for (int j = 0; j < CPL; ++j) ar[j] *= hs;
    __syncthreads();  // the staging buffer becomes the reflector store

    const int gs = __builtin_amdgcn_readfirstlane(g);
    const int rhi = __builtin_amdgcn_readfirstlane((wave & 1) * 64 + 63);  // the wave's last row
    auto wlive = [&](const int k) { return rhi > k; };
    for (int k = 0; k < n - 2; ++k) {
        const int gk = k & 3, jk = k >> 2;
        typedef H H2 __attribute__((ext_vector_type(2)));
        H2 *xe = reinterpret_cast<H2 *>(S.u.s.xe[k & 1]);
        if (g == gk) {
            const H x = pick<CPL>(ar, jk);
            const bool below = r > k + 1 && r < n;
            xe[r] = H2{below ? x : H(0), (r == k + 1) ? H(1) : H(0)};
            if (r == k + 1) S.u.s.red[2] = x;
            if (r == k) S.a[k] = float(x);
            const H s2 = wave_sum_all(below ? x * x : H(0));
            if (lane == 0) S.u.s.red[__builtin_amdgcn_readfirstlane(wave & 1)] = s2;
        }
        __syncthreads();
        const H x0 = S.u.s.red[2];
        const H sig = S.u.s.red[0] + S.u.s.red[1];
        const HhRefl<H> h = hh_reflector<float>(x0, sig);
        // v = (1, x_{k+2..} rv0) = x' rv0 + e_{k+1} with x' the pivot column
        // zeroed at rows <= k + 1 (exact: the products are as before, and the
        // pivot entry is exactly 1 without a per-column select); x is zero
        // past k + 1 too when sig = 0
        const H2 xr2 = xe[r];
        const H vr = fma(xr2.x, h.rv0, xr2.y);
        // Dead work is skipped by wave-uniform branches: chunks of eight of a
        // lane's columns that lie at or left of column k (v is zero there and
        // the columns are never read again), and whole waves whose rows are
        // all <= k (their p and w are not used).
        // v at this wave's columns c = g + 4j, the same for all its lanes: lane
        // j forms column j's entry from one pivot pair and the values are
        // broadcast into scalar registers (one LDS read per lane instead of
        // one per column), where they stay for the update
        const H2 xl = xe[g + 4 * (lane & (CPL - 1))];
        const H vl = fma(xl.x, h.rv0, xl.y);
        H vc[CPL];
        H pp = H(0);
        if (wlive(k)) {
            // independent chains against the FMA latency
            constexpr int NC = 4;
            H pq[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) pq[i] = H(0);
#pragma unroll
            for (int q = 0; q < CPL / 8; ++q) {
                if (gs + 32 * q + 28 <= k) continue;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int j = 8 * q + jj;
                    vc[j] = bcast(vl, j);
                    pq[jj % NC] = fma(ar[j], vc[j], pq[jj % NC]);
                }
            }
            pp = (pq[0] + pq[1]) + (pq[2] + pq[3]);
            S.u.s.part[g][r] = pp;
        }
        const H pv = wave_sum_all(vr * pp);  // partial of v^T A v
        if (lane == 0) S.u.s.red2[wave] = pv;
        if constexpr (std::is_same<H, double>::value) {
            if (g == 0 && r < n) ws.v[(bi * (n - 2) + k) * n + r] = float(vr);
            if (t == 0) ws.tau[bi * n + k] = float(h.tau);
        }
        if (t == 0) S.b[k] = float(h.alpha);
        __syncthreads();
        const H p = h.tau * (S.u.s.part[0][r] + S.u.s.part[1][r] + S.u.s.part[2][r] + S.u.s.part[3][r]);
        H vav = H(0);
#pragma unroll
        for (int w = 0; w < BT / 64; ++w) vav += S.u.s.red2[w];
        const H ptv = h.tau * vav;  // p^T v = tau v^T A v
        const H wr = (r > k) ? p - H(0.5) * h.tau * ptv * vr : H(0);
        if (g == 0) S.u.s.w[r] = wr;
        __syncthreads();
        if (wlive(k)) {
#pragma unroll
            for (int q = 0; q < CPL / 8; ++q) {
                if (gs + 32 * q + 28 <= k) continue;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int j = 8 * q + jj;
                    const int c = g + 4 * j;
                    ar[j] = fma(-vr, S.u.s.w[c], fma(-wr, vc[j], ar[j]));
                }
            }
        }
    }
    // last 2 x 2 block
    {
        const int c0 = n - 2, c1 = n - 1;
        if (g == (c0 & 3)) {
            const H x = pick<CPL>(ar, c0 >> 2);
            if (r == c0) S.a[c0] = float(x);
            if (r == c1) S.b[c0] = float(x);
        }
        if (g == (c1 & 3) && r == c1) S.a[c1] = float(pick<CPL>(ar, c1 >> 2));
    }
    __syncthreads();

    // tear (Eq. (3)): the two children's diagonals and off-diagonals
    {
        const float beta = S.b[s - 1];
        const float rho = f_abs(beta);
        float *C1 = ws.c1 + bi * 2 * n1;
        float *C2 = ws.c2 + bi * 2 * n2;
        for (int e = t; e < 2 * n1 - 1; e += BT)
            C1[e] = (e < n1) ? S.a[e] - (e == s - 1 ? rho : 0.f) : S.b[e - n1];
        for (int e = t; e < 2 * n2 - 1; e += BT)
            C2[e] = (e < n2) ? S.a[s + e] - (e == 0 ? rho : 0.f) : S.b[s + e - n2];
        if (t == 0) ws.meta[bi] = Meta{beta, sh, 0, 0};
    }
}

// ------------------------------------------------------------------ Q_H
// Q_H = H_0 H_1 ... H_{n-3} in compact-WY blocks of 16 reflectors,
// H_{16b} ... H_{16b+15} = I - V_b T_b V_b^T (T_b upper triangular), applied to
// the identity for b = last .. 0 on 16x16x4 binary64 MFMA tiles.  The
// reflectors come rounded to binary32 (exact to convert back) and are staged
// in LDS at odd stride; the binary64 Gram matrices G_b = V_b^T V_b of the
// rounded reflectors and then the T factors sit in packed upper triangles
// (element (i, j) at j (j + 1) / 2 + i).  T is formed with tau_j = 2 / G(j, j),
// so each block is exactly orthogonal for the reflectors as stored, up to
// binary64 rounding; only the final binary32 rounding of Q_H remains
// (binary32 products here would add a few 1e-6 to ||Q^T Q - I||_F at n = 128).
// One wave per block forms G_b and T_b; after one barrier each wave keeps a
// 16-column tile of Q in accumulators through all blocks.
struct QhSmem {
    static constexpr int VLD = BN + 1;
    static constexpr int TP = 136;  // packed 16 x 16 upper triangle
    float V[BN * VLD];
    double tf[(BN / 16) * TP];  // G_b, then T_b
};

__global__ void __launch_bounds__(BT, 4)  // two teams per CU
k_big_qh(int n, int64_t batch, float *__restrict__ Qh, Ws ws)
{
    __shared__ QhSmem S;
    using MF = Mf<double>;
    constexpr int VLD = QhSmem::VLD;
    constexpr int TP = QhSmem::TP;
    const int64_t bi = blockIdx.x;
    if (bi >= batch) return;
    if (ws.meta[bi].bad) return;  // the merge writes NaN
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nb = n - 2;  // reflectors
    const int NB = (nb + 15) / 16;
    {
        // lane (j, i0) = (t % BN, t / BN) stages rows i0, i0 + 4, ... at column
        // j (zero outside the nb x n reflector block), loads first
        constexpr int RPL = BN * BN / BT, RS = BT / BN;
        const int j = t & (BN - 1), i0 = t / BN;
        const float *Vb = ws.v + bi * nb * n;
        float ld[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int i = i0 + RS * q;
            ld[q] = Vb[(i < nb && j < n) ? i * n + j : 0];
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int i = i0 + RS * q;
            S.V[i * VLD + j] = (i < nb && j < n) ? ld[q] : 0.f;
        }
    }
    __syncthreads();
    auto tix = [](int i, int j) { return ((j * (j + 1)) >> 1) + i; };  // i <= j
    const int i16 = lane & 15;
    for (int bk = wave; bk < NB; bk += BT / 64) {
        const int k0 = 16 * bk;
        double *tb = S.tf + bk * TP;
        // G_b: one MFMA chain per row tile at or below the block (rows <= k0 of
        // its reflectors are zero), summed
        MF::acc g = MF::zero();
#pragma unroll
        for (int rt = 0; rt < BN / 16; ++rt) {
            if (rt < bk || 16 * rt >= n) continue;
            MF::acc gt = MF::zero();
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double vv = S.V[(k0 + i16) * VLD + 16 * rt + MF::crow(lane, s4)];
                gt = MF::mma(vv, vv, gt);
            }
            g += gt;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gr = MF::crow(lane, v);
            if (gr <= i16) tb[tix(gr, i16)] = g[v];
        }
        wave_sync();
        // T_b: T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j); lane i <
        // 16 forms row i, then (all reads of G_b done) writes it over G_b
        // tau_j = 2 / G(j, j) on lane j (zero marks a skipped step: v = e_{k+1}
        // stored, no reflection), then broadcast
        double tl = 0.0;
        if (lane < 16 && k0 + lane < nb && ws.tau[bi * n + k0 + lane] != 0.f)
            tl = 2.0 / tb[tix(lane, lane)];
        if (lane < 16) {
            double trow[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double tj = __shfl(tl, j);
                // column j's loads are made to wait for T(i, j - 1) through an
                // empty asm (hoisting all 120 would exhaust the registers)
                int cb = tix(0, j);
                if (j > 0) asm volatile("" : "+v"(cb) : "v"(trow[j - 1]));
                double acc = 0.0;
#pragma unroll
                for (int kk = 0; kk < j; ++kk) acc = fma(trow[kk], tb[cb + kk], acc);
                trow[j] = (lane < j) ? -tj * acc : (lane == j ? tj : 0.0);
            }
            wave_sync();
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (lane <= j) tb[tix(lane, j)] = trow[j];
        }
    }
    __syncthreads();
    // One 16-column tile per wave.  Block b leaves a column c < 16 b of the
    // identity unchanged (v_k is zero at rows <= k), so tile ct takes only
    // the blocks b <= ct; waves w and w + 4 (one SIMD when waves are placed
    // round robin) take tiles w and 7 - w, which balances the work.
    const int ct = (wave < 4) ? wave : 11 - wave;
    if (16 * ct >= n) return;
    const int c = 16 * ct + i16;
    MF::acc qa[BN / 16];
#pragma unroll
    for (int rt = 0; rt < BN / 16; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) qa[rt][v] = (16 * rt + MF::crow(lane, v) == c) ? 1.0 : 0.0;
    for (int bk = min(NB - 1, ct); bk >= 0; --bk) {
        const int k0 = 16 * bk;
        // X = V_b^T Q (16 x 16 tile of this column block); staged rows past the
        // last reflector are zero
        MF::acc xp[2] = {MF::zero(), MF::zero()};  // two chains (MFMA latency)
#pragma unroll
        for (int rt = 0; rt < BN / 16; ++rt) {
            if (rt < bk || 16 * rt >= n) continue;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double va = S.V[(k0 + i16) * VLD + 16 * rt + MF::crow(lane, s4)];
                xp[rt & 1] = MF::mma(va, qa[rt][s4], xp[rt & 1]);
            }
        }
        MF::acc x;
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = xp[0][v] + xp[1][v];
        // Y = T_b X
        MF::acc y = MF::zero();
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int kk = MF::crow(lane, s4);
            const double ta = (kk >= i16) ? S.tf[bk * TP + tix(i16, kk)] : 0.0;
            y = MF::mma(ta, x[s4], y);
        }
        // Q -= V_b Y (its operand loads are not hoisted above X: the register
        // budget holds one product's operands at a time)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rt = 0; rt < BN / 16; ++rt) {
            if (rt < bk || 16 * rt >= n) continue;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double vb = -double(S.V[(k0 + MF::crow(lane, s4)) * VLD + 16 * rt + i16]);
                qa[rt] = MF::mma(vb, y[s4], qa[rt]);
            }
        }
    }
    float *Qb = Qh + bi * n * n;
#pragma unroll
    for (int rt = 0; rt < BN / 16; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * rt + MF::crow(lane, v);
            if (row < n && c < n) Qb[row * n + c] = float(qa[rt][v]);
        }
}

// ------------------------------------------------------------------ top merge
struct MrgSmem {
    static constexpr int LD = BN + 1;  // odd stride; column BN is the padding column of M
    // rows 0 and 1 first hold the children's eigenvalues and z; then the
    // merge matrix M; then E = diag(Q1, Q2) M
    float M[BN * LD];
    // merge state; after the secular solve, the sign candidates of Q
    struct {
        MergeArrays<float, BN> m;
    } u;
    float lout[BN];  // eigenvalues, ascending
    float red[4][2];
    uint64_t live[2], dead[2], cmask[2];
    int capped, anyrot;
};

// Per wave and column: the entry of largest magnitude of the wave's rows of Q
// (lowest row on ties), signed.
struct SignCand {
    float val;
    int row;
};

__global__ void __launch_bounds__(BT, 4)  // two teams per CU
k_big_merge(int n, int64_t batch, float *__restrict__ lam, float *__restrict__ Q,
            int32_t *__restrict__ info, Ws ws)
{
    __shared__ MrgSmem S;
    constexpr int LD = MrgSmem::LD;
    const int64_t bi = blockIdx.x;
    if (bi >= batch) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int s = n / 2, n1 = s, n2 = n - s;
    const Meta md = ws.meta[bi];
    float *Qb = Q ? Q + bi * n * n : nullptr;
    if (md.bad) {
        if (Qb)
            for (int e = t; e < n * n; e += BT) Qb[e] = f_nan<float>();
        for (int e = t; e < n; e += BT) lam[bi * n + e] = f_nan<float>();
        if (t == 0 && info) info[bi] = -1;
        return;
    }
    const float *Q1 = ws.q1 + bi * n1 * n1;
    const float *Q2 = ws.q2 + bi * n2 * n2;
    const float rho = f_abs(md.beta);
    const float sgm = (md.beta < 0.f) ? -1.f : 1.f;
    // the children's eigenvalues, and z (Eq. (5)): sgn(beta) times the last
    // row of Q1 over the first row of Q2, into rows 0 and 1 of M
    float *lamc = S.M, *zin = S.M + LD;
    if (t < n) {
        lamc[t] = (t < n1) ? ws.l1[bi * n1 + t] : ws.l2[bi * n2 + t - n1];
        if (Qb)
            zin[t] = (t < n1) ? sgm * Q1[(n1 - 1) * n1 + t] : Q2[t - n1];
        else  // the children's end rows (last row of Q1 second, first row of Q2 first)
            zin[t] = (t < n1) ? sgm * ws.e1[bi * 2 * n1 + n1 + t] : ws.e2[bi * 2 * n2 + t - n1];
    }
    if (t == 0) {
        S.capped = 0;
        S.anyrot = 0;
    }
    __syncthreads();
    // stable merge of the two ascending child lists
    if (t < n) {
        const float de = lamc[t], ze = zin[t];
        const bool left = t < n1;
        const int pos = (left ? t : t - n1) +
                        count_below(lamc + (left ? n1 : 0), left ? n2 : n1, de, !left);
        S.u.m.sd[pos] = de;
        S.u.m.sz[pos] = ze;
        S.u.m.sperm[pos] = t;
    }
    __syncthreads();
    for (int e = t; e < BN * LD; e += BT) S.M[e] = 0.f;  // the merge matrix, zero padded
    __syncthreads();

    // ---- deflation (type 1: rho |z_i| <= tol; type 2: Givens rotation of a
    // close pair), tol = 8u max(max |d|, rho z^T z), as for n <= 64 ----------
    const bool act = t < n;
    float dp = act ? S.u.m.sd[t] : 0.f, zp = act ? S.u.m.sz[t] : 0.f;
    if (wave < 2) {
        const float v0 = wave_total(zp * zp), v1 = wave_total(dp * zp * zp), v2 = wave_total(dp * dp);
        if (lane == 0) {
            S.red[0][wave] = v0;
            S.red[1][wave] = v1;
            S.red[2][wave] = v2;
        }
    }
    __syncthreads();
    const float zz0 = S.red[0][0] + S.red[0][1];
    const float dz = S.red[1][0] + S.red[1][1];
    const float d2 = S.red[2][0] + S.red[2][1];
    const float dmax = f_max(f_abs(S.u.m.sd[0]), f_abs(S.u.m.sd[n - 1]));
    const float u = fp<float>::u;
    const float tol = 8.f * u * f_max(dmax, rho * zz0);
    const float fro2 = d2 + 2.f * rho * dz + rho * rho * zz0 * zz0;  // ||node||_F^2 (Eq. (10))
    bool defl = act && (rho * f_abs(zp) <= tol);
    if (defl) zp = 0.f;
    if (act) {
        S.u.m.sdefl[t] = defl ? 1 : 0;
        S.u.m.sz[t] = zp;
        S.u.m.rpart[t] = -1;
    }
    {
        const uint64_t lv = __ballot(act && !defl);
        if (wave < 2 && lane == 0) S.live[wave] = lv;
    }
    __syncthreads();
    // Pairs of consecutive live elements that may pass the type-2 test (with
    // a factor 2 of slack for the different rounding of this test) mark their
    // second element as a candidate.
    bool cand = false;
    if (act && !defl) {
        const uint64_t l0 = S.live[0], l1 = S.live[1];
        int prev = -1;
        if (t >= 64) {
            const uint64_t bl = l1 & lane_range(0, t - 64);
            prev = bl ? 64 + 63 - __clzll(bl) : (l0 ? 63 - __clzll(l0) : -1);
        } else {
            const uint64_t bl = l0 & lane_range(0, t);
            prev = bl ? 63 - __clzll(bl) : -1;
        }
        if (prev >= 0) {
            const float zpr = S.u.m.sz[prev], dpr = S.u.m.sd[prev];
            const float rr = f_hypot(zpr, zp);
            cand = f_abs((dp - dpr) * (zp / rr) * (zpr / rr)) <= 2.f * tol;
        }
    }
    {
        const uint64_t cm = __ballot(cand);
        if (wave < 2 && lane == 0) S.cmask[wave] = cm;
    }
    __syncthreads();
    if (t == 0) {
        // The exact sequential scan over consecutive live pairs (last, p) in
        // ascending order changes something only at a pair that passes the
        // test.  A pair whose `last` no rotation has touched and that is not
        // a candidate fails it, so only candidates and the successor of each
        // rotated element are visited (as for n <= 64), each decided by the
        // exact test.  Element masks are two 64-bit words.
        uint64_t lv0 = S.live[0], lv1 = S.live[1];
        uint64_t cm0 = S.cmask[0], cm1 = S.cmask[1];
        auto lowest = [](uint64_t a0, uint64_t a1) {
            return a0 ? __builtin_ctzll(a0) : (a1 ? 64 + __builtin_ctzll(a1) : 128);
        };
        int nr = 0, mod = -1;  // mod: element changed by the latest rotation
        for (;;) {
            int succ = 128;
            if (mod >= 0) {  // first live element after mod
                const uint64_t a0 = (mod < 63) ? (lv0 & ~lane_range(0, mod + 1)) : 0ull;
                const uint64_t a1 = (mod < 63) ? lv1 : (lv1 & ~lane_range(0, mod - 63));
                succ = lowest(a0, a1);
            }
            const int p = min(succ, lowest(cm0, cm1));
            if (p >= n) break;
            if (p < 64) cm0 &= ~(1ull << p);
            else cm1 &= ~(1ull << (p - 64));
            // last live element before p
            int last = -1;
            if (p > 64) {
                const uint64_t b1 = lv1 & lane_range(0, p - 64);
                last = b1 ? 64 + 63 - __builtin_clzll(b1) : (lv0 ? 63 - __builtin_clzll(lv0) : -1);
            } else {
                const uint64_t b0 = lv0 & lane_range(0, p);
                last = b0 ? 63 - __builtin_clzll(b0) : -1;
            }
            if (last < 0) {
                mod = -1;
                continue;
            }
            const float zl = S.u.m.sz[last], zi = S.u.m.sz[p];
            const float dl = S.u.m.sd[last], di = S.u.m.sd[p];
            const float rr = f_hypot(zl, zi);
            const float c = zi / rr, sn = zl / rr;
            if (f_abs((di - dl) * c * sn) <= tol) {
                S.u.m.sd[last] = dl * c * c + di * sn * sn;
                S.u.m.sd[p] = dl * sn * sn + di * c * c;
                S.u.m.sz[last] = 0.f;
                S.u.m.sz[p] = rr;
                S.u.m.sdefl[last] = 1;
                S.u.m.rc[last] = c;
                S.u.m.rs[last] = sn;
                S.u.m.rpart[last] = p;
                S.u.m.rlist[nr++] = last;
                if (last < 64) lv0 &= ~(1ull << last);
                else lv1 &= ~(1ull << (last - 64));
                mod = p;
            } else {
                mod = -1;
            }
        }
        S.u.m.nrot[0] = nr;
        S.anyrot = nr > 0 ? 1 : 0;
    }
    __syncthreads();
    // compaction: non-deflated (poles, weights, child-order rows) first, then
    // the deflated items
    if (act) {
        dp = S.u.m.sd[t];
        zp = S.u.m.sz[t];
        defl = S.u.m.sdefl[t] != 0;
    }
    {
        const uint64_t lv = __ballot(act && !defl), dv = __ballot(act && defl);
        if (wave < 2 && lane == 0) {
            S.live[wave] = lv;
            S.dead[wave] = dv;
        }
        if (wave < 2) {
            const float zz = wave_total((act && !defl) ? zp * zp : 0.f);
            if (lane == 0) S.red[3][wave] = zz;
        }
    }
    __syncthreads();
    const uint64_t L0 = S.live[0], L1 = S.live[1], D0 = S.dead[0], D1 = S.dead[1];
    const int k = __popcll(L0) + __popcll(L1);
    if (act) {
        const int row = S.u.m.sperm[t];
        if (!defl) {
            const int idx = (t < 64) ? __popcll(L0 & lane_range(0, t))
                                     : __popcll(L0) + __popcll(L1 & lane_range(0, t - 64));
            S.u.m.dk[idx] = dp;
            S.u.m.zk[idx] = zp;
            S.u.m.ndrow[idx] = row;
        } else {
            const int idx = k + ((t < 64) ? __popcll(D0 & lane_range(0, t))
                                          : __popcll(D0) + __popcll(D1 & lane_range(0, t - 64)));
            S.u.m.itv[idx] = dp;
            S.u.m.itrow[idx] = row;
        }
    }
    __syncthreads();
    if (t == 0) {
        S.u.m.nk[0] = k;
        S.u.m.nrho[0] = rho;
        S.u.m.nzz[0] = S.red[3][0] + S.red[3][1];
        S.u.m.nfro[0] = f_sqrt(f_max(fro2, 0.f));
    }
    __syncthreads();

    // ---- secular roots, Loewner vectors, merge matrix (one node, depth 0) --
    roots_vectors<float, BN, BT, BN / (BT / BN)>(S, n, 0, t, S.lout, BN / 2);

    // ---- Q = Q_H (diag(Q1, Q2) M) with the sign rule ------------------------
    // Wave w takes row tile w of both products on 16x16x4 MFMA tiles, its A
    // rows (diag(Q1, Q2), then Q_H) loaded from HBM into registers, B from
    // LDS; E = diag(Q1, Q2) M replaces M.  Each wave then leaves, per column,
    // its entry of largest magnitude (lowest row on ties), a barrier later
    // the column's sign is known, and each wave stores its rows.
    if (Qb) {
        using MF = Mf<float>;
        constexpr int KS = BN / 4;  // k steps
        const int i16 = lane & 15, kk = lane >> 4;
        const int r = 16 * wave + i16;  // this lane's A row
        const bool rows = 16 * wave < n;
        f32x4 acc[BN / 16];
        float a[KS];
        if (rows) {
            // loads from clamped addresses (Q1[0] outside both blocks), the
            // zeros selected afterwards
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const int k = 4 * s4 + kk;
                const bool b1 = r < n1 && k < n1;
                const bool b2 = r >= n1 && r < n && k >= n1 && k < n;
                a[s4] = *(b1 ? Q1 + r * n1 + k : (b2 ? Q2 + (r - n1) * n2 + (k - n1) : Q1));
            }
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const int k = 4 * s4 + kk;
                const bool b1 = r < n1 && k < n1;
                const bool b2 = r >= n1 && r < n && k >= n1 && k < n;
                a[s4] = (b1 || b2) ? a[s4] : 0.f;
            }
#pragma unroll
            for (int ct = 0; ct < BN / 16; ++ct) acc[ct] = MF::zero();
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const float *mrow = S.M + (4 * s4 + kk) * LD + i16;
#pragma unroll
                for (int ct = 0; ct < BN / 16; ++ct) acc[ct] = MF::mma(a[s4], mrow[16 * ct], acc[ct]);
            }
        }
        __syncthreads();  // every read of M is done
        if (rows) {
#pragma unroll
            for (int ct = 0; ct < BN / 16; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    S.M[(16 * wave + MF::crow(lane, v)) * LD + 16 * ct + i16] = acc[ct][v];
            // Q_H rows of this tile (held in the Q output; only this wave
            // reads or writes them)
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const int k = 4 * s4 + kk;
                a[s4] = Qb[(r < n && k < n) ? r * n + k : 0];
            }
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const int k = 4 * s4 + kk;
                a[s4] = (r < n && k < n) ? a[s4] : 0.f;
            }
        }
        __syncthreads();  // E complete
        SignCand *cand = reinterpret_cast<SignCand *>(&S.u);  // [wave][column]
        float *csign = reinterpret_cast<float *>(cand + (BT / 64) * BN);
        static_assert(sizeof(S.u) >= sizeof(SignCand) * (BT / 64) * BN + sizeof(float) * BN,
                      "sign candidates");
        if (rows) {
#pragma unroll
            for (int ct = 0; ct < BN / 16; ++ct) acc[ct] = MF::zero();
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const float *erow = S.M + (4 * s4 + kk) * LD + i16;
#pragma unroll
                for (int ct = 0; ct < BN / 16; ++ct) acc[ct] = MF::mma(a[s4], erow[16 * ct], acc[ct]);
            }
#pragma unroll
            for (int ct = 0; ct < BN / 16; ++ct) {
                float best = -1.f, bval = 0.f;
                int brow = 1 << 20;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * wave + MF::crow(lane, v);
                    const float av = f_abs(acc[ct][v]);
                    const bool take = row < n && (av > best || (av == best && row < brow));
                    best = take ? av : best;
                    brow = take ? row : brow;
                    bval = take ? acc[ct][v] : bval;
                }
                {
                    const float ob = xmove<16>(best, lane);
                    const int orow = xmove<16>(brow, lane);
                    const float oval = xmove<16>(bval, lane);
                    const bool take = ob > best || (ob == best && orow < brow);
                    best = take ? ob : best;
                    brow = take ? orow : brow;
                    bval = take ? oval : bval;
                }
                {
                    const float ob = xmove<32>(best, lane);
                    const int orow = xmove<32>(brow, lane);
                    const float oval = xmove<32>(bval, lane);
                    const bool take = ob > best || (ob == best && orow < brow);
                    brow = take ? orow : brow;
                    bval = take ? oval : bval;
                }
                if (kk == 0) cand[wave * BN + 16 * ct + i16] = SignCand{bval, brow};
            }
        }
        __syncthreads();
        if (t < n) {
            float best = -1.f, bval = 0.f;
            int brow = 1 << 20;
            for (int w = 0; w < BT / 64 && 16 * w < n; ++w) {
                const SignCand cw = cand[w * BN + t];
                const float av = f_abs(cw.val);
                const bool take = cw.row < n && (av > best || (av == best && cw.row < brow));
                best = take ? av : best;
                brow = take ? cw.row : brow;
                bval = take ? cw.val : bval;
            }
            csign[t] = (bval < 0.f) ? -1.f : 1.f;
        }
        __syncthreads();
        if (rows) {
#pragma unroll
            for (int ct = 0; ct < BN / 16; ++ct) {
                const int c = 16 * ct + i16;
                const float sgn = (c < n) ? csign[c] : 1.f;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * wave + MF::crow(lane, v);
                    if (row < n && c < n) Qb[row * n + c] = sgn * acc[ct][v];
                }
            }
        }
    }
    const float unscale = fexp<float>::pow2(-md.shift);
    for (int e = t; e < n; e += BT) lam[bi * n + e] = unscale * S.lout[e];
    if (t == 0 && info) info[bi] = S.capped + ws.i1[bi] + ws.i2[bi];
}

// ------------------------------------------------------------------ host
// One workspace per stream, grown on demand.  A buffer that a captured graph
// uses is pinned: it is never freed, and a stream whose pinned buffer is too
// small for a later call gets a new one while the old one stays, retired,
// until the process ends.
struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool pinned = false;
};
std::mutex g_mu;
Lru<void *, Buf> g_bufs(8);
std::vector<void *> g_retired;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace big

bed_status big_solve(bed_dtype dt, int64_t batch, int n, const void *A, void *lam, void *Q,
                     int32_t *info, hipStream_t s)
{
    using namespace big;
    if (dt != BED_F32)
        return fail(BED_ERR_UNSUPPORTED, "n = %d > 64 is supported in binary32 only", n);
    if (n <= 64 || n > BN) return fail(BED_ERR_INVALID_ARG, "big_solve: n = %d", n);
    const int n1 = n / 2, n2 = n - n1;
    const size_t B = (size_t)batch;
    // children contiguous per kind: c1 then c2, q1 then q2, l1 then l2, i1 then i2
    const size_t c_bytes = align_up(B * 2 * (n1 + n2) * sizeof(float));
    const size_t q_bytes = align_up(B * (n1 * n1 + n2 * n2) * sizeof(float));
    const size_t l_bytes = align_up(B * n * sizeof(float));
    const size_t i_bytes = align_up(2 * B * sizeof(int32_t));
    const size_t m_bytes = align_up(B * sizeof(Meta));
    const size_t v_bytes = Q ? align_up(B * (n - 2) * n * sizeof(float)) : 0;
    const size_t t_bytes = Q ? align_up(B * n * sizeof(float)) : 0;
    const size_t need = c_bytes + q_bytes + l_bytes + i_bytes + m_bytes + v_bytes + t_bytes;
    const bool capturing = stream_capturing(s);
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Buf *b = g_bufs.find((void *)s);
        if (!b || b->bytes < need) {
            if (capturing)
                return fail(BED_ERR_CAPTURE, "workspace for n > 64 would be allocated during capture");
            if (b) {
                if (b->pinned) {
                    g_retired.push_back(b->ptr);  // a graph still reads and writes it
                } else {
                    hipError_t e = hipStreamSynchronize(s);
                    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
                    (void)hipFree(b->ptr);
                }
                b->ptr = nullptr;
                b->bytes = 0;
                b->pinned = false;
                hipError_t e = hipMalloc(&b->ptr, need);
                if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
                b->bytes = need;
            } else {
                Buf nb;
                hipError_t e = hipMalloc(&nb.ptr, need);
                if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
                nb.bytes = need;
                std::vector<Buf> old = g_bufs.insert((void *)s, nb);
                if (!old.empty()) {
                    (void)hipDeviceSynchronize();  // their last uses were on other streams
                    for (Buf &o : old) (void)hipFree(o.ptr);
                }
                b = g_bufs.find((void *)s);
            }
        }
        if (capturing) {
            g_bufs.pin((void *)s);
            b->pinned = true;
        }
        base = (char *)b->ptr;
    }
    Ws ws;
    ws.c1 = (float *)base;
    ws.c2 = ws.c1 + B * 2 * n1;
    ws.q1 = (float *)(base + c_bytes);
    ws.q2 = ws.q1 + B * n1 * n1;
    ws.l1 = (float *)(base + c_bytes + q_bytes);
    ws.l2 = ws.l1 + B * n1;
    ws.i1 = (int32_t *)(base + c_bytes + q_bytes + l_bytes);
    ws.i2 = ws.i1 + B;
    ws.meta = (Meta *)(base + c_bytes + q_bytes + l_bytes + i_bytes);
    ws.v = Q ? (float *)(base + c_bytes + q_bytes + l_bytes + i_bytes + m_bytes) : nullptr;
    ws.tau = Q ? (float *)(base + c_bytes + q_bytes + l_bytes + i_bytes + m_bytes + v_bytes)
               : nullptr;
    ws.e1 = Q ? nullptr : ws.q1;
    ws.e2 = Q ? nullptr : ws.q1 + B * 2 * n1;

    if (Q)
        hipLaunchKernelGGL(k_big_reduce<double>, dim3((unsigned)batch), dim3(BT), 0, s,
                           (const float *)A, n, (int64_t)batch, ws);
    else
        hipLaunchKernelGGL(k_big_reduce<float>, dim3((unsigned)batch), dim3(BT), 0, s,
                           (const float *)A, n, (int64_t)batch, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_big_reduce launch");
    if (Q) {
        hipLaunchKernelGGL(k_big_qh, dim3((unsigned)batch), dim3(BT), 0, s, n, (int64_t)batch,
                           (float *)Q, ws);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "k_big_qh launch");
    }
    const bed_tune dflt = default_tune();
    // the halves: eigenvectors, or (eigenvalues only) just the end rows z needs
    float *q1 = Q ? ws.q1 : nullptr, *q2 = Q ? ws.q2 : nullptr;
    if (n1 == n2) {
        e = launch_tri(class_shape(size_class(n1), dflt), ws.c1, n1, 2 * batch, ws.l1, q1,
                       ws.i1, ws.e1, s);
    } else {
        e = launch_tri(class_shape(size_class(n1), dflt), ws.c1, n1, batch, ws.l1, q1, ws.i1,
                       ws.e1, s);
        if (e == hipSuccess)
            e = launch_tri(class_shape(size_class(n2), dflt), ws.c2, n2, batch, ws.l2, q2,
                           ws.i2, ws.e2, s);
    }
    if (e != hipSuccess) return hip_fail(e, "child solve launch");
    hipLaunchKernelGGL(k_big_merge, dim3((unsigned)batch), dim3(BT), 0, s, n, (int64_t)batch,
                       (float *)lam, (float *)Q, info, ws);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_big_merge launch");
    return BED_OK;
}

}  // namespace bed
