// bed_syevd.hpp -- one team (a workgroup or a single wave) computes the full
// eigendecomposition of one symmetric n x n matrix (n <= NMAX <= 64) held in
// LDS/VGPRs:
//
//   load -> Householder tridiagonalization (binary64 arithmetic) -> rank-one
//   tearing (Sec. 2.1, Eq. (1)-(3)) -> leaves of at most 2, 4 or 8 elements by
//   cyclic Jacobi (Sec. 2.2) -> bottom-up merges (Sec. 2.3): z/sort (Eq.
//   (4)-(5)), deflation, secular roots by hybrid-section + Halley under bounded
//   interlacing (Eq. (8)-(21)), progressive removal of converged roots (Eq.
//   (22)), Loewner eigenvectors (Eq. (23)-(25)), back-multiplication (Eq. (4))
//   -> Householder back-transform -> sign canonicalization -> store.  Without
//   eigenvectors the merges carry only the end rows of each node's block.
//
// Team geometry (NT threads, thread t):
//   Householder: HW reducing waves, lane (r, g) holding row r of the columns
//     g + G j (G = HW 64 / NMAX groups); the other waves form Q_H.
//   Per-element phases: wave 0, lane e = element e (n <= 64 fits one wave).
//   Per-root phases: root q = t / LPR, LPR = NT / NMAX lanes share one root's
//     pole sums (aligned lane groups, butterfly reductions).
//   Back-transform: each wave owns NMAX/NW whole columns (no team barrier).
#pragma once

#include <type_traits>

#include "bed_device.hpp"
#include "bed_mfma.hpp"

// Phase markers: no-ops in the library; a profiling build may define
// BED_PHASE(id) to timestamp the phases of one team.
#ifndef BED_PHASE
#define BED_PHASE(id) ((void)0)
#endif
#ifndef BED_COUNT
#define BED_COUNT(id, value) ((void)0)
#endif
#ifndef BED_MARK
#define BED_MARK(depth, id) ((void)0)
#endif
#ifndef BED_ROOT
#define BED_ROOT(depth, root, evals, reason) ((void)0)
#endif
// Householder step markers (a profiling build may timestamp the sub-steps of
// one chosen step k; `wave` and `lane` are in scope where they are used).
#ifndef BED_HSTEP
#define BED_HSTEP(k, id) ((void)0)
#endif
// Deflation counts of one merge depth (type 1: rho |z_i| <= tol; type 2:
// Givens rotations), reported by lane 0 of wave 0 in a profiling build.
#ifndef BED_DEFL
#define BED_DEFL(type1, type2) ((void)0)
#endif

namespace bed {

// Waves that run the Householder reduction of a team: the row block of a
// wave (NMAX^2/(64 HW) registers per lane) must fit the register budget.
// n <= 32 reduces on one wave at every team size (a second one costs its
// cross-wave exchange in every step; larger teams still widen the merges).
#ifndef BED_HH_WAVES
#define BED_HH_WAVES(T, NMAX, NT) ((NMAX) == 64 ? ((NT) / 64 < 4 ? (NT) / 64 : 4) : 1)
#endif
template <typename T, int NMAX, int NT> struct HH_WAVES {
    static constexpr int value = BED_HH_WAVES(T, NMAX, NT);
};

// Waves that form Q_H = H_0 H_1 ... H_{n-3} explicitly while the others reduce
// (0: the back-transform applies the reflectors in compact-WY form instead).
// Each holds NMAX/AW >= 16 rows of Q_H, at most 32 values per lane.
template <typename T, int NMAX, int NT> struct QH_WAVES {
    static constexpr int spare = NT / 64 - HH_WAVES<T, NMAX, NT>::value;
    static constexpr int p = (spare >= 4 && NMAX >= 64) ? 4 : ((spare >= 2 && NMAX >= 32) ? 2 : (spare >= 1 ? 1 : 0));
    static constexpr int value = (p > 0 && NMAX * NMAX / (64 * p) <= 32) ? p : 0;
};
// With a single reducing wave there is no barrier per step; the team meets
// after every QH_SYNC steps so that the accumulating waves can follow.
constexpr int QH_SYNC = 4;

constexpr int SEC_CAP = 100;  // Halley-phase evaluations per root before "capped"

// Arithmetic type of the Householder reduction when eigenvectors are formed.
// Its rounding errors are a backward error of A, which the eigenvalue
// differences and the eigenvectors of close pairs amplify by 1/gap (the
// backward of the decomposition divides by those differences).  In binary64
// -- whose FMA issues at the rate of unpacked binary32 on gfx950 -- they stay
// far below binary32's unit roundoff; T, the reflectors and tau are then
// rounded once to the storage type.  (The LDS buffers of the reduction are
// sized for this type; a reduction in T uses them reinterpreted.)
template <typename T> struct HhArith {
    using type = double;
};

// Per-element state of the merges of one depth; arrays indexed by global
// position (node-local at [lo, hi)).
template <typename T, int NMAX>
struct MergeArrays {
    T sd[NMAX], sz[NMAX];     // sorted poles / weights (deflation in place)
    int sperm[NMAX], sdefl[NMAX];
    T dk[NMAX], zk[NMAX];     // non-deflated poles / weights at [lo, lo + k)
    int ndrow[NMAX];          // child-order row of non-deflated component
    int itrow[NMAX];          // child-order row of deflated item at [lo + k, hi)
    T itv[NMAX];              // item values: roots at [lo, lo+k), deflated after
    T rtau[NMAX], rdo[NMAX];  // root offset and its origin pole value
    T zh[NMAX];
    T rc[NMAX], rs[NMAX];
    int rpart[NMAX];
    int rlist[NMAX], nrot[NMAX];  // per node: deflated index of each rotation, in scan order
    int nlo[NMAX], nhi[NMAX];  // node of each element at this depth
    int ckl[NMAX], ckh[NMAX];  // child block of each row (its own block for an unmerged leaf)
    int tklo[NMAX / 16], tkhi[NMAX / 16];  // per 16-row tile: K range of the product
    int tnlo[NMAX / 16], tnhi[NMAX / 16];  // per 16-row tile: span of its nodes
    int nk[NMAX];
    T nrho[NMAX], nzz[NMAX], nfro[NMAX];
};

template <typename T, int NMAX, int NT>
struct Smem {
    static constexpr int LD = NMAX + 1;  // odd row stride: column walks hit distinct banks
    static constexpr int NW = NT / 64;
    static constexpr int G = NT / NMAX;
    T Q0[NMAX * LD];  // eigenvector blocks (ping)
    T Q1[NMAX * LD];  // eigenvector blocks (pong)
    T M[NMAX * LD];   // load staging, merge matrix, output staging
    // reflector k in row k: Vt[k*VLD + r] = v_k[r].  Compact WY: the odd row
    // stride keeps the MFMA operand reads (16 reflectors x 4 rows per
    // instruction) on distinct banks.  Explicit Q_H: 16-byte aligned rows for
    // vector reads; the buffer holds Q_H (row-major) once the reduction ends.
    static constexpr int VLD = QH_WAVES<T, NMAX, NT>::value ? NMAX + 4 : NMAX + 1;
    alignas(16) T Vt[NMAX * VLD];
    T a[NMAX], b[NMAX], tau[NMAX];
    T lam0[NMAX], lam1[NMAX];
    using H = typename HhArith<T>::type;
    static constexpr int HW = HH_WAVES<T, NMAX, NT>::value;
    union {
        struct {  // Householder (reducing waves only, in the reduction's type)
            H part[2 * HW * NMAX];
            H colb[2 * NMAX];
            alignas(16) H vbuf[HW * NMAX];
            alignas(16) H wbuf[HW * NMAX];
        } h;
        MergeArrays<T, NMAX> m;
        struct {  // back-transform: per block of 16 reflectors, Gram matrix and T factor
            // 16 x 16 tiles with row stride 17 (bank-conflict free column reads)
            T gram[((NMAX + 13) / 16) * 272];
            T tf[((NMAX + 13) / 16) * 272];
        } b;
    } u;
    int badw[NW];
    int expw[NW];  // per wave: largest exponent field of the lower triangle
    int capped;
    int anyrot;
};

// The solver runs on 2^s A with max |a_ij| in [1/2, 1) (s clamped, 0 for a
// zero matrix): the scaling is exact, and keeps the secular offsets of roots
// next to their poles out of the subnormal range, where the hardware
// reciprocal flushes.  Eigenvalues are scaled back on output; eigenvectors do
// not change.  s comes from the per-wave exponents the load leaves in LDS
// (formed where it is needed, so that it holds no registers in between).
template <typename T, int NMAX, int NT>
__device__ __forceinline__ int input_shift(const Smem<T, NMAX, NT>& S)
{
    int emax = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) emax = max(emax, S.expw[w]);
    emax = __builtin_amdgcn_readfirstlane(emax);
    const int sh = (emax == 0) ? 0 : fexp<T>::BIAS - 1 - emax;
    return min(max(sh, -fexp<T>::SMAX), fexp<T>::SMAX);
}

// Node of a dyadic tearing tree over [0, n): node j at depth d covers
// [floor(j n / 2^d), floor((j+1) n / 2^d)); nodes of more than `leaf`
// elements (the cutoff: 2, 4 or 8) split at the floor of their dyadic
// midpoint, the others are leaves.
struct Node {
    int lo, hi, s;
};
__device__ __forceinline__ Node node_of(int e, int d, int n)
{
    int j = (((e + 1) << d) - 1) / n;
    Node nd;
    nd.lo = (j * n) >> d;
    nd.hi = ((j + 1) * n) >> d;
    nd.s = ((2 * j + 1) * n) >> (d + 1);
    return nd;
}

__device__ __forceinline__ int node_index(int e, int d, int n) { return (((e + 1) << d) - 1) / n; }

// Jacobi rotation that annihilates a_pq of the symmetric 2x2 block
// [a_pp a_pq; a_pq a_qq] (Rutishauser's form): t = tan(phi) with
// th = (a_qq - a_pp) / (2 a_pq), t = sgn(th) / (|th| + sqrt(th^2 + 1)),
// c = 1/sqrt(1 + t^2), s = t c.  Then a_pp' = a_pp - t a_pq, a_qq' = a_qq + t a_pq.
// Written without the quotient th: with d = a_qq - a_pp (sgn 0 = +1),
// t = sgn(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), whose denominator is at
// least 2|a_pq|.  The reciprocal and 1/sqrt are refined to about one ulp, so
// that c^2 + s^2 = 1 and the rotation is orthogonal to the working precision.
template <typename T>
__device__ __forceinline__ void jacobi_rot(const T app, const T aqq, const T apq, T& c, T& s, T& t)
{
    const T d = aqq - app;
    const T ap2 = T(2) * apq;
    const T den = f_abs(d) + f_sqrt(fma(d, d, ap2 * ap2));
    // no rotation for a zero (or vanishing) a_pq: the block is already diagonal
    const bool rot = apq != T(0) && den > T(sizeof(T) == 4 ? 1e-30f : 1e-290);
    const T tt = (d < T(0) ? -ap2 : ap2) * f_rcp(rot ? den : T(1));
    const T cc = f_rsqrt(fma(tt, tt, T(1)));
    t = rot ? tt : T(0);
    c = rot ? cc : T(1);
    s = rot ? tt * cc : T(0);
}

// Value of lane ^ K inside aligned groups of 8 lanes, by DPP: a quad permute
// for K < 4; for K >= 4 the half-row mirror (lane ^ 7 within 8), followed by
// the quad permute of K ^ 7 when K < 7 -- lane i then reads lane (i ^ (K ^ 7))
// ^ 7 = i ^ K.
template <int K, typename T> __device__ __forceinline__ T lxor(T x)
{
    if constexpr (K < 4) return qxor<K>(x);
    else if constexpr (K == 7) return xmove<4>(x, 0);
    else return qxor<K ^ 7>(xmove<4>(x, 0));
}

// f(integral_constant<int, K>) for K = B, ..., E - 1 (compile-time indices).
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// One simultaneous round of the leaf Jacobi sweep: the pairs (i, i ^ M) of
// every leaf (GS lanes per leaf).  Lane i keeps row i of A and of V = J_1 J_2
// ... in XOR-relative order, a[k] = A(i, i ^ k), v[k] = V(i, i ^ k).  With J
// the product of the round's disjoint rotations, A <- J^T A J and V <- V J:
// each lane rotates its row's column pairs (j, j ^ M) with the parameters held
// by lane j, then combines its row with the partner row i ^ M.  The pair's own
// 2x2 block takes the exact form (a_pq' = 0, a_pp' = a_pp - t a_pq, a_qq' =
// a_qq + t a_pq).  The rounds M = 1, ..., GS - 1 of a sweep pair every two
// rows of the leaf exactly once (M = i ^ j).
template <int GS, int M, typename T>
__device__ __forceinline__ void jacobi_round(T (&a)[GS], T (&v)[GS], const int i, const int msz)
{
    const int ip = i ^ M;
    const T pd = lxor<M>(a[0]);  // A(ip, ip)
    const T po = lxor<M>(a[M]);  // A(ip, i)
    const bool low = i < ip;     // this row is p of the pair (p, q), p < q
    // both lanes of the pair form the same a_pq (the rounded rows need not be
    // exactly symmetric)
    const T apq = T(0.5) * (a[M] + po);
    T c, s, t;
    jacobi_rot(low ? a[0] : pd, low ? pd : a[0], apq, c, s, t);
    const bool rot = i < msz && ip < msz && apq != T(0);  // pairs with a padding row stay fixed
    c = rot ? c : T(1);
    s = rot ? s : T(0);
    t = rot ? t : T(0);
    const T sg = low ? T(-1) : T(1);  // A'(p, :) = c A(p, :) - s A(q, :), A'(q, :) = c A(q, :) + s A(p, :)
    const T ss = sg * s;
    // column parameters (c_j, sigma_j s_j) of column j = i ^ k
    T cj[GS], sj[GS];
    cj[0] = c;
    sj[0] = ss;
    cj[M] = c;
    sj[M] = -ss;
    static_for<1, GS>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (k != M) {
            cj[k] = lxor<k>(c);
            sj[k] = lxor<k>(ss);
        }
    });
    T b[GS], w[GS];
#pragma unroll
    for (int k = 0; k < GS; ++k) {
        b[k] = fma(sj[k], a[k ^ M], cj[k] * a[k]);
        w[k] = fma(sj[k], v[k ^ M], cj[k] * v[k]);
    }
    // partner row after its column rotation: B(ip, i ^ k) sits in its slot k ^ M
    T pb[GS];
#pragma unroll
    for (int k = 0; k < GS; ++k) pb[k] = lxor<M>(b[k ^ M]);
    const T dnew = fma(sg * t, apq, a[0]);
#pragma unroll
    for (int k = 0; k < GS; ++k) {
        a[k] = fma(ss, pb[k], c * b[k]);
        v[k] = w[k];
    }
    a[0] = rot ? dnew : a[0];
    a[M] = rot ? T(0) : a[M];
}

// Leaves of at most GS elements (the cutoff of the divide step, 2, 4 or 8) are
// solved by cyclic Jacobi -- the divide step may stop at small blocks and hand
// them to another eigensolver (Sec. 2.2).  Wave 0: lane (g, i) = (lane / GS,
// lane % GS) holds row i of the leaf of group g, group g standing for node g
// of depth D (the first such node of a leaf owns it; 2^D <= 64 / GS for n <=
// 64).  Sweeps of the rounds M = 1, ..., GS - 1 run until every off-diagonal
// entry is at most 8u ||T_leaf||_F (the wave's largest); the eigenvalues are
// then ranked ascending and the leaf's block of Q written.
template <int GS, typename T, int NMAX, int NT>
__device__ __forceinline__ void jacobi_leaves(Smem<T, NMAX, NT>& S, const int n, const int D,
                                              const int lane, T* __restrict__ Qc,
                                              T* __restrict__ Lc)
{
    static_assert((GS == 2 || GS == 4 || GS == 8) && NMAX <= 64, "leaf groups of 2, 4 or 8 lanes");
    constexpr int LD = Smem<T, NMAX, NT>::LD;
    constexpr int CAP = 16;  // sweeps (three to five suffice in binary32 and binary64 alike)
    const int g = lane / GS, i = lane % GS;
    const int e0 = (g * n) >> D;  // first element of node g at depth D
    int lo = 0, hi = 0;
    bool found = false;
    for (int d = 0; d <= D; ++d) {
        const Node nd = node_of(e0 < n ? e0 : 0, d, n);
        const bool hit = !found && nd.hi - nd.lo <= GS;
        lo = hit ? nd.lo : lo;
        hi = hit ? nd.hi : hi;
        found = found || hit;
    }
    const bool own = g < (1 << D) && found && lo == e0;
    const int msz = own ? hi - lo : 0;
    const bool row = i < msz;
    T a[GS], v[GS];
#pragma unroll
    for (int k = 0; k < GS; ++k) {
        const int j = i ^ k;
        const bool ok = row && j < msz;
        const bool adj = j == i + 1 || j == i - 1;
        const int bi = lo + (i < j ? i : j);
        T x = T(0);
        if (k == 0) x = S.a[ok ? lo + i : 0];
        else if (adj) x = S.b[ok ? bi : 0];
        a[k] = ok ? x : T(0);
        v[k] = (k == 0) ? T(1) : T(0);
    }
    T f2 = T(0);
#pragma unroll
    for (int k = 0; k < GS; ++k) f2 = fma(a[k], a[k], f2);
    f2 = group_sum<GS>(f2, lane);
    const T thr = T(8) * fp<T>::u * f_sqrt(f2);
    for (int sw = 0; sw < CAP; ++sw) {
        T off = T(0);
#pragma unroll
        for (int k = 1; k < GS; ++k) off = f_max(off, f_abs(a[k]));
        if (!__ballot(off > thr)) break;
        static_for<1, GS>([&](auto K) { jacobi_round<GS, decltype(K)::value>(a, v, i, msz); });
    }
    // ascending rank of this row's eigenvalue among the leaf's (ties by index)
    int rk = 0;
    static_for<1, GS>([&](auto K) {
        constexpr int k = decltype(K)::value;
        const T o = lxor<k>(a[0]);
        rk += ((i ^ k) < msz && (o < a[0] || (o == a[0] && (i ^ k) < i))) ? 1 : 0;
    });
    int rj[GS];
    rj[0] = rk;
    static_for<1, GS>([&](auto K) { rj[decltype(K)::value] = lxor<decltype(K)::value>(rk); });
    if (row) {
        Lc[lo + rk] = a[0];
        // V(i, j) is entry i of the eigenvector of eigenvalue j
#pragma unroll
        for (int k = 0; k < GS; ++k)
            if ((i ^ k) < msz) Qc[(lo + i) * LD + lo + rj[k]] = v[k];
    }
}

// Number of entries of the ascending list x[0..len) that are < v (strict) or
// <= v (inclusive).
template <typename T>
__device__ __forceinline__ int count_below(const T* x, int len, T v, bool inclusive)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        bool below = inclusive ? (x[mid] <= v) : (x[mid] < v);
        if (below) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The same count by binary lifting with power-of-two steps STEP, STEP/2, ..., 1
// (STEP a compile-time bound >= half of the longest list): a fixed chain of
// loads from clamped addresses and selects, with no branch.
template <int STEP, typename T>
__device__ __forceinline__ int count_lift(const T* x, int len, T v, bool inclusive, int base)
{
    const int probe = base + STEP;
    const int idx = (probe <= len ? probe : len) - 1;
    const T xv = x[idx > 0 ? idx : 0];
    const bool below = inclusive ? (xv <= v) : (xv < v);
    base = (probe <= len && below) ? probe : base;
    if constexpr (STEP > 1) return count_lift<STEP / 2>(x, len, v, inclusive, base);
    else return base;
}
template <int NMAX, typename T>
__device__ __forceinline__ int count_below_steps(const T* x, int len, T v, bool inclusive,
                                                 int step)
{
    // step is wave-uniform: one branch selects the unrolled chain
    if (step >= 32 && NMAX >= 64) return count_lift<32>(x, len, v, inclusive, 0);
    if (step >= 16 && NMAX >= 32) return count_lift<16>(x, len, v, inclusive, 0);
    if (step >= 8) return count_lift<8>(x, len, v, inclusive, 0);
    if (step >= 4) return count_lift<4>(x, len, v, inclusive, 0);
    if (step >= 2) return count_lift<2>(x, len, v, inclusive, 0);
    return count_lift<1>(x, len, v, inclusive, 0);
}

// Uniform index into a register array without dynamic VGPR indexing: a
// log-depth chain of selects (idx is wave-uniform in every caller).
template <int N, typename T>
__device__ __forceinline__ T pick(const T* a, int idx)
{
    if constexpr (N == 1) {
        return a[0];
    } else {
        const T lo = pick<N / 2>(a, idx);
        const T hi = pick<N / 2>(a + N / 2, idx);
        return (idx & (N / 2)) ? hi : lo;
    }
}

// M2 of one depth: secular roots (Sec. 2.3.1-2.3.4) with SL lanes per root and
// KPL poles per lane in registers.  Threads [0, NMAX SL) take part (whole
// waves); the per-root bracket and Halley logic runs on every lane of a root,
// so fewer lanes per root cost less issue time than they add in sums.
template <typename T, int NMAX, int NT, int SL, int KPL, typename SM>
__device__ __forceinline__ void secular_roots(SM& S, const int n, const int d, const int t,
                                              const int leaf)
{
    constexpr int LPR = SL;
    const int lane = t & 63;
    const T u = fp<T>::u;
    // absent poles: a far, finite pole with zero weight (its terms vanish and
    // its reciprocal stays a normal number)
    const T FAR = sizeof(T) == 4 ? T(1e30f) : T(1e300);
    const int q = t / LPR, sub = t % LPR;
    const Node qn = node_of(q < n ? q : 0, d, n);
    const bool qact = (q < n) && (qn.hi - qn.lo > leaf);
    const int qlo = qn.lo;
    const int kq = qact ? S.u.m.nk[qlo] : 0;
    const int jr = q - qlo;
    const T* dk = S.u.m.dk + qlo;
    const T* zk = S.u.m.zk + qlo;
    const T rho = qact ? S.u.m.nrho[qlo] : T(0);
    {
        const bool live = qact && jr < kq;
        // this lane's share of the poles: i = sub + LPR*j
        // df = pole - origin pole; the poles themselves are read again from
        // LDS if the origin moves
        T z2[KPL], df[KPL];
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const int i = sub + LPR * j;
            const bool ok = live && i < kq;
            const T dv = dk[ok ? i : 0], zv = zk[ok ? i : 0];
            df[j] = ok ? dv : FAR;
            z2[j] = ok ? zv * zv : T(0);
        }
        T ao = live ? rho * zk[jr] * zk[jr] : T(0);  // rho z_o^2 of the origin pole
        bool done = !live, capped = false;
        T L = T(0), U = T(0), h = T(0), w0 = T(1), gap = T(0), top = T(0);
        const T dj = live ? dk[jr] : T(0);
        const bool topr = live && jr == kq - 1;  // the unbounded-above root
        T dorg = dj;
        if (live) {
            if (!topr) {
                gap = dk[jr + 1] - dj;
                h = T(0.5) * gap;  // Eq. (13): midpoint of the root's own bracket
                w0 = gap;
            } else {
                // bracket (0, rho z^T z]; first probe at the Frobenius bound of
                // Eq. (10)-(11) when it is tighter, else at the midpoint
                top = rho * S.u.m.nzz[qlo];
                const T ubf = S.u.m.nfro[qlo] - dj;
                w0 = top;
                h = (ubf > T(0) && ubf < top) ? ubf : T(0.5) * top;
            }
        }
#pragma unroll
        for (int j = 0; j < KPL; ++j) df[j] = df[j] - dorg;
        int rounds = 0, nev = 0, why = 0, nhal = 0;
        // Eq. (8), (18), (21) at h: delta_i = (d_i - d_o) - h; returns f, f',
        // f'' and the stopping bound 8u(1 + rho sum |z_i^2 / delta_i|)
        auto secular = [&](const T hh, T& f, T& f1, T& f2, T& eb) {
            T s0 = 0, s1 = 0, s2 = 0, e = 0;
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const T rinv = f_rcp(df[j] - hh);
                const T t0 = z2[j] * rinv;
                const T t1 = t0 * rinv;
                s0 += t0;
                s1 += t1;
                s2 = fma(t1, rinv, s2);
                e += f_abs(t0);
            }
            s0 = group_sum<LPR>(s0, lane);
            s1 = group_sum<LPR>(s1, lane);
            s2 = group_sum<LPR>(s2, lane);
            e = group_sum<LPR>(e, lane);
            f = T(1) + rho * s0;
            f1 = rho * s1;
            f2 = T(2) * rho * s2;
            eb = T(8) * u * (T(1) + rho * e);
        };
        // Round 1, bisection (Eq. (14)-(15)): the sign of f at the midpoint
        // picks the nearer pole as origin of tau = lambda - d_origin; the top
        // root keeps d_k and takes the bracket side by the same sign.
        {
            T f, f1, f2, eb;
            secular(h, f, f1, f2, eb);
            rounds = 1;
            nev = live ? 1 : 0;
            const bool up = f > T(0);
            const bool shift = live && !topr && !up && f != T(0);
            if (__ballot(shift)) {
                const T dnew = shift ? dk[jr + 1] : dorg;
                const T znew = shift ? zk[jr + 1] : T(0);
                if (shift) {
                    ao = rho * znew * znew;
#pragma unroll
                    for (int j = 0; j < KPL; ++j) {
                        const int i = sub + LPR * j;
                        const bool ok = i < kq;  // shift implies live
                        df[j] = (ok ? dk[ok ? i : 0] : FAR) - dnew;
                    }
                    dorg = dnew;
                }
            }
            L = up ? T(0) : (topr ? h : h - gap);
            U = up ? h : (topr ? top : T(0));
            // The next point is Halley's from the midpoint (in the shifted
            // variable when the origin moved) when that step is short (within
            // a quarter of the bracket: the root lies near the midpoint), else
            // (Eq. (16)) one multi-section probe toward the origin pole while
            // the bracket is wide, else the one-pole model's point, else the
            // midpoint.
            const T hs = shift ? h - gap : h;  // the evaluated point, from the new origin
            const T den = T(2) * f1 * f1 - f * f2;
            const T hh = hs - T(2) * f * f1 * f_rcp_fast(den);
            const T hm = ao * hs * f_rcp_fast(fma(f, hs, ao));
            const bool okh = den > T(0) && hh > L && hh < U && f_abs(hh - hs) <= T(0.25) * (U - L);
            const bool okm = hm > L && hm < U;
            const bool probe = (U - L) > T(1e-2) * w0;
            const T hp = shift ? U - T(0.25) * (U - L) : L + T(0.25) * (U - L);
            const bool stop = live && f == T(0);
            why = stop ? 1 : 0;
            done = done || stop;
            h = stop ? h : (okh ? hh : (probe ? hp : (okm ? hm : T(0.5) * (L + U))));
            nhal = 0;
        }
        // Progressive removal (Eq. (22)): a converged root's lanes idle; the
        // wave leaves the loop once all of its roots have stopped.  The body
        // is select-based: every live root updates its bracket by the sign of
        // f (Eq. (14)); the next point is Halley's from the evaluated point
        // (the probe's included) if inside the bracket, else the root of the
        // one-pole model f ~ c - ao/tau through (h, f) (exact next to a light
        // origin pole), else the midpoint.  A root stops at
        // f = 0 or |f| <= eb, at a bracket with no interior float, when the
        // step does not move h, or at the cap.
        while (__ballot(!done)) {
            ++rounds;
            nev += done ? 0 : 1;
            T f, f1, f2, eb;
            secular(h, f, f1, f2, eb);
            const bool conv = f == T(0) || f_abs(f) <= eb;
            const bool up = f > T(0);
            const T U2 = up ? h : U;
            const T L2 = up ? L : h;
            const bool tight = (U2 - L2) <= T(2) * u * (f_abs(L2) + f_abs(U2));
            const T den = T(2) * f1 * f1 - f * f2;
            const T hh = h - T(2) * f * f1 * f_rcp_fast(den);
            const T hm = ao * h * f_rcp_fast(fma(f, h, ao));
            const bool okh = den > T(0) && hh > L2 && hh < U2;
            const bool okm = hm > L2 && hm < U2;
            const T mid = T(0.5) * (L2 + U2);
            const T hn = okh ? hh : (okm ? hm : mid);
            const bool step = !(conv || tight) && hn != h;
            // A root that meets the stopping bound still takes the Halley
            // step from its last evaluation when that step stays in the
            // bracket: the bound allows |f| up to 8u(1 + rho sum|z^2/delta|),
            // and the step (third order from there) brings the root to the
            // rounding level of f at no further evaluation.
            const bool fin = conv && okh;
            const int nh = nhal + 1;
            const bool cap = step && nh >= SEC_CAP;
            const bool act = !done;
            U = act ? U2 : U;
            L = act ? L2 : L;
            why = act ? (f == T(0) ? 1 : (conv ? 2 : (tight ? 3 : (!step ? 4 : (cap ? 5 : 0))))) : why;
            h = (act && (step || fin)) ? hn : h;
            nhal = act ? nh : nhal;
            capped = act ? cap : capped;
            done = done || !step || cap;
        }
        BED_COUNT(d, rounds);
        if (live && sub == 0) BED_ROOT(d, q, nev, why);
        if (live && sub == 0) {
            S.u.m.rdo[q] = dorg;
            S.u.m.rtau[q] = h;
            S.u.m.itv[q] = dorg + h;
            if (capped) atomicAdd(&S.capped, 1);
        }
    }
}

// Merge phases M2-M5 of one depth with KPL poles (or items) per lane held in
// registers: secular roots, Loewner zhat, eigenvector norms and output order,
// merge-matrix assembly (incl. type-2 rotations).  All team threads call it.
template <typename T, int NMAX, int NT, int KPL, typename SM>
__device__ __forceinline__ void roots_vectors(SM& S, const int n, const int d, const int t0,
                                              T* __restrict__ Ln, const int leaf)
{
    constexpr int LD = SM::LD;
    constexpr int LPR = NT / NMAX;
    // opaque copy of the thread index: the lane addresses derived from it are
    // formed again at every depth rather than hoisted out of the depth loop
    // (where they would be spilled)
    int t = t0;
    asm volatile("" : "+v"(t));
    const int lane = t & 63;
    (void)lane;
    const int q = t / LPR, sub = t % LPR;
    const Node qn = node_of(q < n ? q : 0, d, n);
    const bool qact = (q < n) && (qn.hi - qn.lo > leaf);
    const int qlo = qn.lo;
    const int mq = qn.hi - qn.lo;
    const int kq = qact ? S.u.m.nk[qlo] : 0;
    const int jr = q - qlo;
    const T* dk = S.u.m.dk + qlo;
    const T* zk = S.u.m.zk + qlo;
    const T rho = qact ? S.u.m.nrho[qlo] : T(0);

    // ---- M2: secular roots --------------------------------------------------
    {
        constexpr int SL = LPR < 4 ? LPR : 4;
        if (t < NMAX * SL) secular_roots<T, NMAX, NT, SL, KPL * LPR / SL>(S, n, d, t, leaf);
    }
    team_sync<NT>();
    BED_PHASE(10 + 8 * d + 1);

    // ---- M3: Loewner zhat (Eq. (25)) as a product of positive ratios ---------
    if (qact && jr < kq) {
        const T di = dk[jr];
        T p = T(1);
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const int jj = sub + LPR * j;
            const bool ok = jj < kq;
            const int js = ok ? jj : 0;
            const T del = (di - S.u.m.rdo[qlo + js]) - S.u.m.rtau[qlo + js];  // d_i - lam_j
            const T fac = -del * f_rcp((jj == jr) ? rho : (dk[js] - di));
            p *= ok ? fac : T(1);
        }
        p = group_prod<LPR>(p, lane);
        if (sub == 0) S.u.m.zh[q] = f_copysign(f_sqrt(p), zk[jr]);
    }
    team_sync<NT>();
    BED_PHASE(10 + 8 * d + 2);

    // ---- M4: output order, eigenvector norms (Eq. (24)) and the merge matrix
    // M = P G (U (+) I) with rows in child order, in one pass per root: the
    // lanes of root j form w_i = zhat_i / (d_i - lambda_j), reduce |w|^2, and
    // write -w_i / ||w|| into column rank(j).  Slots outside the node go to
    // the padding column NMAX of M, which no product reads (no branches).
    if (qact) {
        // rank of item jr among the node's m items (roots, then deflated)
        const T my = S.u.m.itv[q];
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const int vv = sub + LPR * j;
            const bool ok = vv < mq;
            const T ov = S.u.m.itv[qlo + (ok ? vv : 0)];
            cnt += (ok && (ov < my || (ov == my && vv < jr))) ? 1 : 0;
        }
        cnt = group_sum<LPR>(cnt, lane);
        const int c = qlo + cnt;
        if (sub == 0) Ln[c] = my;
        if (jr < kq) {
            const T dorg = S.u.m.rdo[q];
            const T tj = S.u.m.rtau[q];
            T wv[KPL];
            T s2 = T(0);
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const int ii = sub + LPR * j;
                const bool ok = ii < kq;
                const int is = ok ? ii : 0;
                const T w = S.u.m.zh[qlo + is] * f_rcp((dk[is] - dorg) - tj);
                wv[j] = w;
                s2 += ok ? w * w : T(0);
            }
            s2 = group_sum<LPR>(s2, lane);
            const T nr = f_rcp(f_sqrt(s2));
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const int ii = sub + LPR * j;
                const bool nd = ii < kq, df = !nd && ii < mq;
                const int is = (nd || df) ? ii : 0;
                const int rn = S.u.m.ndrow[qlo + is], rd = S.u.m.itrow[qlo + is];
                const int row = nd ? rn : (df ? rd : 0);  // row 0 for unused slots
                S.M[row * LD + ((nd || df) ? c : NMAX)] = nd ? -wv[j] * nr : T(0);
            }
        } else {
            const int myrow = S.u.m.itrow[q];
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const int row = qlo + sub + LPR * j;
                const bool in = row < qlo + mq;
                S.M[(in ? row : qlo) * LD + (in ? c : NMAX)] = (row == myrow) ? T(1) : T(0);
            }
        }
    }
    team_sync<NT>();
    BED_PHASE(10 + 8 * d + 3);
    if (S.anyrot) {
        // Type-2 rotations act on the rows of M in reverse scan order.
        if (qact && sub == 0) {
            const int c = qlo + jr;
            for (int i = S.u.m.nrot[qlo] - 1; i >= 0; --i) {
                const int p = S.u.m.rlist[qlo + i];
                const int part = S.u.m.rpart[p];
                const int rp = S.u.m.sperm[p], ri = S.u.m.sperm[part];
                const T cc = S.u.m.rc[p], ss = S.u.m.rs[p];
                const T mp = S.M[rp * LD + c], mi = S.M[ri * LD + c];
                S.M[rp * LD + c] = cc * mp + ss * mi;
                S.M[ri * LD + c] = -ss * mp + cc * mi;
            }
        }
        team_sync<NT>();
    }
}

// Calls roots_vectors with the smallest power-of-two KPL >= need.
template <typename T, int NMAX, int NT, int KPL, typename SM>
__device__ __forceinline__ void roots_vectors_dispatch(SM& S, const int n,
                                                       const int d, const int t, T* Ln, int need,
                                                       const int leaf)
{
    if constexpr (KPL >= NMAX / (NT / NMAX)) {
        roots_vectors<T, NMAX, NT, KPL>(S, n, d, t, Ln, leaf);
    } else {
        if (need <= KPL)
            roots_vectors<T, NMAX, NT, KPL>(S, n, d, t, Ln, leaf);
        else
            roots_vectors_dispatch<T, NMAX, NT, KPL * 2>(S, n, d, t, Ln, need, leaf);
    }
}

// One 16-row tile of the back-multiplication with a K loop of exactly KS
// steps of four (the caller picks KS >= the tile's K range).  Lane l supplies
// A[r0 + l%16][k] and B[k][c0 + l%16] for k = kb0 + 4 st + l/16; A entries
// outside the row's child block are zero and out-of-range rows of B are read
// at row 0 (finite) against a zero A entry.
template <typename T, int NMAX, int NT, int KS>
__device__ __forceinline__ void backmul_rowtile(Smem<T, NMAX, NT>& S, const T* __restrict__ Qc,
                                                T* __restrict__ Qn, const int n, const int lane,
                                                const int r0, const int cg, const int CG,
                                                const int kb0, const int nlo, const int nhi)
{
    using MF = Mf<T>;
    constexpr int LD = Smem<T, NMAX, NT>::LD;
    constexpr int RT = NMAX / 16;
    const int i16 = lane & 15;
    const int r = r0 + i16;
    const int ckl = S.u.m.ckl[r], ckh = S.u.m.ckh[r];
    T av[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) {
        const int k = kb0 + 4 * st + (lane >> 4);
        const bool ok = k >= ckl && k < ckh;
        const T a = Qc[r * LD + (ok ? k : 0)];
        av[st] = ok ? a : T(0);
    }
    for (int ct = cg; ct < RT; ct += CG) {
        const int c0 = 16 * ct;
        if (c0 >= n || c0 >= nhi || c0 + 16 <= nlo) continue;
        const int c = c0 + i16;
        T bv[KS];
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int k = kb0 + 4 * st + (lane >> 4);
            bv[st] = S.M[(k < NMAX ? k : 0) * LD + c];
        }
        typename MF::acc acc = MF::zero();
#pragma unroll
        for (int st = 0; st < KS; ++st) acc = MF::mma(av[st], bv[st], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) Qn[(r0 + MF::crow(lane, v)) * LD + c] = acc[v];
    }
}

// Householder tridiagonalization (Sec. 2; textbook, Golub-Van Loan 8.3) on HW
// waves of the team.  Lane (r, g) keeps row r of the columns c = g + G j,
// j < CPT, in registers, with G = HW * 64/NMAX column groups (64/NMAX groups
// per wave, each holding all rows): a cyclic split, so every group shrinks at
// the rate of the trailing matrix.  Within a wave p = A v is a per-lane dot
// product plus a butterfly over its groups; across waves one barrier per step
// exchanges the partial products together with the owner's pre-update pivot
// column k+1 (a look-ahead of one column), after which every wave forms w, the
// next pivot column and the next reflector on its own.  v and w reach a
// wave's groups through its own LDS copies (group-major: column c at
// (c % G) CPT + c / G), one 16-byte read per chunk of four columns.
//
// Steps whose dead columns (c <= k, where v_c = 0) fill a wave's first Q0
// chunks run in that wave's instance for Q0, whose chunk range is a
// compile-time constant.  Software pipeline: step k forms the updated pivot
// column and its norm first, then the reflector of step k+1 and its LDS
// broadcast, and issues its own rank-2 update last, so the scalar chain and
// the reductions overlap the update's FMAs.
template <typename T>
struct HhRefl {
    T alpha, tau, rv0;
};
template <typename T, typename H>
__device__ __forceinline__ HhRefl<H> hh_reflector(const H x0, const H sig)
{
    // alpha = -sgn(x0) mu, mu = ||x||; v = (1, x_2.. / (x0 - alpha)) with
    // x0 - alpha = sgn(x0)(|x0| + mu); tau = (mu + |x0|)/mu = 2/(v^T v) in
    // exact arithmetic.  Two independent reciprocals (1/mu, 1/(|x0| + mu)).
    // tau = 0 when the sub-column is already zero.
    // (binary64 arithmetic for binary32 storage: hardware estimates with one
    // Newton step, far more accurate than the binary32 result needs; binary64
    // storage: IEEE operations)
    constexpr bool est = sizeof(T) < sizeof(H);
    const bool z = (sig == H(0));
    const H s2 = fma(x0, x0, sig);
    const H rmu = est ? d_rsqrt_nr(s2) : f_rsqrt(s2);
    const H mu = s2 * rmu;
    const H ax = f_abs(x0);
    const H sg = (x0 < H(0)) ? H(-1) : H(1);
    HhRefl<H> h;
    h.alpha = z ? x0 : -sg * mu;
    h.rv0 = z ? H(1) : sg * (est ? d_rcp_nr(ax + mu) : f_rcp(ax + mu));
    h.tau = z ? H(0) : fma(ax, rmu, H(1));
    return h;
}

template <typename T, int NMAX, int NT, int HW, int Q0, typename H>
__device__ __forceinline__ void hh_range(Smem<T, NMAX, NT>& S, const int n, const int lane,
                                         const int wave, H (&ar)[NMAX * NMAX / (64 * HW)], H& xr,
                                         H& sig, H& vr, H& tauk)
{
    constexpr int GW = 64 / NMAX;   // column groups per wave
    constexpr int G = HW * GW;      // column groups of the team
    constexpr int CPT = NMAX / G;
    constexpr int NCH = CPT / 4;
    const int r = lane % NMAX, gl = lane / NMAX, g = wave * GW + gl;
    const int glast = wave * GW + GW - 1;  // last group of this wave
    const bool g0 = gl == 0;
    const int pos_r = (r % G) * CPT + r / G;
    H* vb = reinterpret_cast<H*>(S.u.h.vbuf) + wave * NMAX;
    H* wb = reinterpret_cast<H*>(S.u.h.wbuf) + wave * NMAX;
    H* colb = reinterpret_cast<H*>(S.u.h.colb);
    // instance Q0 = NCH: every column of this wave is dead, but the wave
    // keeps stepping (barriers, pivot column, next reflector) until n - 2
    const int kb = (Q0 == 0) ? 0 : glast + G * (4 * Q0 - 1);
    const int ke = (Q0 == NCH) ? n - 2 : min(glast + G * (4 * Q0 + 3), n - 2);
    // loop invariant: vr, tauk and this wave's LDS copy of v belong to step
    // k; ar holds the matrix after steps < k
    for (int k = kb; k < ke; ++k) {
        wave_sync();
        BED_HSTEP(k, 0);
        H vc[CPT];
#pragma unroll
        for (int j = 4 * Q0; j < CPT; ++j) vc[j] = vb[g * CPT + j];
        H pp0 = H(0), pp1 = H(0);
#pragma unroll
        for (int q = Q0; q < NCH; ++q) {
            pp0 = fma(ar[4 * q + 0], vc[4 * q + 0], pp0);
            pp1 = fma(ar[4 * q + 1], vc[4 * q + 1], pp1);
            pp0 = fma(ar[4 * q + 2], vc[4 * q + 2], pp0);
            pp1 = fma(ar[4 * q + 3], vc[4 * q + 3], pp1);
        }
        H pr = pp0 + pp1;
        if constexpr (GW >= 4) pr += xmove<16>(pr, lane);
        if constexpr (GW >= 2) pr += xmove<32>(pr, lane);
        BED_HSTEP(k, 1);
        // pivot column k + 1 before this step's update, from its owner group;
        // in this instance its register index lies in [4 Q0, 4 Q0 + 4)
        const int c1 = k + 1;
        const int g1 = c1 % G;
        H a1 = H(0);  // valid in group g1 (never this wave in instance NCH)
        if constexpr (Q0 < NCH) a1 = pick<4>(ar + 4 * Q0, (c1 / G) & 3);
        H cb;
        if constexpr (HW > 1) {
            H* pa = reinterpret_cast<H*>(S.u.h.part) + (k & 1) * HW * NMAX;
            if (g0) pa[wave * NMAX + r] = pr;
            if (g == g1) colb[(k & 1) * NMAX + r] = a1;
            team_sync<NT>();
            H q[HW];
#pragma unroll
            for (int w2 = 0; w2 < HW; ++w2) q[w2] = pa[w2 * NMAX + r];
#pragma unroll
            for (int st = 1; st < HW; st *= 2)  // pairwise (tree) sum
#pragma unroll
                for (int w2 = 0; w2 + st < HW; w2 += 2 * st) q[w2] += q[w2 + st];
            pr = q[0];
            cb = colb[(k & 1) * NMAX + r];
            BED_HSTEP(k, 2);
        } else {
            cb = a1;
            if constexpr (GW == 2) {
                const H o32 = xmove<32>(a1, lane);
                cb = (g == g1) ? a1 : o32;
            } else if constexpr (GW == 4) {
                const H o16 = xmove<16>(a1, lane);
                const H o32 = xmove<32>(a1, lane);
                const H o48 = xmove<32>(o16, lane);
                const int dd = g ^ g1;
                cb = dd == 0 ? a1 : (dd == 1 ? o16 : (dd == 2 ? o32 : o48));
            }
        }
        pr *= tauk;
        const H pv = wave_sum_all(g0 ? pr * vr : H(0));
        BED_HSTEP(k, 3);
        const H wr = pr - H(0.5) * tauk * pv * vr;
        if (g0) wb[pos_r] = wr;
        // v and w at column k + 1 are the values of row k + 1
        const H v1 = bcast(vr, k + 1), w1 = bcast(wr, k + 1);
        wave_sync();
        H wc[CPT];
#pragma unroll
        for (int j = 4 * Q0; j < CPT; ++j) wc[j] = wb[g * CPT + j];
        BED_HSTEP(k, 4);
        const H xn = fma(-wr, v1, fma(-vr, w1, cb));  // pivot column k + 1, row r
        const H sn = wave_sum_all((g0 && r > k + 2) ? xn * xn : H(0));
        BED_HSTEP(k, 5);
        // reflector of step k + 1 (harmless past the last step: nothing reads
        // reflector n - 2, and b[n - 2], a[n - 2] are rewritten afterwards)
        const HhRefl<H> h = hh_reflector<T>(bcast(xn, k + 2), sn);
        const H vn = (r == k + 2) ? H(1) : ((r > k + 2 && sn != H(0)) ? xn * h.rv0 : H(0));
        BED_HSTEP(k, 6);
        if (wave == 0 && lane == 0) {
            S.tau[k + 1] = T(h.tau);
            S.b[k + 1] = T(h.alpha);
        }
        if (g0) {
            if (wave == 0) {
                if (r == k + 1) S.a[k + 1] = T(xn);
                S.Vt[(k + 1) * Smem<T, NMAX, NT>::VLD + r] = T(vn);
            }
            vb[pos_r] = vn;
        }
        BED_HSTEP(k, 7);
        // rank-2 update of step k
#pragma unroll
        for (int j = 4 * Q0; j < CPT; ++j) ar[j] = fma(-wr, vc[j], fma(-vr, wc[j], ar[j]));
        BED_HSTEP(k, 8);
        xr = xn;
        sig = sn;
        vr = vn;
        tauk = h.tau;
        if constexpr (HW == 1 && QH_WAVES<T, NMAX, NT>::value > 0)
            if (k % QH_SYNC == QH_SYNC - 1) team_sync<NT>();
    }
    if constexpr (Q0 < NCH)
        hh_range<T, NMAX, NT, HW, Q0 + 1, H>(S, n, lane, wave, ar, xr, sig, vr, tauk);
}

// Explicit Q_H = H_0 H_1 ... H_{n-3} on the AW waves that do not reduce:
// Q_H <- Q_H (I - tau_k v_k v_k^T) = Q_H - tau_k (Q_H v_k) v_k^T for k = 0, 1,
// ..., once reflector k (row k of Vt, tau[k]) has passed a team barrier.
// Wave aw holds rows [aw RW, aw RW + RW) of Q_H; lane (rl, cg) holds row
// aw RW + rl, columns [cg VPL, cg VPL + VPL).
template <typename T, int NMAX, int NT>
struct QhShape {
    static constexpr int AW = QH_WAVES<T, NMAX, NT>::value;
    static constexpr int RW = AW ? NMAX / AW : NMAX;  // rows per wave
    static constexpr int VPL = AW ? NMAX * RW / 64 : 1;  // values per lane
};
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void qh_apply(const Smem<T, NMAX, NT>& S, const int lane, const int k,
                                         T (&qh)[QhShape<T, NMAX, NT>::VPL])
{
    constexpr int RW = QhShape<T, NMAX, NT>::RW;
    constexpr int VPL = QhShape<T, NMAX, NT>::VPL;
    constexpr int VLD = Smem<T, NMAX, NT>::VLD;
    constexpr int VW = 16 / sizeof(T);
    static_assert(RW >= 16 && VPL % VW == 0 && VLD % VW == 0, "explicit Q_H layout");
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    const int cg = lane / RW;
    const vec_t* vp = reinterpret_cast<const vec_t*>(S.Vt + k * VLD + cg * VPL);
    T v[VPL];
#pragma unroll
    for (int q = 0; q < VPL / VW; ++q) {
        const vec_t x = vp[q];
#pragma unroll
        for (int e = 0; e < VW; ++e) v[q * VW + e] = x[e];
    }
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int i = 0; i < VPL; i += 2) {
        s0 = fma(qh[i], v[i], s0);
        s1 = fma(qh[i + 1], v[i + 1], s1);
    }
    T s = s0 + s1;  // (Q_H v_k) at this row: sum over the column groups
    if constexpr (RW <= 16) s += xmove<16>(s, lane);
    if constexpr (RW <= 32) s += xmove<32>(s, lane);
    const T ts = S.tau[k] * s;
#pragma unroll
    for (int i = 0; i < VPL; ++i) qh[i] = fma(-ts, v[i], qh[i]);
}

// Barrier schedule of the reduction: one barrier at the start of every step
// with several reducing waves; with one, a barrier after every QH_SYNC-th step
// when Q_H is accumulated, else none.  Every wave of the team follows it.
template <int HW, int AW>
__device__ __forceinline__ bool hh_barrier_at(const int k)
{
    return HW > 1 || (AW > 0 && k % QH_SYNC == QH_SYNC - 1);
}

template <typename T, int NMAX, int NT, int HW, typename H>
__device__ __forceinline__ int householder(Smem<T, NMAX, NT>& S, const int n, const int lane,
                                           const int wave, const bool want_q, const T sc,
                                           T (&qh)[QhShape<T, NMAX, NT>::VPL])
{
    constexpr int LD = Smem<T, NMAX, NT>::LD;
    constexpr int GW = 64 / NMAX;
    constexpr int G = HW * GW;
    constexpr int CPT = NMAX / G;
    constexpr int AW = QH_WAVES<T, NMAX, NT>::value;
    static_assert(CPT % 4 == 0, "chunks of four columns");
    if (wave >= HW) {
        if constexpr (AW > 0) {
            if (wave < HW + AW) {
                // returns the first reflector not yet applied (the rest follow
                // the barrier that closes the reduction)
                constexpr int RW = QhShape<T, NMAX, NT>::RW;
                constexpr int VPL = QhShape<T, NMAX, NT>::VPL;
                const int row = (wave - HW) * RW + lane % RW, c0 = (lane / RW) * VPL;
#pragma unroll
                for (int i = 0; i < VPL; ++i) qh[i] = (row == c0 + i) ? T(1) : T(0);
                int j = 0;
                for (int k = 0; k < n - 2; ++k) {
                    if (!hh_barrier_at<HW, AW>(k)) continue;
                    team_sync<NT>();
                    // visible: reflectors up to k (barrier before step k) or up
                    // to k + 1 (barrier after step k)
                    const int jl = min(HW > 1 ? k : k + 1, n - 3);
                    for (; j <= jl; ++j)
                        if (want_q) qh_apply<T, NMAX, NT>(S, lane, j, qh);
                }
                return j;
            }
        }
        // waves outside the reduction only keep the barrier count
        for (int k = 0; k < n - 2; ++k)
            if (hh_barrier_at<HW, AW>(k)) team_sync<NT>();
        return 0;
    }
    // The reduction is one dependent chain; its waves issue ahead of the
    // accumulating waves that share their SIMDs.
    if constexpr (AW > 0) __builtin_amdgcn_s_setprio(1);
    const int r = lane % NMAX, gl = lane / NMAX, g = wave * GW + gl;
    const bool g0 = gl == 0;
    const H hs = H(sc);  // exact power of two
    H ar[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = g + G * j;
        ar[j] = (r < n && c < n) ? hs * H(c <= r ? S.M[r * LD + c] : S.M[c * LD + r]) : H(0);
    }
    H xr = (r < n) ? hs * H(S.M[r * LD]) : H(0);  // pivot column 0 (lower triangle)
    H sig = wave_total((g0 && r > 1) ? xr * xr : H(0));
    // reflector of step 0 (harmless when n <= 2, as above)
    const HhRefl<H> h = hh_reflector<T>(bcast(xr, 1), sig);
    H vr = (r == 1) ? H(1) : ((r > 1 && sig != H(0)) ? xr * h.rv0 : H(0));
    H tauk = h.tau;
    if (wave == 0 && lane == 0) {
        S.tau[0] = T(h.tau);
        S.b[0] = T(h.alpha);
    }
    if (g0) {
        if (wave == 0) {
            if (r == 0) S.a[0] = T(xr);
            S.Vt[r] = T(vr);
        }
        reinterpret_cast<H*>(S.u.h.vbuf)[wave * NMAX + (r % G) * CPT + r / G] = vr;
    }
    hh_range<T, NMAX, NT, HW, 0, H>(S, n, lane, wave, ar, xr, sig, vr, tauk);
    wave_sync();
    if (wave == 0 && g0 && n >= 2) {
        if (r == n - 2) S.a[n - 2] = T(xr);
        if (r == n - 1) S.b[n - 2] = T(xr);
    }
    if (g == (n - 1) % G && r == n - 1) S.a[n - 1] = T(pick<CPT>(ar, (n - 1) / G));
    if constexpr (AW > 0) __builtin_amdgcn_s_setprio(0);
    return 0;
}

// TRI: the input is already tridiagonal, given as its diagonal a (n values)
// followed by its off-diagonal b (n - 1 values) at Ain; there is no reduction
// and Q_H is the identity, so Q is Q_T (no back-transform).  ends_out (TRI,
// eigenvalues only): the first and last rows of Q_T, all that a merge above
// reads (Eq. (5)), as 2n values.
template <typename T, int NMAX, int NT, bool TRI = false>
__device__ __forceinline__ void syevd_team(const T* __restrict__ Ain, const int n,
                                           T* __restrict__ lam_out, T* __restrict__ Q_out,
                                           int* __restrict__ info_out, Smem<T, NMAX, NT>& S,
                                           const int t, const int leaf = 4,
                                           T* __restrict__ ends_out = nullptr)
{
    static_assert(NMAX <= 64 && (NMAX & (NMAX - 1)) == 0, "NMAX: power of two <= 64");
    static_assert(NT % 64 == 0 && NT >= NMAX && NT % NMAX == 0, "team geometry");
    constexpr int LD = Smem<T, NMAX, NT>::LD;
    constexpr int NW = NT / 64;
    constexpr int G = NT / NMAX;
    constexpr int CPT = NMAX / G;
    constexpr int LPR = NT / NMAX;
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int r = t % NMAX, g = t / NMAX;
    const T u = fp<T>::u;

    BED_PHASE(0);
    // ------------------------------------------------------------ load
    // 16-byte loads when the rows allow it (n a multiple of the vector width
    // and A 16-byte aligned), else one element per thread and step.  A
    // non-finite entry of the lower triangle is flagged per wave by a ballot,
    // and the largest magnitude's exponent is kept for the scaling below.
    {
        constexpr int VW = 16 / sizeof(T);
        bool bad = false;
        T amax = T(0);
        if constexpr (TRI) {
            for (int e = t; e < 2 * n - 1; e += NT) {
                const T v = Ain[e];
                bad = bad || !f_finite(v);
                amax = f_max(amax, f_abs(v));
                if (e < n) S.a[e] = v;
                else S.b[e - n] = v;
            }
        } else if (n % VW == 0 && (reinterpret_cast<uintptr_t>(Ain) & 15) == 0) {
            typedef T vec_t __attribute__((ext_vector_type(VW)));
            const vec_t* Av = reinterpret_cast<const vec_t*>(Ain);
            const int nv = n * n / VW;
            for (int e = t; e < nv; e += NT) {
                const vec_t v = Av[e];
                const int i = (e * VW) / n, j = (e * VW) % n;
#pragma unroll
                for (int q = 0; q < VW; ++q) {
                    if (j + q <= i && !f_finite(v[q])) bad = true;
                    amax = (j + q <= i) ? f_max(amax, f_abs(v[q])) : amax;
                    S.M[i * LD + j + q] = v[q];
                }
            }
        } else {
            for (int i = t / n, j = t % n, e = t; e < n * n; e += NT) {
                T v = Ain[e];
                if (j <= i && !f_finite(v)) bad = true;  // lower triangle only
                amax = (j <= i) ? f_max(amax, f_abs(v)) : amax;
                S.M[i * LD + j] = v;
                j += NT % n;
                i += NT / n;
                if (j >= n) {
                    j -= n;
                    ++i;
                }
            }
        }
        const bool wbad = __ballot(bad) != 0;
        const int wexp = group_max<64>(exp_field(amax), lane);
        if (lane == 0) {
            S.badw[wave] = wbad ? 1 : 0;
            S.expw[wave] = wexp;
        }
        if (t == 0) S.capped = 0;
    }
    team_sync<NT>();
    int anybad = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) anybad |= S.badw[w];
    if (anybad) {
        if (Q_out)
            for (int e = t; e < n * n; e += NT) Q_out[e] = f_nan<T>();
        for (int e = t; e < n; e += NT) lam_out[e] = f_nan<T>();
        if (t == 0 && info_out) *info_out = -1;
        return;
    }
    BED_PHASE(1);

    // ------------------------------------------------------------ Householder
    constexpr int HW = HH_WAVES<T, NMAX, NT>::value;
    constexpr int AW = QH_WAVES<T, NMAX, NT>::value;
    const bool qh_wave = AW > 0 && wave >= HW && wave < HW + AW && Q_out != nullptr;
    T qh[QhShape<T, NMAX, NT>::VPL];
    // binary64 arithmetic when eigenvectors are formed; for eigenvalues alone
    // the storage type (their error is the reduction's backward error, which
    // no eigenvalue gap amplifies)
    using H64 = typename HhArith<T>::type;
    int qj;
    if constexpr (TRI) {
        static_assert(QH_WAVES<T, NMAX, NT>::value > 0, "tridiagonal input: explicit Q_H shapes");
        // exact power-of-two scaling of the given diagonals (the same threads
        // wrote them); Q_H = I on the waves that would form it
        const T sc = fexp<T>::pow2(input_shift(S));
        for (int e = t; e < 2 * n - 1; e += NT) {
            if (e < n) S.a[e] *= sc;
            else S.b[e - n] *= sc;
        }
        if (qh_wave) {
            constexpr int RW = QhShape<T, NMAX, NT>::RW;
            constexpr int VPL = QhShape<T, NMAX, NT>::VPL;
            const int row = (wave - HW) * RW + lane % RW, c0 = (lane / RW) * VPL;
#pragma unroll
            for (int i = 0; i < VPL; ++i) qh[i] = (row == c0 + i) ? T(1) : T(0);
        }
        qj = n - 2;
    } else if constexpr (std::is_same<H64, T>::value)
        qj = householder<T, NMAX, NT, HW, T>(S, n, lane, wave, Q_out != nullptr,
                                             fexp<T>::pow2(input_shift(S)), qh);
    else if (Q_out)
        qj = householder<T, NMAX, NT, HW, H64>(S, n, lane, wave, true,
                                               fexp<T>::pow2(input_shift(S)), qh);
    else
        qj = householder<T, NMAX, NT, HW, T>(S, n, lane, wave, false,
                                             fexp<T>::pow2(input_shift(S)), qh);
    team_sync<NT>();
    if constexpr (AW > 0) {
        // reflectors written after the last barrier of the reduction
        if (qh_wave)
            for (; qj < n - 2; ++qj) qh_apply<T, NMAX, NT>(S, lane, qj, qh);
    }
    // The staging buffer becomes the merge matrix M: clear it so that entries
    // outside every node block (never written by a merge) are zero -- the MFMA
    // back-multiplication reads them against zero A entries.
    for (int e = t; e < NMAX * LD; e += NT) S.M[e] = T(0);
    team_sync<NT>();
    if constexpr (AW > 0 && !TRI) {
        // every reflector has been read: Q_H replaces them
        if (qh_wave) {
            constexpr int RW = QhShape<T, NMAX, NT>::RW;
            constexpr int VPL = QhShape<T, NMAX, NT>::VPL;
            constexpr int VLD = Smem<T, NMAX, NT>::VLD;
            constexpr int VW = 16 / sizeof(T);
            typedef T vec_t __attribute__((ext_vector_type(VW)));
            const int row = (wave - HW) * RW + lane % RW, c0 = (lane / RW) * VPL;
            vec_t* qp = reinterpret_cast<vec_t*>(S.Vt + row * VLD + c0);
#pragma unroll
            for (int q = 0; q < VPL / VW; ++q) {
                vec_t x;
#pragma unroll
                for (int e = 0; e < VW; ++e) x[e] = qh[q * VW + e];
                qp[q] = x;
            }
        }
    }
    BED_PHASE(2);

    // ------------------------------------------------------------ tear + leaves
    int D = 0;  // depth of the smallest leaves
    while (((n + (1 << D) - 1) >> D) > leaf) ++D;
    T* Qc = S.Q0;
    T* Qn = S.Q1;
    T* Lc = S.lam0;
    T* Ln = S.lam1;
    if (wave == 0) {
        const int e = lane;
        T ae = (e < n) ? S.a[e] : T(0);
        // Eq. (3): every split s of a node with more than `leaf` elements
        // subtracts |b_{s-1}| from a_{s-1} and a_s (branch-free: every depth's
        // coupling is read from a clamped address and applied by a select)
        for (int d = 0; d < D; ++d) {
            const Node nd = node_of(e < n ? e : 0, d, n);
            const bool split = nd.hi - nd.lo > leaf && (e == nd.s - 1 || e == nd.s);
            const T bs = S.b[nd.s >= 1 ? nd.s - 1 : 0];
            ae -= (e < n && split) ? f_abs(bs) : T(0);
        }
        if (e < n) S.a[e] = ae;  // torn diagonal
        wave_sync();
        if (leaf <= 2) jacobi_leaves<2>(S, n, D, lane, Qc, Lc);
        else if (leaf <= 4) jacobi_leaves<4>(S, n, D, lane, Qc, Lc);
        else jacobi_leaves<8>(S, n, D, lane, Qc, Lc);
    }
    team_sync<NT>();
    BED_PHASE(3);

    // ------------------------------------------------------------ merges
    for (int d = D - 1; d >= 0; --d) {
        // ---- M1: node structure (data-independent) on the last wave while
        // wave 0 forms z, sorts, deflates and compacts --------------------------
        if (wave == NW - 1) {
            const int e = lane;
            const Node nd = node_of(e < n ? e : 0, d, n);
            const bool act = (e < n) && (nd.hi - nd.lo > leaf);
            const int lo = act ? nd.lo : e, hi = act ? nd.hi : e, s = nd.s;
            {
                // Rows of a leaf that is not merged at this depth pass through
                // the back-multiplication unchanged: their child block is the
                // leaf itself and M is the identity on it.
                const bool leaf = (e < n) && !act;
                const int kl = act ? (e < s ? lo : s) : (leaf ? nd.lo : NMAX);
                const int kh = act ? (e < s ? s : hi) : (leaf ? nd.hi : 0);
                if (e < NMAX) {
                    S.u.m.nlo[e] = (e < n) ? nd.lo : e;
                    S.u.m.nhi[e] = (e < n) ? nd.hi : e;
                    S.u.m.ckl[e] = kl;
                    S.u.m.ckh[e] = kh;
                }
                if (leaf)
                    for (int cc = nd.lo; cc < nd.hi; ++cc) S.M[e * LD + cc] = (cc == e) ? T(1) : T(0);
                const int tkl = group_min<16>(kl, lane), tkh = group_max<16>(kh, lane);
                const int tnl = group_min<16>((e < n) ? nd.lo : NMAX, lane);
                const int tnh = group_max<16>((e < n) ? nd.hi : 0, lane);
                if ((e & 15) == 0 && e < NMAX) {
                    S.u.m.tklo[e >> 4] = tkl;
                    S.u.m.tkhi[e >> 4] = tkh;
                    S.u.m.tnlo[e >> 4] = tnl;
                    S.u.m.tnhi[e >> 4] = tnh;
                }
            }
        }
        if (wave == 0) {
            const int e = lane;
            const Node nd = node_of(e < n ? e : 0, d, n);
            BED_MARK(d, 8);
            const bool act = (e < n) && (nd.hi - nd.lo > leaf);
            const int lo = act ? nd.lo : e, hi = act ? nd.hi : e, s = nd.s;
            const T bet = act ? S.b[s - 1] : T(0);
            const T rho = f_abs(bet);
            const T sgm = (bet < T(0)) ? T(-1) : T(1);
            BED_MARK(d, 9);
            // largest power of two <= the largest child size at this depth
            const int cmax = (((n + (1 << d) - 1) >> d) + 1) >> 1;
            const int sstep = 1 << (31 - __builtin_clz(cmax > 0 ? cmax : 1));
            if (act) {
                const T de = Lc[e];
                const T ze = (e < s) ? sgm * Qc[(s - 1) * LD + e] : Qc[s * LD + e];
                // rank among the sibling's sorted values (one chain per lane:
                // left elements count right ones strictly below, right
                // elements count left ones below or equal -- a stable merge)
                const bool left = e < s;
                const int pos = (left ? e - lo : e - s) +
                                count_below_steps<NMAX>(Lc + (left ? s : lo), left ? hi - s : s - lo,
                                                        de, !left, sstep);
                S.u.m.sd[lo + pos] = de;
                S.u.m.sz[lo + pos] = ze;
                S.u.m.sperm[lo + pos] = e;
            }
            wave_sync();
            BED_MARK(d, 10);
            T dp = act ? S.u.m.sd[e] : T(0);
            T zp = act ? S.u.m.sz[e] : T(0);
            // node sums over [lo, hi) from wave prefix sums: z^T z, d^T (z o z),
            // d^T d; max |d| from the sorted end points
            const T pz = wave_prefix_sum(zp * zp);
            const T pdz = wave_prefix_sum(dp * zp * zp);
            const T pd2 = wave_prefix_sum(dp * dp);
            const int ilo = (lo > 0) ? lo - 1 : 0, ihi = (hi > lo) ? hi - 1 : e;
            const T zz0 = __shfl(pz, ihi) - (lo > 0 ? __shfl(pz, ilo) : T(0));
            const T dz = __shfl(pdz, ihi) - (lo > 0 ? __shfl(pdz, ilo) : T(0));
            const T d2 = __shfl(pd2, ihi) - (lo > 0 ? __shfl(pd2, ilo) : T(0));
            const T dmax = act ? f_max(f_abs(S.u.m.sd[lo]), f_abs(S.u.m.sd[hi - 1])) : T(0);
            BED_MARK(d, 11);
            const T tol = T(8) * u * f_max(dmax, rho * zz0);
            // Frobenius norm of the node (Eq. (10)), from D + rho z z^T
            const T fro2 = d2 + T(2) * rho * dz + rho * rho * zz0 * zz0;
            bool defl = act && (rho * f_abs(zp) <= tol);  // type 1
            const int n_type1 = __popcll(__ballot(defl));
            if (defl) zp = T(0);
            // type 2 candidates against the previous non-deflated component
            const uint64_t live = __ballot(act && !defl);
            const uint64_t below = live & lane_range(lo, e);
            const int prev = below ? 63 - __clzll(below) : e;
            const T zpr = __shfl(zp, prev), dpr = __shfl(dp, prev);
            bool cand = false;
            if (act && !defl && prev != e) {
                // |z| >= tol/rho here (no under/overflow in the squares).  This
                // test rounds differently from the exact one of the scan below
                // (reciprocal square root against hypot and division), so it
                // allows a factor 2: every pair that passes the exact test is
                // a candidate, and the scan decides each candidate exactly.
                const T ir = f_rcp(f_sqrt(fma(zpr, zpr, zp * zp)));
                cand = f_abs((dp - dpr) * (zp * ir) * (zpr * ir)) <= T(2) * tol;
            }
            const uint64_t cmask = __ballot(cand);
            BED_MARK(d, 12);
            if (act) {
                S.u.m.rpart[e] = -1;
                S.u.m.sdefl[e] = defl ? 1 : 0;
                S.u.m.sz[e] = zp;
            }
            bool hasrot = false;
            int my_nrot = 0;
            if (cmask) {
                // Rare path: the exact sequential Givens scan for nodes that
                // have a type-2 candidate (one lane per such node).
                wave_sync();
                const bool mine = act && e == lo && (cmask & lane_range(lo, hi));
                if (mine) {
                    // The scan over consecutive live pairs (last, p) changes
                    // something only at a pair that passes the test.  A pair
                    // whose `last` no rotation has touched and that is not a
                    // candidate fails it (the candidate test is looser), so
                    // only candidates and the successor of each rotated
                    // element are visited, in ascending order, each decided
                    // by the exact test: the decisions of the full scan.
                    uint64_t lv = live & lane_range(lo, hi);
                    uint64_t cm = cmask & lane_range(lo, hi);
                    int mod = -1;  // element changed by the latest rotation
                    for (;;) {
                        const uint64_t after = (mod >= 0) ? (lv & ~lane_range(0, mod + 1)) : 0;
                        const int succ = after ? __builtin_ctzll(after) : 64;
                        const int cnd = cm ? __builtin_ctzll(cm) : 64;
                        const int p = succ < cnd ? succ : cnd;
                        if (p >= hi) break;
                        cm &= ~(1ull << p);
                        const uint64_t bl = lv & lane_range(lo, p);
                        if (!bl) {
                            mod = -1;
                            continue;
                        }
                        const int last = 63 - __clzll(bl);
                        const T zl = S.u.m.sz[last], zi = S.u.m.sz[p];
                        const T dl = S.u.m.sd[last], di = S.u.m.sd[p];
                        const T rr = f_hypot(zl, zi);
                        const T c = zi / rr, sn = zl / rr;
                        if (f_abs((di - dl) * c * sn) <= tol) {
                            S.u.m.sd[last] = dl * c * c + di * sn * sn;
                            S.u.m.sd[p] = dl * sn * sn + di * c * c;
                            S.u.m.sz[last] = T(0);
                            S.u.m.sz[p] = rr;
                            S.u.m.sdefl[last] = 1;
                            S.u.m.rc[last] = c;
                            S.u.m.rs[last] = sn;
                            S.u.m.rpart[last] = p;
                            S.u.m.rlist[lo + my_nrot++] = last;
                            lv &= ~(1ull << last);
                            mod = p;
                        } else {
                            mod = -1;
                        }
                    }
                }
                wave_sync();
                if (act) {
                    dp = S.u.m.sd[e];
                    zp = S.u.m.sz[e];
                    defl = S.u.m.sdefl[e] != 0;
                }
                hasrot = (cmask & lane_range(lo, hi)) != 0;
            }
            const uint64_t live2 = __ballot(act && !defl);
            BED_MARK(d, 13);
            const uint64_t dead = __ballot(act && defl);
            const int k = __popcll(live2 & lane_range(lo, hi));
            if (act) {
                const int row = S.u.m.sperm[e];
                if (!defl) {
                    const int idx = __popcll(live2 & lane_range(lo, e));
                    S.u.m.dk[lo + idx] = dp;
                    S.u.m.zk[lo + idx] = zp;
                    S.u.m.ndrow[lo + idx] = row;
                } else {
                    const int idx = k + __popcll(dead & lane_range(lo, e));
                    S.u.m.itv[lo + idx] = dp;
                    S.u.m.itrow[lo + idx] = row;
                }
            }
            const T pzz = wave_prefix_sum((act && !defl) ? zp * zp : T(0));
            BED_MARK(d, 14);
            const T zz = __shfl(pzz, ihi) - (lo > 0 ? __shfl(pzz, ilo) : T(0));
            if (act && e == lo) {
                S.u.m.nk[lo] = k;
                S.u.m.nrho[lo] = rho;
                S.u.m.nzz[lo] = zz;
                S.u.m.nfro[lo] = f_sqrt(f_max(fro2, T(0)));
                S.u.m.nrot[lo] = my_nrot;
            }
            const bool anyrot = __ballot(hasrot) != 0;
            if (e == 0) S.anyrot = anyrot ? 1 : 0;
            BED_DEFL(n_type1, (int)wave_total(float(act && e == lo ? my_nrot : 0)));
            (void)n_type1;
            BED_MARK(d, 15);
        }
        team_sync<NT>();
        BED_PHASE(10 + 8 * d + 0);

        {
            // poles (and items) per lane at this depth: ceil(max node size / LPR)
            const int need = ((((n + (1 << d) - 1) >> d)) + LPR - 1) / LPR;
            roots_vectors_dispatch<T, NMAX, NT, 1>(S, n, d, t, Ln, need, leaf);
        }
        BED_PHASE(10 + 8 * d + 4);

        // ---- M6: back-multiplication Q_next = blockdiag(Q1, Q2) M (Eq. (4)) --
        // 16x16 MFMA tiles.  A = Q_cur restricted to each row's child block,
        // B = M (zero outside the node blocks, the identity on unmerged
        // leaves), so every computed entry is final: the product of a row and
        // a column of different nodes is exactly zero, and such entries are
        // never read.  A wave loads the A operand of its row tile once and
        // reuses it for every column tile that meets the tile's nodes.  The
        // K loop has a fixed length (4, 8 or 16 steps, chosen once per row
        // tile) and operands come from clamped addresses, so the tile has no
        // per-step branches.
        if (!Q_out) {
            // Eigenvalues only: the next depth's z (Eq. (5)) reads the last
            // row of each left child and the first row of each right child,
            // i.e. the end rows of this depth's nodes -- and an end row of a
            // node is the matching end row of one child times M.  So only the
            // two end rows of every node are formed (2 m^2 flops per node
            // instead of the block product), wave w taking rows w, w + NW, ...
            // with one lane per column; unmerged leaves pass theirs through M
            // = I.  The other rows of the buffers are never read again.
            for (int r = wave; r < n; r += NW) {
                const int nlo = S.u.m.nlo[r], nhi = S.u.m.nhi[r];
                if (r != nlo && r != nhi - 1) continue;
                const int c = lane;
                if (c < nlo || c >= nhi) continue;
                const int kl = S.u.m.ckl[r], kh = S.u.m.ckh[r];
                T acc = T(0);
                for (int k = kl; k < kh; ++k) acc = fma(Qc[r * LD + k], S.M[k * LD + c], acc);
                Qn[r * LD + c] = acc;
            }
            for (int e = t; e < n; e += NT) {
                if (S.u.m.nhi[e] - S.u.m.nlo[e] <= leaf) Ln[e] = Lc[e];
            }
        } else {
            constexpr int RT = NMAX / 16;
            constexpr int CG = (NW >= RT) ? NW / RT : 1;    // column groups per row tile
            BED_MARK(d, 0);
            for (int idx = wave; idx < RT * CG; idx += NW) {
                const int rt = idx % RT, cg = idx / RT;
                const int r0 = 16 * rt;
                if (r0 >= n) continue;
                const int klo = S.u.m.tklo[rt], khi = S.u.m.tkhi[rt];
                const int nlo = S.u.m.tnlo[rt], nhi = S.u.m.tnhi[rt];
                BED_MARK(d, 4);
                if (klo >= khi) continue;
                const int kb0 = klo & ~3;
                const int nks = __builtin_amdgcn_readfirstlane((khi - kb0 + 3) >> 2);
                BED_MARK(d, 5);
                if (nks <= 4)
                    backmul_rowtile<T, NMAX, NT, 4>(S, Qc, Qn, n, lane, r0, cg, CG, kb0, nlo, nhi);
                else if (nks <= 8)
                    backmul_rowtile<T, NMAX, NT, 8>(S, Qc, Qn, n, lane, r0, cg, CG, kb0, nlo, nhi);
                else
                    backmul_rowtile<T, NMAX, NT, NMAX / 4>(S, Qc, Qn, n, lane, r0, cg, CG, kb0, nlo,
                                                           nhi);
            }
            BED_MARK(d, 2);
            // eigenvalues of nodes not merged at this depth
            for (int e = t; e < n; e += NT) {
                if (S.u.m.nhi[e] - S.u.m.nlo[e] <= leaf) Ln[e] = Lc[e];
            }
            BED_MARK(d, 3);
        }
        team_sync<NT>();
        BED_PHASE(10 + 8 * d + 5);
        T* tq = Qc; Qc = Qn; Qn = tq;
        T* tl = Lc; Lc = Ln; Ln = tl;
    }

    if (!Q_out) {  // eigenvalues only
        for (int e = t; e < n; e += NT) lam_out[e] = fexp<T>::pow2(-input_shift(S)) * Lc[e];
        if (t == 0 && info_out) *info_out = S.capped;
        if constexpr (TRI) {
            // the root's end rows, carried through every depth
            if (ends_out)
                for (int e = t; e < 2 * n; e += NT)
                    ends_out[e] = (e < n) ? Qc[e] : Qc[(n - 1) * LD + e - n];
        }
        return;
    }

    // ------------------------------------------------------------ back-transform
    // (TRI: Q_H = I, the compact-WY branch with no reflectors stores Q_T)
    if constexpr (AW > 0 && !TRI) {
        // Q_A = Q_H Q_T on 16x16x4 MFMA tiles: wave w computes row tiles
        // [p RPW, p RPW + RPW) of column tile w % CT (p = w / CT).  Lane group kk
        // covers k in [kk KS, kk KS + KS), so each lane reads a contiguous
        // slice of its Q_H row.  The product goes to Qn unsigned; each wave
        // leaves, per column, its entry of largest magnitude (lowest row on
        // ties) for the sign rule applied by the store.
        using MF = Mf<T>;
        constexpr int CT = NMAX / 16;
        constexpr int RT = NMAX / 16;
        static_assert(NW >= CT, "one wave per column tile at least");
        constexpr int WPC = (NW / CT > RT) ? RT : NW / CT;  // waves per column tile
        constexpr int RPW = RT / WPC;
        constexpr int KS = NMAX / 4;
        constexpr int VLD = Smem<T, NMAX, NT>::VLD;
        constexpr int VW = 16 / sizeof(T);
        static_assert(WPC * NMAX <= int(sizeof(S.u.b.gram) / sizeof(T)), "sign candidates");
        typedef T vec_t __attribute__((ext_vector_type(VW)));
        const int i16 = lane & 15, kk = lane >> 4;
        if (wave < CT * WPC) {
            const int ct = wave % CT, part = wave / CT;
            const int c = 16 * ct + i16;
            T bq[KS];
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const int k = kk * KS + s4;
                bq[s4] = (k < n) ? Qc[k * LD + c] : T(0);
            }
            typename MF::acc q[RPW];
#pragma unroll
            for (int pr = 0; pr < RPW; ++pr) {
                const int rt = part * RPW + pr;
                const vec_t* ap = reinterpret_cast<const vec_t*>(S.Vt + (16 * rt + i16) * VLD + kk * KS);
                T a[KS];
#pragma unroll
                for (int q4 = 0; q4 < KS / VW; ++q4) {
                    const vec_t x = ap[q4];
#pragma unroll
                    for (int e = 0; e < VW; ++e) a[q4 * VW + e] = x[e];
                }
                q[pr] = MF::zero();
#pragma unroll
                for (int s4 = 0; s4 < KS; ++s4) q[pr] = MF::mma(a[s4], bq[s4], q[pr]);
            }
            T best = T(-1), bval = T(0);
            int brow = 1 << 20;
#pragma unroll
            for (int pr = 0; pr < RPW; ++pr) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * (part * RPW + pr) + MF::crow(lane, v);
                    const T av = f_abs(q[pr][v]);
                    const bool take = row < n && (av > best || (av == best && row < brow));
                    best = take ? av : best;
                    brow = take ? row : brow;
                    bval = take ? q[pr][v] : bval;
                    if (row < n && c < n) Qn[row * LD + c] = q[pr][v];
                }
            }
            {
                const T ob = xmove<16>(best, lane);
                const int orow = xmove<16>(brow, lane);
                const T oval = xmove<16>(bval, lane);
                const bool take = ob > best || (ob == best && orow < brow);
                best = take ? ob : best;
                brow = take ? orow : brow;
                bval = take ? oval : bval;
            }
            {
                const T ob = xmove<32>(best, lane);
                const int orow = xmove<32>(brow, lane);
                const T oval = xmove<32>(bval, lane);
                const bool take = ob > best || (ob == best && orow < brow);
                bval = take ? oval : bval;
            }
            if (kk == 0) S.u.b.gram[part * NMAX + c] = bval;
        }
        team_sync<NT>();
        BED_PHASE(4);
        // Sign of column j: parts in increasing row order, a later part wins
        // only when strictly larger in magnitude.  16-byte stores when the
        // rows allow them, as for the load.
        auto colsign = [&](const int j) {
            T bv = S.u.b.gram[j];
#pragma unroll
            for (int pp = 1; pp < WPC; ++pp) {
                const T o = S.u.b.gram[pp * NMAX + j];
                bv = (f_abs(o) > f_abs(bv)) ? o : bv;
            }
            return bv;
        };
        if (n % VW == 0 && (reinterpret_cast<uintptr_t>(Q_out) & 15) == 0) {
            vec_t* Qv = reinterpret_cast<vec_t*>(Q_out);
            const int nv = n * n / VW;
            for (int e = t; e < nv; e += NT) {
                const int i = (e * VW) / n, j = (e * VW) % n;
                vec_t x;
#pragma unroll
                for (int q4 = 0; q4 < VW; ++q4) {
                    const T y = Qn[i * LD + j + q4];
                    x[q4] = (colsign(j + q4) < T(0)) ? -y : y;
                }
                Qv[e] = x;
            }
        } else {
            for (int i = t / n, j = t % n, e = t; e < n * n; e += NT) {
                const T x = Qn[i * LD + j];
                Q_out[e] = (colsign(j) < T(0)) ? -x : x;
                j += NT % n;
                i += NT / n;
                if (j >= n) {
                    j -= n;
                    ++i;
                }
            }
        }
        for (int e = t; e < n; e += NT) lam_out[e] = fexp<T>::pow2(-input_shift(S)) * Lc[e];
        if (t == 0 && info_out) *info_out = S.capped;
        BED_PHASE(5);
        return;
    } else {
    // Q_A = H_0 H_1 ... H_{n-3} Q_T in compact-WY blocks of 16 reflectors,
    // H_{16b} ... H_{16b+15} = I - V_b T_b V_b^T (T_b upper triangular), applied
    // for b = last .. 0.  Each wave keeps whole 16-column tiles of Q in MFMA
    // accumulators for all blocks, so the update needs no team barrier.
    {
        using MF = Mf<T>;
        constexpr int RT = NMAX / 16;
        constexpr int VLD = Smem<T, NMAX, NT>::VLD;
        const int nb = (!TRI && n > 2) ? n - 2 : 0;  // reflectors
        const int NB = (nb + 15) / 16;
        const int i16 = lane & 15;
        BED_MARK(7, 0);
        // Gram matrices G_b = V_b^T V_b (one wave per block); one MFMA chain
        // per row tile, summed at the end (independent chains overlap)
        for (int bk = wave; bk < NB; bk += NW) {
            const int k0 = 16 * bk;
            const bool okr = k0 + i16 < nb;
            typename MF::acc g = MF::zero();
            typename MF::acc gt[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                gt[rt] = MF::zero();
                if (rt < bk) continue;  // rows above the block's first reflector are zero
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    const int row = 16 * rt + MF::crow(lane, s4);
                    const T vv = okr ? S.Vt[(k0 + i16) * VLD + row] : T(0);
                    gt[rt] = MF::mma(vv, vv, gt[rt]);
                }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                if (rt >= bk) g += gt[rt];
#pragma unroll
            for (int v = 0; v < 4; ++v) S.u.b.gram[bk * 272 + MF::crow(lane, v) * 17 + i16] = g[v];
            wave_sync();
            // T_b: T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j)
            BED_MARK(7, 1);
            if (lane < 16) {
                T trow[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const T tj = (k0 + j < nb) ? S.tau[k0 + j] : T(0);
                    T acc = T(0);
#pragma unroll
                    for (int kk = 0; kk < j; ++kk) acc = fma(trow[kk], S.u.b.gram[bk * 272 + kk * 17 + j], acc);
                    trow[j] = (lane < j) ? -tj * acc : (lane == j ? tj : T(0));
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) S.u.b.tf[bk * 272 + lane * 17 + j] = trow[j];
            }
        }
        BED_MARK(7, 2);
        team_sync<NT>();
        constexpr int NBMAX = (NMAX + 13) / 16;  // blocks for n = NMAX
        for (int ct = wave; ct < RT; ct += NW) {
            const int c0 = 16 * ct;
            if (c0 >= n) continue;
            BED_MARK(7, 3);
            const int c = c0 + i16;
            typename MF::acc q[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rt + MF::crow(lane, v);
                    q[rt][v] = (row < n && c < n) ? Qc[row * LD + c] : T(0);
                }
            }
            // blocks last to first, unrolled so that the zero row tiles of
            // each V_b (below its first reflector) are skipped at compile time
#pragma unroll
            for (int bi = 0; bi < NBMAX; ++bi) {
                const int bk = NBMAX - 1 - bi;
                if (bk >= NB) continue;
                const int k0 = 16 * bk;
                const bool okr = k0 + i16 < nb;
                // operands of this block, loaded before the MFMA chains
                T va[RT][4], vb[RT][4], tv[4];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int row = 16 * rt + MF::crow(lane, s4);
                        const int kr = k0 + MF::crow(lane, s4);
                        va[rt][s4] = okr ? S.Vt[(k0 + i16) * VLD + row] : T(0);
                        vb[rt][s4] = (kr < nb) ? -S.Vt[kr * VLD + 16 * rt + i16] : T(0);
                    }
                }
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) tv[s4] = S.u.b.tf[bk * 272 + i16 * 17 + MF::crow(lane, s4)];
                // X = V_b^T Q (16 x 16 tile of this column block): one chain
                // per row tile at or below the block, then summed
                typename MF::acc xt[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    xt[rt] = MF::zero();
                    if (rt < bk) continue;
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) xt[rt] = MF::mma(va[rt][s4], q[rt][s4], xt[rt]);
                }
                typename MF::acc x = xt[RT - 1];
#pragma unroll
                for (int rt = 0; rt < RT - 1; ++rt)
                    if (rt >= bk) x += xt[rt];
                // Y = T_b X
                typename MF::acc y = MF::zero();
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) y = MF::mma(tv[s4], x[s4], y);
                // Q -= V_b Y, the row tiles' chains interleaved
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        if (rt >= bk) q[rt] = MF::mma(vb[rt][s4], y[s4], q[rt]);
                }
            }
            BED_MARK(7, 4);
            // sign canonicalization: largest |.| entry positive, lowest row on ties
            T best = T(-1), bval = T(0);
            int brow = 1 << 20;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rt + MF::crow(lane, v);
                    const T av = f_abs(q[rt][v]);
                    if (row < n && (av > best || (av == best && row < brow))) {
                        best = av;
                        brow = row;
                        bval = q[rt][v];
                    }
                }
            }
            {
                const T ob = xmove<16>(best, lane);
                const int orow = xmove<16>(brow, lane);
                const T oval = xmove<16>(bval, lane);
                if (ob > best || (ob == best && orow < brow)) {
                    best = ob;
                    brow = orow;
                    bval = oval;
                }
            }
            {
                const T ob = xmove<32>(best, lane);
                const int orow = xmove<32>(brow, lane);
                const T oval = xmove<32>(bval, lane);
                if (ob > best || (ob == best && orow < brow)) {
                    best = ob;
                    brow = orow;
                    bval = oval;
                }
            }
            const T sgn = (bval < T(0)) ? T(-1) : T(1);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rt + MF::crow(lane, v);
                    if (row < n && c < n) Qn[row * LD + c] = sgn * q[rt][v];
                }
            }
        }
    }
    team_sync<NT>();
    BED_PHASE(4);
    for (int i = t / n, j = t % n, e = t; e < n * n; e += NT) {
        Q_out[e] = Qn[i * LD + j];
        j += NT % n;
        i += NT / n;
        if (j >= n) {
            j -= n;
            ++i;
        }
    }
    for (int e = t; e < n; e += NT) lam_out[e] = fexp<T>::pow2(-input_shift(S)) * Lc[e];
    if (t == 0 && info_out) *info_out = S.capped;
    BED_PHASE(5);
    }
}

}  // namespace bed
