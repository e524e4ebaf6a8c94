// Trust-region Newton inversion of the element map (Section 3.2.1) for
// (point, candidate element) pairs grouped by element, with the element-map
// contraction on the matrix cores.  Instantiated in kernels_newton.hip
// (hex, quad and surface kinds); kernels_eval.hip shares its LDS layout.
//
// Task = one element and the queue of its pairs.  The wave stages the
// element's nodal coordinates in LDS and serves 16 pairs at a time, one per
// slot; slot s owns lanes s, s+16, s+32, s+48 (g = lane / 16 picks the
// quarter).  When a slot's pair is done it takes the next pair of the queue.
//
// One map evaluation for the 16 slots at their reference points q_s:
//   stage 1 (MFMA, v_mfma_{f64,f32}_16x16x4):
//       C[row][s] = sum_i X[c][i][row] phi_i(q_s,0)   (and phi' / phi'')
//     where row = (j, k) flattened (hex) or j (quad); A = node rows from LDS,
//     B = the slot's bases (lane provides phi_i for i = 4 ks + g), so the
//     16 MFMA columns are the 16 slots and lane l receives four rows of each
//     16-row tile (which four depends on the instruction) for its own slot.
//   stage 2+3 (VALU): each lane weights its rows with phi_j(s) phi_k(t) (and
//     derivatives) of its slot, read from a per-slot LDS table (for N = 4, 8
//     summed over k first, then weighted per j), and the four lanes of a
//     slot are summed by lane swaps, four values at a time.  Each sum is
//     formed once and broadcast, so the four lanes hold bit-identical values
//     and run the Newton update redundantly and in step.
// Second derivatives (beta = 1 passes on faces/edges, eq. eq_newton_hessian)
// are computed in a separate sweep contracted with the slot's residual dx,
// run when enough slots wait for it (or nothing else can proceed).
//
// Mixed precision: the FP32 phase runs every pair of the element on FP32
// nodes stored as offsets from the element centre (points shifted the same
// way in FP64 before rounding) until ||dr|| < mixed_tol (default 1e-3) or
// mixed_max_iter passes; the FP64 phase then evaluates the map at that r
// and takes one Newton step, which ends the iteration when it is at most
// kPolishTol and off the faces (the polish step), else the iteration goes
// on in FP64 from there with alpha = 1.  Codes, distances and the final
// residual come from the FP64 phase.
#pragma once
#include <cfloat>
#include <type_traits>

#include "fpts_internal.hpp"
#include "gll_table.hpp"

namespace fpts {
namespace newton {

template <typename T> struct V4;
template <> struct V4<double> { typedef double __attribute__((ext_vector_type(4))) type; };
template <> struct V4<float> { typedef float __attribute__((ext_vector_type(4))) type; };

__device__ __forceinline__ V4<double>::type mfma16(double a, double b, V4<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ V4<float>::type mfma16(float a, float b, V4<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ inline T eps_of();
template <> __device__ inline double eps_of<double>() { return DBL_EPSILON; }
template <> __device__ inline float eps_of<float>() { return FLT_EPSILON; }

// 1/x for a positive normal x (an LDL^T pivot): the hardware reciprocal,
// refined by two Newton steps in FP64 (its first guess is good to about 23
// bits) and used as it is in FP32 (1 ulp).  A step direction needs no
// correctly rounded quotient, and this is a third of the division sequence.
template <typename T> __device__ T rcp_pos(T x);
template <> __device__ __forceinline__ double rcp_pos<double>(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}
template <> __device__ __forceinline__ float rcp_pos<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);
}

// Square root to about 23 bits (one hardware instruction): only for the
// rounding-noise threshold of the trust-region test, a scale, not a result.
template <typename T> __device__ T sqrt_scale(T x);
template <> __device__ __forceinline__ double sqrt_scale<double>(double x)
{
    return __builtin_amdgcn_sqrt(x);
}
template <> __device__ __forceinline__ float sqrt_scale<float>(float x)
{
    return __builtin_amdgcn_sqrtf(x);
}

template <typename T> __device__ __forceinline__ T xor_shfl(T v, int m);
template <> __device__ __forceinline__ double xor_shfl<double>(double v, int m)
{
    return __shfl_xor(v, m);
}
template <> __device__ __forceinline__ float xor_shfl<float>(float v, int m)
{
    return __shfl_xor(v, m);
}

// Orders LDS accesses between the lanes of a wave (every workgroup here is
// one wave).  The LDS instructions of a wave complete in issue order, so only
// compiler motion has to be fenced: no wait is emitted.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The two results of v_permlane16_swap (v_permlane32_swap) applied to (x, y):
// the instruction trades rows (16-lane rows; 32-lane halves) between its two
// registers, so each result holds, row by row, values of x from one row of
// a row pair and values of y from the same row.  Used only in sums that
// come out the same whichever half of a pair moves.
template <typename T> struct Two { T a, b; };
__device__ __forceinline__ Two<float> swap16(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                    false);
    return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ Two<float> swap32(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                    false);
    return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ Two<double> swap16(double x, double y)
{
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x),
                                                     (unsigned)__double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x),
                                                     (unsigned)__double2hiint(y), false, false);
    return {__hiloint2double((int)hi[0], (int)lo[0]), __hiloint2double((int)hi[1], (int)lo[1])};
}
__device__ __forceinline__ Two<double> swap32(double x, double y)
{
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x),
                                                     (unsigned)__double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x),
                                                     (unsigned)__double2hiint(y), false, false);
    return {__hiloint2double((int)hi[0], (int)lo[0]), __hiloint2double((int)hi[1], (int)lo[1])};
}

// Sum of v over the four lanes of a slot (lanes l, l^16, l^32, l^48): the
// swap of v with itself gives every lane its own value and its partner's, in
// the same order in both lanes of the pair, so the four lanes end with
// bit-identical sums.
template <typename T>
__device__ __forceinline__ T slot_sum(T v)
{
    Two<T> p = swap16(v, v);
    v = p.a + p.b;
    p = swap32(v, v);
    return p.a + p.b;
}

// slot_sum of K values, four at a time by transposition: the 16-lane swap of
// (v0, v1) followed by an add leaves the row-pair sums of v0 in one row of
// each pair and those of v1 in the other; the 32-lane swap of two such
// results (v0/v1 and v2/v3) and an add complete the sums, the total of one
// value per row.  The same swaps of a total with itself then broadcast each
// row's total to the four rows.  Each total is formed once (bit-identical in
// the four lanes), with 9 swaps per four values instead of 16.
template <typename T, int K>
__device__ __forceinline__ void slot_sum_all(T (&v)[K])
{
    constexpr int Q = K / 4;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        Two<T> p = swap16(v[4 * i], v[4 * i + 1]);
        const T w01 = p.a + p.b;
        p = swap16(v[4 * i + 2], v[4 * i + 3]);
        const T w23 = p.a + p.b;
        p = swap32(w01, w23);
        const T z = p.a + p.b;
        p = swap32(z, z);
        const Two<T> h0 = swap16(p.a, p.a), h1 = swap16(p.b, p.b);
        v[4 * i] = h0.a;
        v[4 * i + 1] = h0.b;
        v[4 * i + 2] = h1.a;
        v[4 * i + 3] = h1.b;
    }
    if constexpr (K % 4 >= 2) {
        constexpr int i = 4 * Q;
        Two<T> p = swap16(v[i], v[i + 1]);
        T w = p.a + p.b;
        p = swap32(w, w);
        w = p.a + p.b;
        p = swap16(w, w);
        v[i] = p.a;
        v[i + 1] = p.b;
    }
    if constexpr (K % 2 == 1) v[K - 1] = slot_sum(v[K - 1]);
}

// Contraction row of the 16x16 output tile m held by lane quarter g in item
// qq: 16 m + g + 4 qq.  The FP64 instruction interleaves the tile's rows that
// way (item qq of quarter g is tile row g + 4 qq); the FP32 one gives each
// quarter four consecutive tile rows (4 g + qq), so the FP32 A operand
// supplies the rows transposed (a_row) to land on the same contraction rows.
// Both layouts checked on gfx950.
__device__ __forceinline__ int out_row(int m, int g, int qq) { return 16 * m + g + 4 * qq; }
template <typename T>
__device__ __forceinline__ int a_row(int m, int slot)
{
    return 16 * m + (std::is_same<T, double>::value ? slot : (slot >> 2) + 4 * (slot & 3));
}

template <int D, int R, int N>
struct Shape {
    static constexpr int NP = (R == 3) ? N * N * N : N * N;
    static constexpr int ROWS = (R == 3) ? N * N : N;   // contraction rows
    static constexpr int MT = (ROWS + 15) / 16;         // 16-row tiles
    static constexpr int KS = (N + 3) / 4;              // 4-wide K steps
};

// Where node (coordinate c, contraction row `row`, first index i) of the
// element sits in LDS.  The 16 lanes of a lane quarter read the A operand
// from 16 consecutive rows at one i; with rows of an even number of values
// stored back to back those reads share a few LDS banks (N = 8 doubles: two
// banks pairs for 16 lanes).  Rows of an odd length P = N + 1 spread them
// over 16; FP64 with N = 8 instead rotates each row by row / 2 positions
// (no padding: the wave's LDS stays within 20 KB, eight waves per CU).
template <typename T, int D, int R, int N>
struct NodeLds {
    typedef Shape<D, R, N> S;
    static constexpr bool ROT = std::is_same<T, double>::value && N == 8;
    static constexpr int P = (ROT || N % 2) ? N : N + 1;
    static constexpr int RP = S::ROWS * P;               // per coordinate
    static constexpr int SIZE = D * RP;
    static constexpr bool PLAIN = !ROT && P == N;        // the global layout
    __device__ static __forceinline__ int at(int c, int row, int i)
    {
        return c * RP + row * P + (ROT ? ((i + (row >> 1)) & (N - 1)) : i);
    }
};

// Packed symmetric R x R matrices: diagonal first, then the upper triangle.
template <int R> constexpr int kSym = R * (R + 1) / 2;
template <int R>
__device__ constexpr int sym(int a, int b)
{
    if (a == b) return a;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return R == 2 ? 2 : (lo == 0 ? (hi == 1 ? 3 : 4) : 5);
}

// phi_i, phi_i', phi_i'' at x for ONE index i (runtime, per lane): the
// product over m != i of (x - z_m) carried as a jet, times w_i.
template <typename T, int N>
__device__ __forceinline__ void basis_at(T x, int i, T &v, T &d, T &dd)
{
    constexpr gll::Table<N> G = gll::Nodes<N>::t;
    T pv = T(1), pd = T(0), pdd = T(0), wi = T(0);
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const bool self = (m == i);
        const T u = self ? T(1) : x - T(G.z[m]);
        const T du = self ? T(0) : T(1);
        pdd = pdd * u + T(2) * pd * du;
        pd = pd * u + pv * du;
        pv = pv * u;
        wi = self ? T(G.w[m]) : wi;
    }
    v = wi * pv;
    d = wi * pd;
    dd = wi * pdd;
}

// All N bases of one direction at x (prefix/suffix jets), written to the
// per-slot LDS table tab[kind][i][slot] (kind 0: phi, 1: phi', 2: phi'')
// when `write` holds.
template <typename T, int N, bool H2>
__device__ __forceinline__ void basis_table(T x, T *tab, int slot, bool write)
{
    constexpr gll::Table<N> G = gll::Nodes<N>::t;
    // The jets of the first one or two factors are written out (1, 0, 0),
    // (t, 1, 0), (., ., 2): products with the constants 0 and 1 would
    // otherwise be issued, since they cannot be folded for a general x.
    T pv[N], pd[N], pdd[N];
    pv[0] = T(1);
    pd[0] = T(0);
    pdd[0] = T(0);
#pragma unroll
    for (int i = 1; i < N; ++i) {
        const T t = x - T(G.z[i - 1]);
        if (H2) pdd[i] = i == 1 ? T(0) : i == 2 ? T(2) * pd[1] : pdd[i - 1] * t + T(2) * pd[i - 1];
        pd[i] = i == 1 ? T(1) : pd[i - 1] * t + pv[i - 1];
        pv[i] = i == 1 ? t : pv[i - 1] * t;
    }
    T sv = T(1), sd = T(0), sdd = T(0);
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        const int ns = N - 1 - i;   // factors in the suffix
        if (write) {
            const T v = ns == 0 ? pv[i] : pv[i] * sv;
            const T d = ns == 0 ? pd[i] : ns == 1 ? pd[i] * sv + pv[i] : pd[i] * sv + pv[i] * sd;
            tab[(0 * N + i) * 16 + slot] = T(G.w[i]) * v;
            tab[(1 * N + i) * 16 + slot] = T(G.w[i]) * d;
            if (H2) {
                const T dd = ns == 0   ? pdd[i]
                             : ns == 1 ? pdd[i] * sv + T(2) * pd[i]
                                       : pdd[i] * sv + T(2) * pd[i] * sd + pv[i] * sdd;
                tab[(2 * N + i) * 16 + slot] = T(G.w[i]) * dd;
            }
        }
        const T t = x - T(G.z[i]);
        if (H2) sdd = ns == 0 ? T(0) : ns == 1 ? T(2) * sd : sdd * t + T(2) * sd;
        sd = ns == 0 ? T(1) : sd * t + sv;
        sv = ns == 0 ? t : sv * t;
    }
}

// Pairs staged per refill of a wave's slots (coordinates, start and id).
// 32 keeps the FP64 LDS footprint of hexes with N <= 8 within 20 KB, so that
// eight waves fit a CU.
constexpr int kCache = 32;

// LDS layout of one wave: nodes [D][NP] of type T, then the per-slot basis
// tables of directions 1 and 2 (s, t): [2][3][N][16] of type T.
template <typename T, int D, int R, int N>
struct Lds {
    static constexpr int NODES = NodeLds<T, D, R, N>::SIZE;
    static constexpr int TAB = 3 * N * 16;
    // pair cache: kCache x (point coordinates D, start r R) of type T, then
    // kCache item ids and kCache start-node indices
    static constexpr int CACHE = kCache * (D + R);
    static constexpr size_t bytes()
    {
        return sizeof(T) * (NODES + 2 * TAB + CACHE) + sizeof(int) * 2 * kCache;
    }
    __device__ static int *citem(void *lds)
    {
        return reinterpret_cast<int *>(reinterpret_cast<char *>(lds) + bytes() -
                                       sizeof(int) * 2 * kCache);
    }
};

// Rows of the differentiation matrix at the GLL nodes: v[a][m] = phi_m'(z_a),
// by the same prefix/suffix product rule as the sweeps' bases (compile time).
template <typename T, int N>
struct DiffRows {
    T v[N][N];
};
template <typename T, int N>
constexpr DiffRows<T, N> make_diff()
{
    constexpr gll::Table<N> G = gll::Nodes<N>::t;
    DiffRows<T, N> d{};
    for (int a = 0; a < N; ++a) {
        const double x = G.z[a];
        double pv[N] = {}, pd[N] = {};
        pv[0] = 1.0;
        for (int i = 1; i < N; ++i) {
            const double t = x - G.z[i - 1];
            pd[i] = pd[i - 1] * t + pv[i - 1];
            pv[i] = pv[i - 1] * t;
        }
        double sv = 1.0, sd = 0.0;
        for (int i = N - 1; i >= 0; --i) {
            d.v[a][i] = T(G.w[i] * (pd[i] * sv + pv[i] * sd));
            const double t = x - G.z[i];
            sd = sd * t + sv;
            sv = sv * t;
        }
    }
    return d;
}
template <typename T, int N>
__device__ const DiffRows<T, N> kDiff = make_diff<T, N>();

// Stage 2+3 factored by j for hexes whose 16-row tiles hold whole (j, k)
// blocks (N = 4, 8): a lane's rows 16 m + g + 4 qq have j = g + 4 (qq % NJ)
// whatever m is, so the k-weights are summed per j first and the j-weights
// applied once at the end.
template <int R, int N>
struct Factor {
    static constexpr bool ON = R == 3 && (N == 4 || N == 8);
    static constexpr int NJ = N / 4 > 0 ? N / 4 : 1;   // the lane's distinct j
};

// Sweep 1 for all 16 slots: x(q) and G = dx/dr of each slot's point.
template <typename T, int D, int R, int N>
__device__ __forceinline__ void sweep1(const T *xl, T *tab, int lane, const T (&q)[R], T (&X)[D],
                                       T (&G)[D][R])
{
    typedef Shape<D, R, N> S;
    typedef Factor<R, N> F;
    typedef typename V4<T>::type v4;
    const int slot = lane & 15, g = lane >> 4;
    // per-slot tables [direction][kind][i][slot] (kinds phi, phi'): lane
    // quarter g builds direction g of its slot, so the R tables of all 16
    // slots are built at once
    wave_lds_sync();   // the previous sweep's reads of the tables come first
    {
        // q[g] by exact arithmetic selection (one weight is 1, the others
        // 0), which keeps q in registers
        const T w0 = T(g != 1 && g != 2), w1 = T(g == 1), w2 = T(R == 3 && g == 2);
        T x = q[0] * w0;
        x = fma(q[1], w1, x);
        if (R == 3) x = fma(q[R == 3 ? 2 : 0], w2, x);
        basis_table<T, N, false>(x, tab + (g < R ? g : 0) * 2 * N * 16, slot, g < R);
    }
    wave_lds_sync();
    const T *tr = tab, *ts = tab + 2 * N * 16, *tt = tab + 4 * N * 16;
    // B operand: this lane's bases in direction 0 for i = 4 ks + g
    T b0[S::KS], b1[S::KS];
#pragma unroll
    for (int ks = 0; ks < S::KS; ++ks) {
        const int i = 4 * ks + g;
        b0[ks] = i < N ? tr[(0 * N + i) * 16 + slot] : T(0);
        b1[ks] = i < N ? tr[(1 * N + i) * 16 + slot] : T(0);
    }
    // the lane's partial sums: X, G directly, or (factored) per j the
    // k-weighted sums Zv = sum_k C0 t_k, Zd = sum_k C1 t_k, Zt = sum_k C0 t'_k
    T Zv[F::NJ][D], Zd[F::NJ][D], Zt[F::NJ][D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        X[c] = T(0);
#pragma unroll
        for (int a = 0; a < R; ++a) G[c][a] = T(0);
#pragma unroll
        for (int js = 0; js < F::NJ; ++js) {
            Zv[js][c] = T(0);
            Zd[js][c] = T(0);
            Zt[js][c] = T(0);
        }
    }
    constexpr bool kFullA = (N % 4 == 0) && (S::ROWS % 16 == 0);
    // one row tile; the first is issued on its own, where the partial sums
    // are still the constant 0 (no registers to clear for the loop)
    auto tile = [&](int m) __attribute__((always_inline)) {
        v4 acc0[D], acc1[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            acc0[c] = v4{0, 0, 0, 0};
            acc1[c] = v4{0, 0, 0, 0};
        }
        const int arow = a_row<T>(m, slot);   // A-operand row of this lane
#pragma unroll
        for (int ks = 0; ks < S::KS; ++ks) {
            const int ai = 4 * ks + g;      // A-operand column (node index i)
            const bool aok = kFullA || (arow < S::ROWS && ai < N);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                // out-of-range A entries meet a zero B entry (ai >= N) or
                // land in output rows that are dropped (arow >= ROWS); the
                // clamped address keeps the read inside the node block
                const T a = xl[aok ? NodeLds<T, D, R, N>::at(c, arow, ai) : 0];
                acc0[c] = mfma16(a, b0[ks], acc0[c]);
                acc1[c] = mfma16(a, b1[ks], acc1[c]);
            }
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int row = out_row(m, g, qq);
            if (S::ROWS % 16 != 0 && row >= S::ROWS) continue;
            if constexpr (F::ON) {
                const int k = (16 * m + 4 * qq) / N, js = qq % F::NJ;   // row / N (g < 4)
                const T tv = tt[(0 * N + k) * 16 + slot], td = tt[(1 * N + k) * 16 + slot];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    Zv[js][c] = fma(acc0[c][qq], tv, Zv[js][c]);
                    Zd[js][c] = fma(acc1[c][qq], tv, Zd[js][c]);
                    Zt[js][c] = fma(acc0[c][qq], td, Zt[js][c]);
                }
            } else if constexpr (R == 3) {
                const int j = row % N, k = row / N;
                const T sv = ts[(0 * N + j) * 16 + slot], sd = ts[(1 * N + j) * 16 + slot];
                const T tv = tt[(0 * N + k) * 16 + slot], td = tt[(1 * N + k) * 16 + slot];
                const T w00 = sv * tv, w10 = sd * tv, w01 = sv * td;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    X[c] = fma(acc0[c][qq], w00, X[c]);
                    G[c][0] = fma(acc1[c][qq], w00, G[c][0]);
                    G[c][1] = fma(acc0[c][qq], w10, G[c][1]);
                    G[c][2] = fma(acc0[c][qq], w01, G[c][2]);
                }
            } else {
                const int j = row;
                const T sv = ts[(0 * N + j) * 16 + slot], sd = ts[(1 * N + j) * 16 + slot];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    X[c] = fma(acc0[c][qq], sv, X[c]);
                    G[c][0] = fma(acc1[c][qq], sv, G[c][0]);
                    G[c][1] = fma(acc0[c][qq], sd, G[c][1]);
                }
            }
        }
    };
    tile(0);
#pragma unroll 1
    for (int m = 1; m < S::MT; ++m) tile(m);
    if constexpr (F::ON) {
#pragma unroll
        for (int js = 0; js < F::NJ; ++js) {
            const int j = g + 4 * js;
            const T sv = ts[(0 * N + j) * 16 + slot], sd = ts[(1 * N + j) * 16 + slot];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                X[c] = fma(Zv[js][c], sv, X[c]);
                G[c][0] = fma(Zd[js][c], sv, G[c][0]);
                G[c][1] = fma(Zv[js][c], sd, G[c][1]);
                G[c][2] = fma(Zt[js][c], sv, G[c][2]);
            }
        }
    }
    T v[D * (R + 1)];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        v[c] = X[c];
#pragma unroll
        for (int a = 0; a < R; ++a) v[D + c * R + a] = G[c][a];
    }
    slot_sum_all(v);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        X[c] = v[c];
#pragma unroll
        for (int a = 0; a < R; ++a) G[c][a] = v[D + c * R + a];
    }
}

// Sweep 2: S_ab = sum_c dx_c d2x_c/dr_a dr_b at each slot's q.
template <typename T, int D, int R, int N>
__device__ __forceinline__ void sweep2(const T *xl, T *tab, int lane, const T (&q)[R],
                                       const T (&dx)[D], T (&Sout)[kSym<R>])
{
    typedef Shape<D, R, N> S;
    typedef Factor<R, N> F;
    typedef typename V4<T>::type v4;
    const int slot = lane & 15, g = lane >> 4;
    T b0[S::KS], b1[S::KS], b2[S::KS];
#pragma unroll
    for (int ks = 0; ks < S::KS; ++ks) {
        const int i = 4 * ks + g;
        T v, d, dd;
        basis_at<T, N>(q[0], i, v, d, dd);
        b0[ks] = i < N ? v : T(0);
        b1[ks] = i < N ? d : T(0);
        b2[ks] = i < N ? dd : T(0);
    }
    // per-slot tables [direction - 1][kind][i][slot] (phi, phi', phi'') of
    // directions 1 (lane quarter 1) and 2 (lane quarter 2)
    wave_lds_sync();
    {
        const T x = (R == 3 && g == 2) ? q[R == 3 ? 2 : 0] : q[1];
        const bool w = g == 1 || (R == 3 && g == 2);
        basis_table<T, N, true>(x, tab + (g == 2 ? 3 * N * 16 : 0), slot, w);
    }
    wave_lds_sync();
    const T *tt = tab + 3 * N * 16;
    T Sa[kSym<R>];
    // factored: per j, Z[0..5] = sum_k of C2 t, C0 t, C0 t'', C1 t, C1 t',
    // C0 t' (then times s, s'', s, s', s, s' of j)
    T Z[F::NJ][6];
#pragma unroll
    for (int a = 0; a < kSym<R>; ++a) Sa[a] = T(0);
#pragma unroll
    for (int js = 0; js < F::NJ; ++js)
#pragma unroll
        for (int a = 0; a < 6; ++a) Z[js][a] = T(0);
    auto tile = [&](int m) __attribute__((always_inline)) {
        // the slot's residual enters the B operand, so one accumulator per
        // basis kind collects sum_c dx_c C_c[row][slot] over the coordinates
        v4 acc0 = v4{0, 0, 0, 0}, acc1 = v4{0, 0, 0, 0}, acc2 = v4{0, 0, 0, 0};
        const int arow = a_row<T>(m, slot);
#pragma unroll
        for (int ks = 0; ks < S::KS; ++ks) {
            const int ai = 4 * ks + g;
            const bool aok = ((N % 4 == 0) && (S::ROWS % 16 == 0)) || (arow < S::ROWS && ai < N);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T a = xl[aok ? NodeLds<T, D, R, N>::at(c, arow, ai) : 0];
                acc0 = mfma16(a, dx[c] * b0[ks], acc0);
                acc1 = mfma16(a, dx[c] * b1[ks], acc1);
                acc2 = mfma16(a, dx[c] * b2[ks], acc2);
            }
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int row = out_row(m, g, qq);
            if (S::ROWS % 16 != 0 && row >= S::ROWS) continue;
            const T C0 = acc0[qq], C1 = acc1[qq], C2 = acc2[qq];
            if constexpr (F::ON) {
                const int k = (16 * m + 4 * qq) / N, js = qq % F::NJ;
                const T tv = tt[(0 * N + k) * 16 + slot], td = tt[(1 * N + k) * 16 + slot];
                const T tdd = tt[(2 * N + k) * 16 + slot];
                Z[js][0] = fma(C2, tv, Z[js][0]);
                Z[js][1] = fma(C0, tv, Z[js][1]);
                Z[js][2] = fma(C0, tdd, Z[js][2]);
                Z[js][3] = fma(C1, tv, Z[js][3]);
                Z[js][4] = fma(C1, td, Z[js][4]);
                Z[js][5] = fma(C0, td, Z[js][5]);
            } else if constexpr (R == 3) {
                const int j = row % N, k = row / N;
                const T sv = tab[(0 * N + j) * 16 + slot], sd = tab[(1 * N + j) * 16 + slot];
                const T sdd = tab[(2 * N + j) * 16 + slot];
                const T tv = tt[(0 * N + k) * 16 + slot], td = tt[(1 * N + k) * 16 + slot];
                const T tdd = tt[(2 * N + k) * 16 + slot];
                Sa[0] = fma(C2, sv * tv, Sa[0]);    // rr
                Sa[1] = fma(C0, sdd * tv, Sa[1]);   // ss
                Sa[2] = fma(C0, sv * tdd, Sa[2]);   // tt
                Sa[3] = fma(C1, sd * tv, Sa[3]);    // rs
                Sa[4] = fma(C1, sv * td, Sa[4]);    // rt
                Sa[5] = fma(C0, sd * td, Sa[5]);    // st
            } else {
                const int j = row;
                const T sv = tab[(0 * N + j) * 16 + slot], sd = tab[(1 * N + j) * 16 + slot];
                const T sdd = tab[(2 * N + j) * 16 + slot];
                Sa[0] = fma(C2, sv, Sa[0]);         // rr
                Sa[1] = fma(C0, sdd, Sa[1]);        // ss
                Sa[2] = fma(C1, sd, Sa[2]);         // rs
            }
        }
    };
    tile(0);
#pragma unroll 1
    for (int m = 1; m < S::MT; ++m) tile(m);
    if constexpr (F::ON) {
#pragma unroll
        for (int js = 0; js < F::NJ; ++js) {
            const int j = g + 4 * js;
            const T sv = tab[(0 * N + j) * 16 + slot], sd = tab[(1 * N + j) * 16 + slot];
            const T sdd = tab[(2 * N + j) * 16 + slot];
            Sa[0] = fma(Z[js][0], sv, Sa[0]);    // rr
            Sa[1] = fma(Z[js][1], sdd, Sa[1]);   // ss
            Sa[2] = fma(Z[js][2], sv, Sa[2]);    // tt
            Sa[3] = fma(Z[js][3], sd, Sa[3]);    // rs
            Sa[4] = fma(Z[js][4], sv, Sa[4]);    // rt
            Sa[5] = fma(Z[js][5], sd, Sa[5]);    // st
        }
    }
    slot_sum_all(Sa);
#pragma unroll
    for (int a = 0; a < kSym<R>; ++a) Sout[a] = Sa[a];
}

// Objective at a point: f = |x* - x|^2, g = G^T dx, Hgn = G^T G (packed).
template <typename T, int D, int R>
struct Obj {
    T f;
    T g[R];
    T Hgn[kSym<R>];
};

template <typename T, int D, int R>
__device__ __forceinline__ void objective(const T (&xs)[D], const T (&X)[D], const T (&G)[D][R],
                                          Obj<T, D, R> &o, T (&dx)[D])
{
    o.f = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) o.g[a] = T(0);
#pragma unroll
    for (int a = 0; a < kSym<R>; ++a) o.Hgn[a] = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        dx[c] = xs[c] - X[c];
        o.f = fma(dx[c], dx[c], o.f);
#pragma unroll
        for (int a = 0; a < R; ++a) {
            o.g[a] = fma(G[c][a], dx[c], o.g[a]);
#pragma unroll
            for (int b = a; b < R; ++b)
                o.Hgn[sym<R>(a, b)] = fma(G[c][a], G[c][b], o.Hgn[sym<R>(a, b)]);
        }
    }
}

// Solve H dr = g on the free coordinates (rows/columns of held coordinates
// replaced by the identity, right-hand side 0) by LDL^T; false when a pivot
// is not positive.
template <typename T, int R>
__device__ __forceinline__ bool solve_free(const T (&H)[kSym<R>], const T (&g)[R],
                                           const bool (&held)[R], T (&x)[R])
{
    T A[R][R], b[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
        b[a] = held[a] ? T(0) : g[a];
#pragma unroll
        for (int c = 0; c < R; ++c)
            A[a][c] = (held[a] || held[c]) ? (a == c ? T(1) : T(0)) : H[sym<R>(a, c)];
    }
    T L[R][R], d[R], inv[R];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < R; ++a) {
        T s = A[a][a];
#pragma unroll
        for (int k = 0; k < a; ++k) s -= L[a][k] * L[a][k] * d[k];
        d[a] = s;
        ok = ok && (s > T(0));
        inv[a] = rcp_pos(s);   // one reciprocal per pivot (unused when s <= 0)
#pragma unroll
        for (int c = a + 1; c < R; ++c) {
            T t = A[c][a];
#pragma unroll
            for (int k = 0; k < a; ++k) t -= L[c][k] * L[a][k] * d[k];
            L[c][a] = t * inv[a];
        }
    }
    T y[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
        T s = b[a];
#pragma unroll
        for (int k = 0; k < a; ++k) s -= L[a][k] * y[k];
        y[a] = s;
    }
#pragma unroll
    for (int a = R - 1; a >= 0; --a) {
        T s = y[a] * inv[a];
#pragma unroll
        for (int k = a + 1; k < R; ++k) s -= L[k][a] * x[k];
        x[a] = s;
    }
    return ok;
}

template <typename T, int R>
__device__ __forceinline__ bool on_face(const T (&r)[R])
{
    bool b = false;
#pragma unroll
    for (int a = 0; a < R; ++a) b = b || (fabs(r[a]) == T(1));
    return b;
}

struct NewtonArgs {
    const double *nodes;     // [nel][D][NP]
    const float *nodes32;    // [nel][D][NP] x - x_c (mixed mode)
    const double *near;      // [nel][4][NearLds NPAD] nearest-node score rows (FP64)
    const double *xc;        // [nel][D]     (mixed mode)
    const double *pts;       // [D][n]
    int n;
    int nel;
    NewtonIO io;             // io.r holds the start on entry, the result on exit
    int max_iter;
    double tol;
    double eps_d;
    int max_iter32;
    float tol32;
};

// Coordinate c of point p: from the packed copy when the caller made one.
template <int D>
__device__ __forceinline__ double point_coord(const NewtonArgs &a, int p, int c)
{
    return a.io.pts4 ? a.io.pts4[(size_t)p * pt_stride(D) + c] : a.pts[(size_t)c * a.n + p];
}

enum { S_FREE = 0, S_INIT = 1, S_STEP = 2, S_WAIT = 3 };

// Newton launches.  kPrimary: the primary candidates; in FP64 a pair whose
// next pass needs second derivatives is parked (NewtonIO::park_*) and the
// wave goes on with other pairs; in FP32 (mixed mode) such a pair ends the
// FP32 phase.  kResolve: the other candidates of unsettled points, second
// derivatives in the wave.  kFace: the parked pairs, resumed from their
// saved point, radius and pass count, second derivatives in the wave.
// kPolish: the primary candidates in the FP64 phase of mixed mode (as
// kPrimary, with the polish step and the double-batch refill).
enum { kPrimary = 0, kResolve = 1, kFace = 2, kPolish = 3 };

// per-slot counters are kept by the slot's leader lane, per-wave (sweep)
// counters by lane 0
struct Counters {
    unsigned long long pairs = 0, passes = 0, evals = 0, evals_h2 = 0, passes32 = 0,
                       evals32 = 0, evals_h2_exec = 0, sweeps = 0, sweeps_h2 = 0, sweeps32 = 0,
                       evals32_node = 0;
};

// Run the iteration of Section 3.2.1 for every pair of element e (its queue
// [q0, q1) in io.list), in precision T, 16 slots at a time.  FINAL: write
// code/elem/dist/r (FP64 phase); otherwise write r only (FP32 phase of mixed
// mode).  Each trip evaluates either sweep 1 at the slots' query points
// (start points of new pairs, trial points of the others) or, when enough
// slots wait for it, sweep 2 at the waiting slots' current points.
// stage(): stages the element's nodes in LDS (a no-op where the caller
// staged them: kResolve, before it wrote the starts, and kFace).
template <typename T, int D, int R, int N, bool FINAL, int KIND, typename Stage>
__device__ __forceinline__ void run_element(const NewtonArgs &a, int e, int q0, int q1,
                                            const T *xl, T *tab, T *cache, int *citem, int lane,
                                            int max_iter, T tol, const double *shift,
                                            Counters &cn, Stage &&stage)
{
    const int slot = lane & 15;
    const bool leader = lane < 16;
    const NewtonIO &io = a.io;
    int state = S_FREE, item = 0, pass = 0, pos = 0;
    // start node of the slot's pair (packed index, -1: the start is not a
    // node or not used); fresh: the slot's start was evaluated at its node
    // this trip.  Only the FP32 phase of mixed mode evaluates starts at their
    // nodes: its pairs take about two evaluations, so the start is half of
    // them; in FP64 (three to four) the extra refill-and-plan round per trip
    // cost more than the sweeps it saved (measured on hex48).
    constexpr bool kNodeStart = KIND != kFace && !FINAL;
    int nodeix = -1;
    bool fresh = false;
    int *cnode = citem + kCache;
    T xs[D], r[R], q[R], dx[D], Hs[kSym<R>], alpha = T(1), pred = T(0), dmax = T(0),
        xnorm = T(0);
    Obj<T, D, R> cur;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        xs[c] = T(0);
        dx[c] = T(0);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        r[k] = T(0);
        q[k] = T(0);
    }
#pragma unroll
    for (int k = 0; k < kSym<R>; ++k) Hs[k] = T(0);
    cur.f = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) cur.g[k] = T(0);
#pragma unroll
    for (int k = 0; k < kSym<R>; ++k) cur.Hgn[k] = T(0);
    bool hb_ok = false;
    int head = q0, cstart = q0, cend = q0;
    // Refill free slots from the element's queue, through a cache of the
    // next kCache pairs (one coalesced load per kCache pairs).  Wave-uniform.
    // When the staged batch runs out before every free slot has a pair, the
    // next batch is staged at once where pairs take one or two evaluations
    // (the FP32 phase and the polish phase of mixed mode: their slots turn
    // over every trip); with three to four evaluations per pair (FP64) the
    // slot waits for the next trip instead (the loop cost more there than
    // the idle slots, measured on hex48).
    constexpr int batches = (!FINAL || KIND == kPolish) ? 2 : 1;
    // The pair ids, points and starts of a batch of the queue (lane l: list
    // position b0 + l) are loaded into registers by fetch and written to the
    // cache when the batch is staged.  The batches follow each other in
    // list order, so where an element's queue spans many batches (the
    // primary and polish passes) the next batch is fetched as soon as the
    // current one is staged, and its loads complete behind the sweeps.
    // The starts are read at the pair's list position (io.start: issued at
    // once, beside the chain list -> point) or with its item (io.r; kFace:
    // the list holds park indices, and the point, the saved iterate and the
    // rest of the pair's state come from the park record).  Plain loads, as
    // an earlier kernel wrote them -- except in kResolve, whose wave wrote
    // its starts moments ago (agent-scope loads, which bypass L1).
    constexpr bool kAhead = KIND == kPrimary || KIND == kPolish;
    int nb_it = 0;
    double nb_pc[D], nb_sv[R];
    auto fetch = [&](int b0) __attribute__((always_inline)) {
        auto load_start = [&](const double *src) __attribute__((always_inline)) {
            if constexpr (KIND == kResolve)
                return __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                return *src;
        };
        const int idx = b0 + lane;
        nb_it = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) nb_pc[c] = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) nb_sv[k] = 0.0;
        if (lane < kCache && idx < q1) {
            const bool by_pos = KIND != kFace && io.start != nullptr;
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (by_pos) nb_sv[k] = load_start(io.start + (size_t)k * io.start_stride + idx);
            nb_it = io.list[idx];
            int p;
            if constexpr (KIND == kFace) p = io.park_meta[nb_it].x;
            else p = io.slot_pt ? io.slot_pt[nb_it] : nb_it;
#pragma unroll
            for (int c = 0; c < D; ++c) nb_pc[c] = point_coord<D>(a, p, c);
            if (!by_pos) {
#pragma unroll
                for (int k = 0; k < R; ++k)
                    nb_sv[k] = load_start(KIND == kFace ? io.park_r + (size_t)k * io.park_cap + nb_it
                                                        : io.r + (size_t)k * io.ostride + nb_it);
            }
        }
    };
    // the primary and polish passes fetch the first batch before the nodes
    // are staged, so that the two wait together (the face kernel would spill
    // registers for it; kResolve writes its starts after staging)
    constexpr bool kEarly = kAhead;
    if constexpr (kEarly) fetch(q0);
    stage();
    auto refill = [&]() {
#pragma unroll 1
        for (int round = 0; round < batches; ++round) {
            const unsigned long long freem = __ballot(leader && state == S_FREE);
            const int nfree = __popcll(freem);
            if (!nfree || head >= q1) return;
            if (head >= cend) {
                // the next batch starts where the staged one ended
                wave_lds_sync();   // earlier reads of the cache come first
                cstart = head;
                cend = min(q1, head + kCache);
                if constexpr (!kAhead) {
                    if (!kEarly || cstart != q0) fetch(cstart);
                }
                const int idx = cstart + lane;
                if (lane < kCache && idx < cend) {
                    citem[lane] = nb_it;
#pragma unroll
                    for (int c = 0; c < D; ++c)
                        cache[c * kCache + lane] = T(nb_pc[c] - (shift ? shift[c] : 0.0));
#pragma unroll
                    for (int k = 0; k < R; ++k) cache[(D + k) * kCache + lane] = T(nb_sv[k]);
                    // a start that is a GLL node (every nearest-node start): its
                    // packed index, so that the start is evaluated from the node
                    // block directly (kFace resumes from parked iterates)
                    int node = -1;
                    if constexpr (kNodeStart) {
                        constexpr gll::Table<N> G = gll::Nodes<N>::t;
                        int mul = 1;
                        node = 0;
#pragma unroll
                        for (int k = 0; k < R; ++k) {
                            const T v = cache[(D + k) * kCache + lane];
                            int ik = -1;
#pragma unroll
                            for (int m = 0; m < N; ++m)
                                if (v == T(G.z[m])) ik = m;
                            node = (node < 0 || ik < 0) ? -1 : node + mul * ik;
                            mul *= N;
                        }
                    }
                    cnode[lane] = node;
                }
                if constexpr (kAhead)
                    if (cend < q1) fetch(cend);
                wave_lds_sync();
            }
            if (state == S_FREE) {
                const int rank = __popcll(freem & ((1ull << slot) - 1));
                const int idx = head + rank;
                if (idx < cend) {
                    const int c0 = idx - cstart;
                    item = citem[c0];
                    nodeix = cnode[c0];
                    pos = idx;
#pragma unroll
                    for (int c = 0; c < D; ++c) xs[c] = cache[c * kCache + c0];
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        r[k] = cache[(D + k) * kCache + c0];
                        q[k] = r[k];
                    }
                    T xn = T(0);
#pragma unroll
                    for (int c = 0; c < D; ++c) xn = fma(xs[c], xs[c], xn);
                    xnorm = sqrt_scale(xn);
                    state = S_INIT;
                    pass = 0;
                    alpha = T(1);
                    hb_ok = false;
                    if constexpr (KIND == kFace) {
                        // resumed where it was parked: same point, radius and
                        // pass count (the pair was counted by the primary pass)
                        const int4 mt = io.park_meta[item];
                        pass = mt.w;
                        alpha = T(io.park_r[(size_t)R * io.park_cap + item]);
                        if (item < io.park_state_cap) {
                            // with the state the evaluation at r left: the
                            // pair waits for its second derivatives at once
                            const double *ps = io.park_state + (size_t)item * kParkState;
                            cur.f = T(ps[0]);
#pragma unroll
                            for (int j = 0; j < R; ++j) cur.g[j] = T(ps[1 + j]);
#pragma unroll
                            for (int j = 0; j < kSym<R>; ++j) cur.Hgn[j] = T(ps[1 + R + j]);
#pragma unroll
                            for (int c = 0; c < D; ++c) dx[c] = T(ps[1 + R + kSym<R> + c]);
                            state = S_WAIT;
                        }
                        item = mt.x;
                        pos = mt.y;
                    } else if (leader && FINAL) {
                        cn.pairs++;
                    }
                }
            }
            head = min(head + nfree, cend);
        }
    };
    // A pair is done: results out, slot free.
    auto finish = [&](bool converged) {
        if (leader) {
            if (FINAL && io.conv) io.conv[item] = converged ? 1 : 0;
            if (FINAL) {
                bool inside = true;
#pragma unroll
                for (int k = 0; k < R; ++k) inside = inside && (fabs(r[k]) < T(1));
                if (R < D) inside = inside && (cur.f < T(a.eps_d));
                io.code[item] = inside ? FPTS_INTERIOR : FPTS_BORDER;
                if (io.elem) io.elem[item] = e;
                io.dist[item] = sqrt((double)cur.f);
                if (io.rs) {
                    double mg = 1.0;
#pragma unroll
                    for (int k = 0; k < R; ++k) mg = fmin(mg, 1.0 - fabs((double)r[k]));
                    const bool settles = inside && mg > kSettleGuard;
#pragma unroll
                    for (int k = 0; k < R; ++k)
                        io.rs[(size_t)k * io.rs_stride + pos] =
                            settles ? (double)r[k] : __builtin_nan("");
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (!FINAL && io.start)   // the FP64 phase's start
                    io.start[(size_t)k * io.start_stride + pos] = (double)r[k];
                else
                    io.r[(size_t)k * io.ostride + item] = (double)r[k];
            }
        }
        state = S_FREE;
    };
    // Slots whose new pair starts at a GLL node: the map there is the node
    // itself and dx/dr_d = sum_m phi_m'(z_{a_d}) x[.. m ..] (an N-term sum
    // along direction d through the node), read from the node block: no
    // sweep.  Quarter g < R sums direction g, quarter R reads the node; the
    // slot's four lanes are then summed (three of each four terms are zero).
    // Such slots go to S_STEP with the objective at the start, as an
    // evaluation by sweep 1 would leave them.  Returns whether any did.
    auto node_init = [&]() -> bool {
        if constexpr (!kNodeStart) {
            return false;
        } else {
            typedef NodeLds<T, D, R, N> NL;
            const bool mine = state == S_INIT && nodeix >= 0;
            if (!__ballot(leader && mine)) return false;
            const int g = lane >> 4;
            const int a0 = nodeix % N, a1 = (nodeix / N) % N, a2 = R == 3 ? nodeix / (N * N) : 0;
            T v[D * (R + 1)];
#pragma unroll
            for (int k = 0; k < D * (R + 1); ++k) v[k] = T(0);
            if (mine && g < R) {
                const int ag = g == 0 ? a0 : g == 1 ? a1 : a2;
                T dphi[N];
#pragma unroll
                for (int m = 0; m < N; ++m) dphi[m] = kDiff<T, N>.v[ag][m];
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const int ii = g == 0 ? m : a0, jj = g == 1 ? m : a1, kk = g == 2 ? m : a2;
                    const int base = NL::at(0, R == 3 ? jj + N * kk : jj, ii);
#pragma unroll
                    for (int c = 0; c < D; ++c)
                        v[D + c * R + g] = fma(dphi[m], xl[base + c * NL::RP], v[D + c * R + g]);
                }
            } else if (mine && g == R) {
                const int base = NL::at(0, R == 3 ? a1 + N * a2 : a1, a0);
#pragma unroll
                for (int c = 0; c < D; ++c) v[c] = xl[base + c * NL::RP];
            }
            slot_sum_all(v);
            if (mine) {
                T X[D], Gm[D][R];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    X[c] = v[c];
#pragma unroll
                    for (int k = 0; k < R; ++k) Gm[c][k] = v[D + c * R + k];
                }
                objective<T, D, R>(xs, X, Gm, cur, dx);
                hb_ok = false;
                state = S_STEP;
                fresh = true;
                if (leader) {
                    cn.evals32++;
                    cn.evals32_node++;
                }
            }
            return true;
        }
    };
    // Trial point of each stepping slot (only the fresh ones when asked):
    // the Newton step of Section 3.2.1 on the free coordinates, clipped to
    // the trust region and the box; a step below the tolerance ends the
    // iteration.  Returns, per lane, whether its slot's pair ended.
    auto plan = [&](bool only_fresh) -> bool {
        bool ended = false;
        if (state == S_STEP && (!only_fresh || fresh)) {
            const bool beta = (pass > 0) && on_face(r);
            if (beta && !hb_ok) {
                // a face pass needs second derivatives at r: dx at r is
                // current (r was evaluated last), so wait for sweep 2
                state = S_WAIT;
            } else {
                T H[kSym<R>];
#pragma unroll
                for (int k = 0; k < kSym<R>; ++k) H[k] = beta ? cur.Hgn[k] - Hs[k] : cur.Hgn[k];
                // held: at a bound of the box with the gradient pointing
                // out of it (r = +-1 exactly, so r g has the sign test)
                bool held[R];
#pragma unroll
                for (int k = 0; k < R; ++k)
                    held[k] = (fabs(r[k]) == T(1)) & (r[k] * cur.g[k] > T(0));
                T x[R];
                bool ok = solve_free<T, R>(H, cur.g, held, x);
                if (!ok && beta) {
#pragma unroll
                    for (int k = 0; k < kSym<R>; ++k) H[k] = cur.Hgn[k];
                    ok = solve_free<T, R>(H, cur.g, held, x);
                }
                T dr[R];
                dmax = T(0);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    T d = ok ? x[k] : T(0);
                    d = fmin(fmax(d, -alpha), alpha);
                    const T t = fmin(fmax(r[k] + d, T(-1)), T(1));
                    q[k] = t;
                    dr[k] = t - r[k];
                    dmax = fmax(dmax, fabs(dr[k]));
                }
                T gd = T(0), dHd = T(0);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    gd = fma(cur.g[k], dr[k], gd);
                    T w = T(0);   // (H dr)_k
#pragma unroll
                    for (int b = 0; b < R; ++b) w = fma(H[sym<R>(k, b)], dr[b], w);
                    dHd = fma(dr[k], w, dHd);
                }
                pred = T(2) * gd - dHd;
                if (dmax < tol) {
                    // converged: the step is taken without evaluating the
                    // map at q; the squared residual there is the model's,
                    // f - pred, whose error is third order in the step
                    ++pass;
                    if (leader) {
                        if (FINAL) cn.passes++;
                        else cn.passes32++;
                    }
#pragma unroll
                    for (int k = 0; k < R; ++k) r[k] = q[k];
                    cur.f = fmax(cur.f - pred, T(0));
                    finish(true);
                    ended = true;
                } else if (KIND == kPolish && R == D && io.polish && pass == 0 &&
                           dmax <= T(kPolishTol) && !on_face(r) && !on_face(q)) {
                    // mixed mode: the first FP64 step from the FP32 result
                    // is small and stays inside, so the start is within
                    // about kPolishTol of the solution and Newton's step
                    // leaves an error of second order in it; that step ends
                    // the iteration, with the model residual f - pred
                    ++pass;
                    if (leader) cn.passes++;
#pragma unroll
                    for (int k = 0; k < R; ++k) r[k] = q[k];
                    cur.f = fmax(cur.f - pred, T(0));
                    finish(true);
                    ended = true;
                }
            }
        }
        return ended;
    };
    const int guard = (q1 - q0 + 16) * (2 * max_iter + 4);
    for (int trip = 0; trip < guard; ++trip) {
        if constexpr (KIND == kPrimary || KIND == kPolish) {
            // pairs whose next pass needs second derivatives leave the wave:
            // FP64 parks them (the face kernel resumes them, many to a wave),
            // FP32 ends its phase there (the FP64 phase takes over)
            const unsigned long long pm = __ballot(leader && state == S_WAIT);
            if (pm) {
                // (a launch without a park buffer -- the hinted search of
                // particle tracking -- ends such pairs unconverged)
                if (FINAL && io.park_meta) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(io.park_count, __popcll(pm));
                    base = __shfl(base, 0);
                    if (state == S_WAIT) {
                        // park_cap is the pass's pair count: every pair is
                        // parked at most once, so k < park_cap
                        const int k = base + __popcll(pm & ((1ull << slot) - 1));
                        if (leader && k < io.park_cap) {
                            io.park_meta[k] = make_int4(item, pos, e, pass);
#pragma unroll
                            for (int j = 0; j < R; ++j)
                                io.park_r[(size_t)j * io.park_cap + k] = (double)r[j];
                            io.park_r[(size_t)R * io.park_cap + k] = (double)alpha;
                            static_assert(1 + R + kSym<R> + D <= kParkState, "park state");
                            if (k < io.park_state_cap) {
                                // the state at r, as the evaluation there left it
                                double *ps = io.park_state + (size_t)k * kParkState;
                                ps[0] = (double)cur.f;
#pragma unroll
                                for (int j = 0; j < R; ++j) ps[1 + j] = (double)cur.g[j];
#pragma unroll
                                for (int j = 0; j < kSym<R>; ++j)
                                    ps[1 + R + j] = (double)cur.Hgn[j];
#pragma unroll
                                for (int c = 0; c < D; ++c)
                                    ps[1 + R + kSym<R> + c] = (double)dx[c];
                            }
                        }
                        state = S_FREE;
                    }
                } else {
                    if (state == S_WAIT) finish(false);
                }
            }
        }
        // free slots take new pairs (those starting at a node are evaluated
        // there), then the trial points of the stepping slots; the slots
        // whose pairs that ends take new pairs at once, and those starting
        // at a node get their first trial point too (a second round), so no
        // slot idles in this trip's sweep.  One copy of each step.
        bool done = false;
        for (int round = 0;; round = 1) {
            refill();
            fresh = false;
            const bool any = node_init();
            if (round == 0) {
                const unsigned long long waitm = __ballot(leader && state == S_WAIT);
                const unsigned long long stepm =
                    __ballot(leader && (state == S_STEP || state == S_INIT));
                if (!waitm && !stepm) {
                    done = true;
                    break;
                }
                // a slot that waits for second derivatives gets them at
                // once: holding it back to batch more waiting slots (4 or
                // 8) costs more in idle slots than the batching saves
                // (measured on hex48); it is then planned with the others
                // and takes part in this trip's sweep 1
                if (KIND != kPrimary && KIND != kPolish && waitm != 0) {
                    T Sn[kSym<R>];
                    sweep2<T, D, R, N>(xl, tab, lane, r, dx, Sn);
                    if (lane == 0) {
                        if (FINAL) cn.sweeps_h2++;
                        else cn.sweeps32++;
                    }
                    if (state == S_WAIT) {
#pragma unroll
                        for (int k = 0; k < kSym<R>; ++k) Hs[k] = Sn[k];
                        hb_ok = true;
                        state = S_STEP;
                        if (leader && FINAL) cn.evals_h2++;
                    }
                    if (leader && FINAL && state != S_FREE) cn.evals_h2_exec++;
                }
            } else if (!any) {
                break;
            }
            const bool ended = plan(round == 1);
            if (round == 1 || !__ballot(leader && ended)) break;
        }
        if (done) break;
        if (state != S_INIT && state != S_STEP) {
#pragma unroll
            for (int k = 0; k < R; ++k) q[k] = r[k];
        }
        if (!__ballot(leader && (state == S_INIT || state == S_STEP))) continue;
        T X[D], Gm[D][R], dxn[D];
        sweep1<T, D, R, N>(xl, tab, lane, q, X, Gm);
        if (lane == 0) {
            if (FINAL) cn.sweeps++;
            else cn.sweeps32++;
        }
        Obj<T, D, R> nw;
        objective<T, D, R>(xs, X, Gm, nw, dxn);
        if (state == S_INIT) {
            cur = nw;
#pragma unroll
            for (int c = 0; c < D; ++c) dx[c] = dxn[c];
            hb_ok = false;
            state = S_STEP;
            // a resumed pair re-evaluates the point it was parked at (the
            // same values as before): not a new evaluation of the iteration
            if (leader && KIND != kFace) {
                if (FINAL) cn.evals++;
                else cn.evals32++;
            }
        } else if (state == S_STEP) {
            ++pass;
            if (leader) {
                if (FINAL) {
                    cn.evals++;
                    cn.passes++;
                } else {
                    cn.evals32++;
                    cn.passes32++;
                }
            }
            // trust-region test (the step is at least the tolerance here)
            bool accept;
            const T decr = cur.f - nw.f;
            const T sf = sqrt_scale(cur.f);
            const T noise = T(64) * eps_of<T>() * sf * (xnorm + sf);
            if (pred > T(0) && pred <= noise) {
                accept = true;
            } else if (pred > T(0) && decr >= T(0.9) * pred) {
                accept = true;
                alpha *= T(2);
            } else if (pred > T(0) && decr >= T(0.01) * pred) {
                accept = true;
            } else {
                accept = false;
                alpha *= T(0.25);
            }
            if (accept) {
#pragma unroll
                for (int k = 0; k < R; ++k) r[k] = q[k];
                cur = nw;
#pragma unroll
                for (int c = 0; c < D; ++c) dx[c] = dxn[c];
                hb_ok = false;
            }
            if (pass >= max_iter) finish(false);
            else if (accept && on_face(r)) state = S_WAIT;   // next pass: beta = 1
        }
    }
}

// Copies COUNT values of an element block from global memory to LDS (one
// wave), issuing every load before the first store, then waits for the
// workgroup.
template <typename T, int COUNT>
__device__ __forceinline__ void stage(T *lds, const T *src, int lane)
{
    typedef __attribute__((ext_vector_type(4))) unsigned int u4;
    constexpr int WORDS = COUNT * (int)sizeof(T) / 16;
    constexpr int PER = (WORDS + kWave - 1) / kWave;
    constexpr int BATCH = 4;   // 16-byte loads in flight per lane
    const u4 *s = reinterpret_cast<const u4 *>(src);
    u4 *d = reinterpret_cast<u4 *>(lds);
#pragma unroll 1
    for (int k0 = 0; k0 < PER; k0 += BATCH) {
        u4 v[BATCH];
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int w = (k0 + k) * kWave + lane;
            if (w < WORDS) v[k] = s[w];
        }
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int w = (k0 + k) * kWave + lane;
            if (w < WORDS) d[w] = v[k];
        }
    }
    constexpr int REST = COUNT * (int)sizeof(T) - WORDS * 16;   // 0, 4, 8 or 12 bytes
    const unsigned *s4 = reinterpret_cast<const unsigned *>(src);
    unsigned *d4 = reinterpret_cast<unsigned *>(lds);
    if (lane < REST / 4) d4[WORDS * 4 + lane] = s4[WORDS * 4 + lane];
    __syncthreads();
}

// Copies an element's node block [D][NP] (rows of N values) from global
// memory to LDS in the NodeLds layout, then waits for the workgroup.
template <typename T, int D, int R, int N>
__device__ __forceinline__ void stage_nodes(T *lds, const T *src, int lane)
{
    typedef NodeLds<T, D, R, N> L;
    constexpr int NP = Shape<D, R, N>::NP;
    if constexpr (L::PLAIN) {
        stage<T, D * NP>(lds, src, lane);
    } else {
        constexpr int COUNT = D * NP;
        constexpr int BATCH = 8;
#pragma unroll 1
        for (int v0 = 0; v0 < COUNT; v0 += BATCH * kWave) {
            T v[BATCH];
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int idx = v0 + k * kWave + lane;
                if (idx < COUNT) v[k] = src[idx];
            }
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int idx = v0 + k * kWave + lane;
                if (idx < COUNT) {
                    const int c = idx / NP, rem = idx - c * NP;
                    const int row = rem / N, i = rem - row * N;
                    lds[L::at(c, row, i)] = v[k];
                }
            }
        }
        __syncthreads();
    }
}

// Nearest-node contraction operands: B rows [4][NPAD] (-2 x_j, -2 y_j,
// -2 z_j, |x_j|^2 of every node j, element-local; padding columns score a
// large constant) and A rows [4][64] (x, y, z, 1 of each pair).  FP64 reads
// B from rows precomputed at setup (L2-resident per element), so its LDS
// holds only A and the item ids; FP32 builds B in LDS from the FP32 nodes.
template <typename T, int D, int R, int N>
struct NearLds {
    static constexpr int NPAD = (Shape<D, R, N>::NP + 31) / 32 * 32;   // even tile count
    static constexpr bool B_IN_LDS = std::is_same<T, float>::value;
    static constexpr size_t bytes()
    {
        return sizeof(T) * (4 * ((B_IN_LDS ? NPAD : 0) + 64) + 64) + sizeof(int) * 64;
    }
};

// Nearest element node of up to 64 pairs of one element (Euclidean; among
// equal scores the lowest node index), the start of Newton (Section 3.2.1).
// The squared distance |x - x_j|^2 = |x|^2 - 2 x.x_j + |x_j|^2 has the same
// minimiser as the score |x_j|^2 - 2 x.x_j, a K = 4 contraction of
// (x, y, z, 1) with (-2 x_j, -2 y_j, -2 z_j, |x_j|^2): one 16 x 16 x 4 MFMA
// scores 16 pairs against 16 nodes.  Coordinates are element-local (node
// block minus the element centre) to keep the cancellation small.
// FP64: the accumulator starts at |x|^2, so the MFMA yields the squared
// distance itself (non-negative), and the node index replaces the low
// kNodeBits mantissa bits; one minimum per score then keeps the nearest node
// with ties (equal to 2^-42 relative) to the lowest index.
constexpr int kNodeBits = 10;   // node indices below 1024 (N <= 10)
// one bit-field insert (mask from a scalar register: no literal operands
// here), in place in the low word; written out because the compiler would
// fold the node index's own arithmetic into an AND and an OR per score
__device__ __forceinline__ double with_node(double d, int node)
{
    const unsigned m = (1u << kNodeBits) - 1;
    unsigned lo = (unsigned)__double2loint(d);
    asm("v_bfi_b32 %0, %1, %2, %0" : "+v"(lo) : "s"(m), "v"(node));
    return __hiloint2double(__double2hiint(d), (int)lo);
}
// min of two keys: the keys are finite or +inf (never NaN), so the plain
// instruction serves; fmin() would first quiet both operands, which the
// compiler cannot prove to be ordinary numbers after the bit insertion.
__device__ __forceinline__ double key_min(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
template <int D, int R, int N, bool MIXED>
__device__ __forceinline__ void nearest_body(const NewtonArgs &a)
{
    typedef Shape<D, R, N> S;
    typedef NearLds<typename std::conditional<MIXED, float, double>::type, D, R, N> L;
    typedef typename std::conditional<MIXED, float, double>::type T;
    typedef typename V4<T>::type v4;
    constexpr gll::Table<N> GT = gll::Nodes<N>::t;
    constexpr int NT = L::NPAD / 16;   // node tiles (even)
    const T kBig = MIXED ? T(1e30f) : T(1e300);
    extern __shared__ double lds_raw[];
    T *Bt = reinterpret_cast<T *>(lds_raw);                  // [4][NPAD] (FP32)
    T *Pt = Bt + (L::B_IN_LDS ? 4 * L::NPAD : 0);            // [4][64]
    T *Xx = Pt + 4 * 64;                                     // [64] |x|^2
    int *items = reinterpret_cast<int *>(Xx + 64);           // [64]
    const int lane = threadIdx.x, col = lane & 15, g = lane >> 4;
    const NewtonIO &io = a.io;
    const int total = io.chunk_off[a.nel];
    const int G = gridDim.x;
    // A task's inputs arrive through a chain of dependent loads (task ->
    // element offsets -> pair ids -> point coordinates).  The chain of the
    // wave's next task is started level by level while the current one is
    // scored, so that its latency hides behind the MFMA work.
    auto task_of = [&](int t, int &e, int &beg, int &cnt) __attribute__((always_inline)) {
        e = __builtin_amdgcn_readfirstlane(io.task_elem[t]);
        beg = io.elem_off[e] + (t - io.chunk_off[e]) * kChunk;
        cnt = min(io.elem_off[e + 1] - beg, kChunk);
    };
    auto pair_of = [&](int beg, int cnt) __attribute__((always_inline)) { return lane < cnt ? io.list[beg + lane] : 0; };
    // (the primary pass only: its items are the points themselves)
    auto coords_of = [&](int cnt, int item, double (&x)[D]) __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = lane < cnt ? point_coord<D>(a, item, c) : 0.0;
    };
    int t = task_of_block();
    if (t >= total) return;
    int e, beg, cnt;
    task_of(t, e, beg, cnt);
    int item = pair_of(beg, cnt);
    double px[D];
    coords_of(cnt, item, px);
    for (;;) {
        const int tn = t + G;
        const bool more = tn < total;
        int en = 0, begn = 0, cntn = 0;
        if (more) task_of(tn, en, begn, cntn);   // next task, level 1
        double xc[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xc[c] = a.xc[(size_t)e * D + c];
        wave_lds_sync();   // the previous task's reads come first
        // B rows of the element's nodes (FP32; FP64 reads the setup rows)
#pragma unroll 1
        for (int j = lane; L::B_IN_LDS && j < L::NPAD; j += kWave) {
            T b[4] = {T(0), T(0), T(0), T(0)};
            if (j < S::NP) {
                T n2 = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const T v = MIXED ? T(a.nodes32[((size_t)e * D + c) * S::NP + j])
                                      : T(a.nodes[((size_t)e * D + c) * S::NP + j] - xc[c]);
                    b[c] = T(-2) * v;
                    n2 = fma(v, v, n2);
                }
                b[D] = n2;
            } else {
                b[D] = kBig;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) Bt[k * L::NPAD + j] = b[k];
        }
        // A rows of the pairs
        {
            const bool has = lane < cnt;
            items[lane] = item;
            T pa[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < D; ++c) pa[c] = has ? T(px[c] - xc[c]) : T(0);
            pa[D] = T(1);
            T xx = T(0);
#pragma unroll
            for (int c = 0; c < D; ++c) xx = fma(pa[c], pa[c], xx);
#pragma unroll
            for (int k = 0; k < 4; ++k) Pt[k * 64 + lane] = pa[k];
            Xx[lane] = xx;
        }
        wave_lds_sync();
        const int itemn = more ? pair_of(begn, cntn) : 0;   // next task, level 2
        const int ntile = (cnt + 15) >> 4;   // pair tiles of this task (wave-uniform)
        // the start of the pair at task position pl: node bi's reference point
        auto write_start = [&](int bi, int pl) __attribute__((always_inline)) {
            const int it = items[pl];
            const int ii[3] = {bi % N, (bi / N) % N, bi / (N * N)};
#pragma unroll
            for (int k = 0; k < R; ++k) {
                double v = GT.z[0];
#pragma unroll
                for (int m = 1; m < N; ++m)
                    if (ii[k] == m) v = GT.z[m];
                if (io.start)
                    io.start[(size_t)k * io.start_stride + beg + pl] = v;
                else
                    io.r[(size_t)k * io.ostride + it] = v;
            }
        };
        double pxn[D];
        if constexpr (!MIXED) {
            v4 seed[4];
            double av[4], best[4][4];
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) {
                av[pt] = Pt[g * 64 + 16 * pt + col];
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    seed[pt][qq] = Xx[16 * pt + g + 4 * qq];   // pair of output row g + 4 qq
                    best[pt][qq] = __builtin_huge_val();
                }
            }
            // One loop per pair-tile count, free of branches, so that the
            // tiles' MFMAs issue back to back and each result is taken up
            // after the others are issued.  Each lane's B values are loaded
            // four node tiles ahead into four registers, each reloaded right
            // after its tile's MFMAs have read it (no copy at the loop's back
            // edge, which would wait for the load); NT is even, NT >= 2.
            const double *brow = a.near + ((size_t)e * 4 + g) * L::NPAD + col;
            auto scan = [&](auto tiles) __attribute__((always_inline)) {
                constexpr int NTL = decltype(tiles)::value;
                auto tile = [&](int nt, double bv) __attribute__((always_inline)) {
                    if (nt == NT / 2 && more) coords_of(cntn, itemn, pxn);   // next task, level 3
                    const int node = 16 * nt + col;
                    v4 d[NTL];
#pragma unroll
                    for (int pt = 0; pt < NTL; ++pt) d[pt] = mfma16(av[pt], bv, seed[pt]);
#pragma unroll
                    for (int pt = 0; pt < NTL; ++pt)
#pragma unroll
                        for (int qq = 0; qq < 4; ++qq)
                            best[pt][qq] = key_min(best[pt][qq], with_node(d[pt][qq], node));
                };
                constexpr int NT4 = NT & ~3;
                double b0 = brow[0], b1 = brow[16], b2 = 0.0, b3 = 0.0;
                if constexpr (NT > 2) {
                    b2 = brow[32];
                    b3 = brow[48];
                }
                // The reloads are unconditional (past the row's end they read
                // its last tile again), so that the wait before each tile
                // counts on the three loads issued after its own.  Their
                // offsets pass through an empty asm statement: otherwise the
                // compiler proves each reload equal to the next iteration's
                // tile and loads it there, just before its use.
                auto ahead = [&](int t) __attribute__((always_inline)) {
                    int off = 16 * min(t, NT - 1);
                    asm volatile("" : "+s"(off));
                    return brow[off];
                };
#pragma unroll 1
                for (int nt = 0; nt < NT4; nt += 4) {
                    tile(nt, b0);
                    b0 = ahead(nt + 4);
                    tile(nt + 1, b1);
                    b1 = ahead(nt + 5);
                    tile(nt + 2, b2);
                    b2 = ahead(nt + 6);
                    tile(nt + 3, b3);
                    b3 = ahead(nt + 7);
                }
                if constexpr (NT4 < NT) {
                    // the last two tiles (NT = 2 mod 4), in b0 and b1
                    tile(NT4, b0);
                    tile(NT4 + 1, b1);
                }
            };
            switch (ntile) {
            case 1: scan(std::integral_constant<int, 1>()); break;
            case 2: scan(std::integral_constant<int, 2>()); break;
            case 3: scan(std::integral_constant<int, 3>()); break;
            default: scan(std::integral_constant<int, 4>()); break;
            }
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) {
                if (pt >= ntile) break;
#pragma unroll
                for (int o = 1; o < 16; o <<= 1)
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq)
                        best[pt][qq] = key_min(best[pt][qq], __shfl_xor(best[pt][qq], o));
                // lane `col` < 4 writes the pair of output row g + 4 col
                // (the node index is in the low word; masks, not a select
                // chain, which the compiler would turn into a stack array)
                int lo = 0;
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) lo |= __double2loint(best[pt][qq]) & -(col == qq);
                const int pl = 16 * pt + g + 4 * col;
                if (col < 4 && pl < cnt) write_start(lo & ((1 << kNodeBits) - 1), pl);
            }
        } else {
            T av[4], best[4][4];
            int bix[4][4];
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) {
                av[pt] = Pt[g * 64 + 16 * pt + col];
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    best[pt][qq] = T(__builtin_huge_valf());
                    bix[pt][qq] = 0;
                }
            }
            // node tiles outside, pair tiles inside: each B value is read once
            // per task and scores every pair tile; one branch-free loop per
            // pair-tile count, the tiles' MFMAs issued back to back
            auto scan = [&](auto tiles) __attribute__((always_inline)) {
                constexpr int NTL = decltype(tiles)::value;
#pragma unroll 2
                for (int nt = 0; nt < NT; ++nt) {
                    if (nt == NT / 2 && more) coords_of(cntn, itemn, pxn);   // next task, level 3
                    const T bv = Bt[g * L::NPAD + 16 * nt + col];
                    const int node = 16 * nt + col;
                    v4 d[NTL];
#pragma unroll
                    for (int pt = 0; pt < NTL; ++pt) d[pt] = mfma16(av[pt], bv, v4{0, 0, 0, 0});
#pragma unroll
                    for (int pt = 0; pt < NTL; ++pt)
#pragma unroll
                        for (int qq = 0; qq < 4; ++qq) {
                            const bool lt = d[pt][qq] < best[pt][qq];
                            bix[pt][qq] = lt ? node : bix[pt][qq];
                            best[pt][qq] = lt ? d[pt][qq] : best[pt][qq];
                        }
                }
            };
            switch (ntile) {
            case 1: scan(std::integral_constant<int, 1>()); break;
            case 2: scan(std::integral_constant<int, 2>()); break;
            case 3: scan(std::integral_constant<int, 3>()); break;
            default: scan(std::integral_constant<int, 4>()); break;
            }
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) {
                if (pt >= ntile) break;
                // lexicographic (score, node) minimum over the 16 lanes of a row
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const T so = __shfl_xor(best[pt][qq], o);
                        const int io2 = __shfl_xor(bix[pt][qq], o);
                        const bool take =
                            so < best[pt][qq] || (so == best[pt][qq] && io2 < bix[pt][qq]);
                        bix[pt][qq] = take ? io2 : bix[pt][qq];
                        best[pt][qq] = take ? so : best[pt][qq];
                    }
                }
                // lane `col` < 4 writes the pair of its row group held in item qq = col
                int bi = bix[pt][0] * (col == 0) + bix[pt][1] * (col == 1) +
                         bix[pt][2] * (col == 2) + bix[pt][3] * (col == 3);
                const int pl = 16 * pt + 4 * g + col;   // FP32 output layout
                if (col < 4 && pl < cnt) write_start(bi, pl);
            }
        }
        if (!more) break;
        t = tn;
        e = en;
        beg = begn;
        cnt = cntn;
        item = itemn;
#pragma unroll
        for (int c = 0; c < D; ++c) px[c] = pxn[c];
    }
}

// Nearest node of x among the element's nodes staged in LDS (FP64, NodeLds
// layout): the squared distance summed over the coordinates in order, the
// lowest node index among equal distances (Section 3.2.1 starts Newton
// there).  Wave-cooperative: each lane scans every 64th node, then the
// lanes are reduced; every lane returns the index.
template <int D, int R, int N>
__device__ __forceinline__ int nearest_staged(const double *xl, const double (&x)[D], int lane)
{
    double bd = __builtin_huge_val();
    int bi = 0;
    for (int j = lane; j < Shape<D, R, N>::NP; j += kWave) {
        double d2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double t = x[d] - xl[NodeLds<double, D, R, N>::at(d, j / N, j % N)];
            d2 = fma(t, t, d2);
        }
        if (d2 < bd) {
            bd = d2;
            bi = j;
        }
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double od = __shfl_xor(bd, o);
        const int oi = __shfl_xor(bi, o);
        if (od < bd || (od == bd && oi < bi)) {
            bd = od;
            bi = oi;
        }
    }
    return bi;
}

// Reference coordinate k of node `node` (packed index i + N j + N^2 l): the
// GLL point of its k-th index.
template <int N>
__device__ __forceinline__ double node_coord(int node, int k)
{
    constexpr gll::Table<N> GT = gll::Nodes<N>::t;
    const int ik = k == 0 ? node % N : k == 1 ? (node / N) % N : node / (N * N);
    double v = GT.z[0];
#pragma unroll
    for (int m = 1; m < N; ++m)
        if (ik == m) v = GT.z[m];
    return v;
}

// Newton over the element queue in precision T: one wave per element (task
// counter io.counter[8] for the FP64 kernel, [9] for the FP32 phase of mixed
// mode), over the elements that have pairs.  The start of every pair is
// read from io.start (or io.r): the nearest node, or the FP32 result in
// mixed mode.
// TASKS: the waves stride over the 64-pair tasks of io.task_elem instead
// (no counter).  The other candidates of unsettled points are a few pairs
// scattered over many elements; a counter would be stepped once per element
// of the mesh, mostly past empty queues, one same-address atomic after the
// other.  The parked pairs of the face kernel are likewise spread thinly.
// kResolve finds the starts of its pairs itself, from the nodes it stages
// anyway: a separate nearest-node pass would read every such element's
// node data once more for about one pair each, and score that pair on
// matrix tiles of 16.
template <typename T, int D, int R, int N, bool TASKS, int KIND>
__device__ __forceinline__ void newton_body(const NewtonArgs &a)
{
    typedef Shape<D, R, N> S;
    constexpr bool FINAL = std::is_same<T, double>::value;
    extern __shared__ double lds_raw[];
    int *citem = Lds<T, D, R, N>::citem(lds_raw);
    const int lane = threadIdx.x;
    const NewtonIO &io = a.io;
    T *xl = reinterpret_cast<T *>(lds_raw);
    T *tab = xl + Lds<T, D, R, N>::NODES;
    T *cache = tab + 2 * Lds<T, D, R, N>::TAB;
    Counters cn;
    const int total = TASKS ? io.chunk_off[a.nel] : 0;
    int ticket = -1;   // (lane 0) the element counter's value for the next element
    for (int t = TASKS ? task_of_block() : 0;; t += gridDim.x) {
        int e = 0, q0, q1;
        if constexpr (TASKS) {
            if (t >= total) break;
            e = __builtin_amdgcn_readfirstlane(io.task_elem[t]);
            q0 = io.elem_off[e] + (t - io.chunk_off[e]) * kChunk;
            q1 = min(io.elem_off[e + 1], q0 + kChunk);
        } else {
            if (lane == 0) {
                // the element of the ticket taken before, or the next one with
                // a non-empty queue; then the ticket for the wave's next
                // element, taken now so that its atomic completes while this
                // element is staged (every ticket below nel is processed by
                // the wave that took it)
                int *ctr = io.counter + (FINAL ? 8 : 9);
                e = ticket < 0 ? atomicAdd(ctr, 1) : ticket;
                while (e < a.nel && io.elem_off[e + 1] <= io.elem_off[e]) e = atomicAdd(ctr, 1);
                ticket = e < a.nel ? atomicAdd(ctr, 1) : a.nel;
            }
            e = __builtin_amdgcn_readfirstlane(__shfl(e, 0));
            if (e >= a.nel) break;
            q0 = io.elem_off[e];
            q1 = io.elem_off[e + 1];
        }
        __syncthreads();
        if constexpr (FINAL) {
            // kResolve: lane l < q1 - q0 (at most kChunk = 64) loads pair
            // q0 + l (slot id, point) before the nodes are staged
            int it = 0;
            double px[D];
#pragma unroll
            for (int d = 0; d < D; ++d) px[d] = 0.0;
            if constexpr (KIND == kResolve) {
                static_assert(kChunk <= kWave, "one lane per pair of a task");
                if (lane < q1 - q0) {
                    it = io.list[q0 + lane];
                    const int p = io.slot_pt[it];
#pragma unroll
                    for (int d = 0; d < D; ++d) px[d] = point_coord<D>(a, p, d);
                }
            }
            const double *src = a.nodes + (size_t)e * D * S::NP;
            if constexpr (KIND == kResolve) {
                stage_nodes<double, D, R, N>(xl, src, lane);
                for (int j = 0; j < q1 - q0; ++j) {
                    double x[D];
#pragma unroll
                    for (int d = 0; d < D; ++d) x[d] = __shfl(px[d], j);
                    const int bi = nearest_staged<D, R, N>(xl, x, lane);
                    const int itj = __shfl(it, j);
                    if (lane < R) io.r[(size_t)lane * io.ostride + itj] = node_coord<N>(bi, lane);
                }
                // the refill reads the starts back with loads that bypass
                // L1; this wave's stores only have to be complete (a
                // device-scope fence would also write back and invalidate
                // the L2, once per task)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                run_element<double, D, R, N, true, KIND>(a, e, q0, q1, xl, tab, cache, citem,
                                                         lane, a.max_iter, a.tol, nullptr, cn,
                                                         [] {});
            } else if constexpr (KIND == kFace) {
                stage_nodes<double, D, R, N>(xl, src, lane);
                run_element<double, D, R, N, true, KIND>(a, e, q0, q1, xl, tab, cache, citem,
                                                         lane, a.max_iter, a.tol, nullptr, cn,
                                                         [] {});
            } else {
                // the primary and polish passes stage the nodes after their
                // first batch of pairs has been fetched
                run_element<double, D, R, N, true, KIND>(
                    a, e, q0, q1, xl, tab, cache, citem, lane, a.max_iter, a.tol, nullptr, cn,
                    [&] { stage_nodes<double, D, R, N>(xl, src, lane); });
            }
        } else {
            const float *src = a.nodes32 + (size_t)e * D * S::NP;
            run_element<float, D, R, N, false, KIND>(
                a, e, q0, q1, xl, tab, cache, citem, lane, a.max_iter32, a.tol32,
                a.xc + (size_t)e * D, cn, [&] { stage_nodes<float, D, R, N>(xl, src, lane); });
        }
    }
    unsigned long long v[11] = {cn.pairs,  cn.passes,        cn.evals,  cn.evals_h2,
                                cn.passes32, cn.evals32,     cn.evals_h2_exec,
                                cn.sweeps, cn.sweeps_h2, cn.sweeps32, cn.evals32_node};
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        unsigned long long x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0 && x) atomicAdd(&io.stats[k], x);
    }
}

// The primary pass and the pass over the other candidates of unsettled
// points run the same Newton code under two kernel names, so that a kernel
// trace reports them apart (the latter finds its starts itself).
// (at least three waves per SIMD: the register budget then stays within the
// 256 VGPRs, and the compiler gives the MFMA results VGPRs, not AGPRs that
// the selection would first have to copy out)
template <int D, int R, int N, bool MIXED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void
k_nearest(NewtonArgs a)
{
    nearest_body<D, R, N, MIXED>(a);
}
template <int D, int R, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_newton(NewtonArgs a)
{
    newton_body<double, D, R, N, false, kPrimary>(a);
}
template <int D, int R, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_newton_polish(NewtonArgs a)
{
    newton_body<double, D, R, N, false, kPolish>(a);
}
template <int D, int R, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_newton_resolve(NewtonArgs a)
{
    newton_body<double, D, R, N, true, kResolve>(a);
}
template <int D, int R, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_newton_face(NewtonArgs a)
{
    newton_body<double, D, R, N, true, kFace>(a);
}
template <int D, int R, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 3))) void
k_newton32(NewtonArgs a)
{
    newton_body<float, D, R, N, false, kPrimary>(a);
}

// Phase D for the points whose other candidates found no room in the slot
// array (more candidate pairs than the workspace holds): one wavefront per
// point, its other candidates in ascending id order, each started from its
// nearest node (squared distances to every node of the element, ties to the
// lowest index) and iterated by the same code as the pass kernels, on a
// one-pair queue; then the selection rule of Section 3.2 over the primary
// and them.  One pair per wavefront: a path for rare overloads only.
template <int D, int R, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_resolve_overflow(NewtonArgs a, HashView h)
{
    typedef Shape<D, R, N> S;
    extern __shared__ double lds_raw[];
    int *citem = Lds<double, D, R, N>::citem(lds_raw);
    double *xl = lds_raw;
    double *tab = xl + Lds<double, D, R, N>::NODES;
    double *cache = tab + 2 * Lds<double, D, R, N>::TAB;
    const int lane = threadIdx.x, b = blockIdx.x, G = gridDim.x;
    const NewtonIO &io = a.io;
    const int cnt = *io.ocount;
    // this block's one-pair queue: item b of the scratch outputs
    int *ov_item = io.ov_int, *ov_pt = io.ov_int + G, *ov_code = io.ov_int + 2 * G;
    NewtonArgs la = a;
    la.io.list = ov_item;
    la.io.slot_pt = ov_pt;
    la.io.code = ov_code;
    la.io.elem = nullptr;
    la.io.r = io.ov_dbl;
    la.io.ostride = G;
    la.io.dist = io.ov_dbl + (size_t)R * G;
    la.io.start = nullptr;
    la.io.rs = nullptr;
    la.io.conv = nullptr;
    la.io.park_meta = nullptr;
    la.io.polish = 0;
    if (lane == 0) ov_item[b] = b;
    Counters cn;
    for (int i = b; i < cnt; i += G) {
        const int p = io.list[i];
        const int prim = io.cand[p].y, c = io.cellpt[p];
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = point_coord<D>(a, p, d);
        if (lane == 0) ov_pt[b] = p;
        // the primary's result is the best so far
        int bcode = io.code[p], belem = prim;
        double bdist = io.dist[p], br[R];
#pragma unroll
        for (int k = 0; k < R; ++k) br[k] = io.r[(size_t)k * io.ostride + p];
        bool changed = false;
        for (int q = h.cell_off[c]; q < h.cell_off[c + 1]; ++q) {
            const int e = h.cell_el[q];
            double depth;
            if (e == prim || !box_pass<D>(h.box + (size_t)e * (3 * D + D * D), x, depth))
                continue;
            __syncthreads();
            stage_nodes<double, D, R, N>(xl, a.nodes + (size_t)e * D * S::NP, lane);
            const int bi = nearest_staged<D, R, N>(xl, x, lane);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < R; ++k) la.io.r[(size_t)k * G + b] = node_coord<N>(bi, k);
            }
            // lane 0 wrote the queue entry and the start and reads them back
            // in the refill (same lane, program order)
            run_element<double, D, R, N, true, kResolve>(la, e, b, b + 1, xl, tab, cache, citem,
                                                        lane, a.max_iter, a.tol, nullptr, cn,
                                                        [] {});
            // slot 0's leader (lane 0) wrote the result
            int cd = 0;
            double dd = 0.0, rr[R];
            if (lane == 0) {
                cd = ov_code[b];
                dd = la.io.dist[b];
            }
#pragma unroll
            for (int k = 0; k < R; ++k) rr[k] = lane == 0 ? la.io.r[(size_t)k * G + b] : 0.0;
            cd = __shfl(cd, 0);
            dd = __shfl(dd, 0);
#pragma unroll
            for (int k = 0; k < R; ++k) rr[k] = __shfl(rr[k], 0);
            // Section 3.2: the lowest-id INTERIOR candidate, else the
            // smallest distance, the lower id on ties
            bool take;
            if (bcode == FPTS_INTERIOR) take = cd == FPTS_INTERIOR && e < belem;
            else if (cd == FPTS_INTERIOR) take = true;
            else take = dd < bdist || (dd == bdist && e < belem);
            if (take) {
                bcode = cd;
                belem = e;
                bdist = dd;
#pragma unroll
                for (int k = 0; k < R; ++k) br[k] = rr[k];
                changed = true;
            }
        }
        if (lane == 0 && changed) {
            io.code[p] = bcode;
            io.elem[p] = belem;
            io.dist[p] = bdist;
#pragma unroll
            for (int k = 0; k < R; ++k) io.r[(size_t)k * io.ostride + p] = br[k];
        }
    }
    unsigned long long v[11] = {cn.pairs,  cn.passes,        cn.evals,  cn.evals_h2,
                                cn.passes32, cn.evals32,     cn.evals_h2_exec,
                                cn.sweeps, cn.sweeps_h2, cn.sweeps32, cn.evals32_node};
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        unsigned long long xv = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) xv += __shfl_xor(xv, o);
        if (lane == 0 && xv) atomicAdd(&io.stats[k], xv);
    }
}

typedef void (*KernelFn)(NewtonArgs);
typedef void (*OverflowFn)(NewtonArgs, HashView);

struct Kernels {
    KernelFn nearest = nullptr, newton32 = nullptr, newton = nullptr, face = nullptr;
    OverflowFn overflow = nullptr;
    size_t lds_nearest = 0, lds_newton32 = 0, lds_newton = 0;
};

template <int D, int R, bool MIXED>
Kernels pick_kernels(int N, bool resolve)
{
    typedef typename std::conditional<MIXED, float, double>::type TN;
    Kernels k;
#define FPTS_CASE(NN)                                                                       \
    case NN:                                                                                \
        k.nearest = resolve ? nullptr : k_nearest<D, R, NN, MIXED>;                          \
        k.newton = resolve ? k_newton_resolve<D, R, NN> : k_newton<D, R, NN>;               \
        k.face = k_newton_face<D, R, NN>;                                                   \
        k.overflow = k_resolve_overflow<D, R, NN>;                                          \
        if (MIXED && !resolve) {                                                            \
            k.newton32 = k_newton32<D, R, NN>;                                              \
            k.newton = k_newton_polish<D, R, NN>;                                           \
        }                                                                                   \
        k.lds_nearest = NearLds<TN, D, R, NN>::bytes();                                     \
        k.lds_newton32 = Lds<float, D, R, NN>::bytes();                                     \
        k.lds_newton = Lds<double, D, R, NN>::bytes();                                      \
        break;
    switch (N) {
        FPTS_CASE(2)
        FPTS_CASE(3)
        FPTS_CASE(4)
        FPTS_CASE(5)
        FPTS_CASE(6)
        FPTS_CASE(7)
        FPTS_CASE(8)
        FPTS_CASE(9)
        FPTS_CASE(10)
    default:
        break;
    }
#undef FPTS_CASE
    return k;
}

// Launches on the caller's stream: nearest nodes (which & 1; task grid of
// 64-pair tasks over io.chunk_off, io.task_elem; not for the *_resolve
// kernels, which find them from the nodes they stage), then Newton (which & 2; element
// tasks: in mixed mode the FP32 phase, counter io.counter[9], then the FP64
// kernel, counter io.counter[8]); which & 4 runs the face kernel over the
// parked pairs (io.list = park indices binned by element, io.elem_off /
// chunk_off / task_elem their buckets and tasks).  io.counter[0..15] must be
// zero.  A list with io.slot_pt set (other candidates) selects the *_resolve
// kernels, whose Newton strides over the 64-pair tasks like the nearest-node
// kernel.
template <int D, int R>
hipError_t launch_newton_kind(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s)
{
    const bool resolve = io.slot_pt != nullptr;
    const Kernels k = mixed ? pick_kernels<D, R, true>(m->N, resolve)
                            : pick_kernels<D, R, false>(m->N, resolve);
    if ((!k.nearest && !resolve) || !k.newton) return hipErrorInvalidValue;
    NewtonArgs a;
    a.nodes = m->d_nodes;
    a.nodes32 = m->d_nodes32;
    a.near = m->d_near;
    if (m->near_npad != (m->NP + 31) / 32 * 32) return hipErrorInvalidValue;
    a.xc = m->d_xc;
    a.pts = pts;
    a.n = (int)n;
    a.nel = (int)m->nel;
    a.io = io;
    a.max_iter = io.max_iter > 0 ? io.max_iter : m->p.max_iter;
    a.tol = m->p.newton_tol;
    a.eps_d = m->p.surf_eps_d;
    a.max_iter32 = m->p.mixed_max_iter;
    a.tol32 = (float)m->p.mixed_tol;
    // the other candidates' Newton kernel finds their starts itself
    if ((which & 1) && !resolve) {
        hipLaunchKernelGGL(k.nearest, dim3(task_grid(io.task_bound, m->cus)), dim3(64),
                           k.lds_nearest, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (which & 2) {
        if (k.newton32) {
            // three waves per SIMD, as the kernel's register budget allows
            hipLaunchKernelGGL(k.newton32, dim3(m->cus * 12), dim3(64), k.lds_newton32, s, a);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k.newton, dim3(m->cus * 8), dim3(64), k.lds_newton, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (which & 4) {
        if (!k.face) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k.face, dim3(m->cus * 8), dim3(64), k.lds_newton, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (which & 8) {
        // grid = the scratch's block count (io.task_bound)
        if (!k.overflow || io.task_bound < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k.overflow, dim3((unsigned)io.task_bound), dim3(64), k.lds_newton, s,
                           a, hash_view(m));
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace newton
}  // namespace fpts
