// gfx950 kernels of one BP RI-OEDG stage (2D Euler, P1/P2 modal DG on triangles).
//
// Two passes per stage over a state stored as structure-of-arrays, cell
// fastest: cell averages [var][cell] and higher modes [var][mode][cell]:
//   k_residual  volume + edge quadrature of eq. DGSystem:Dis with the LF flux
//               (eq. fluxLF), the diagonal mass and the SSP-RK3 combination (eq.
//               RKTime); writes the pre-filter state and per-workgroup partials of
//               sum |K| ubar_K, of min/max at the volume points and of
//               |m - mbar|^2 there (eq. normOmg; mbar known in advance by
//               conservation, see the pass).
//   k_filter    RIOE damping (eq. oe:sys with eqs. OEScalar:beta, OEScalar:Coef2,
//               oe:sysdelta2, RIOESys:CoefM), the BP limiter at the decomposition
//               nodes (Sec. 4.4) and the max wave speed of the result (eq. 1250);
//               also the momentum bookkeeping of its output for the next residual.
// Each pass is followed by a one-workgroup finalize kernel that reduces the
// partials in a fixed order, so results do not depend on scheduling and no
// workgroup needs a device-scope fence.
//
// Lane layout of the residual and filter passes: the 4 lanes of a DPP quad own
// one cell, lane v holding conservative variable v (rho, m1, m2, E).  A lane
// keeps only its variable's modes in registers; values at a quadrature point are
// exchanged inside the quad with DPP quad_perm moves.  Workgroups are spread so
// that each XCD walks a contiguous range of the (Hilbert-ordered) cells, which
// keeps neighbour gathers inside that XCD's L2.
//
// Precision: every pass is instantiated for a bulk type T, double (FP64) or
// float (mixed).  Cell averages are stored, updated and reduced in FP64 in both
// forms; modes >= 1, the volume and surface quadrature and the OE filter run in
// T.  The BP limiter's point values, theta, the internal energy and the max wave
// speed always run in FP64.  In the mixed form the limited modes are rounded to
// float, so theta aims above the floors by a bound of that rounding, and the
// stored coefficients are checked again: a cell whose stored state still dips
// below half a floor at a node keeps only its average.  The stored state thus
// has rho > 0 and rho e > 0 at every limiter node, evaluated in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "oedg_internal.h"

namespace oedg {
namespace {


template <int K>
struct Rule;

// Volume rules of App. A with (xi, eta) = (b2, b3); edge Gauss nodes on [0, 1]
// (App. B with s = (1 + x)/2) and weights summing to one.
template <>
struct Rule<1> {
    static constexpr int NM = 3, NQ = 3, NE = 2;
    static constexpr double xi[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    static constexpr double eta[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
    static constexpr double w[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};
    static constexpr double s[3] = {0.2113248654051871, 0.7886751345948129, 0.0};
    static constexpr double ws[3] = {0.5, 0.5, 0.0};
};
template <>
struct Rule<2> {
    static constexpr int NM = 6, NQ = 6, NE = 3;
    // (a, a, 1-2a), (a, 1-2a, a), (1-2a, a, a) and the same with b (tab:4th)
    static constexpr double A = 0.4459484909159649, A2 = 0.10810301816807023;
    static constexpr double B = 0.09157621350977074, B2 = 0.8168475729804585;
    static constexpr double WA = 0.22338158967801147, WB = 0.10995174365532187;
    static constexpr double xi[6] = {A, A2, A, B, B2, B};
    static constexpr double eta[6] = {A2, A, A, B2, B, B};
    static constexpr double w[6] = {WA, WA, WA, WB, WB, WB};
    static constexpr double s[3] = {0.11270166537925831, 0.5, 0.8872983346207417};
    static constexpr double ws[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
};

// 1 / (a_K^(l) / |K|) for the orthogonal basis of eq. basisfunc
__device__ constexpr double kInvMass[6] = {1.0, 1.5, 2.0, 15.0 / 16.0, 9.0 / 4.0, 3.0};
// A^{k,j} = (2j+1)/((2k-1) j!)
__device__ constexpr double kA[3][3] = {{0, 0, 0}, {1.0, 3.0, 0.0}, {1.0 / 3.0, 1.0, 5.0 / 6.0}};

constexpr double kEpsOE = 1e-12;
constexpr double kEpsBP = 1e-13;

// Mixed form: rounding theta * c_l to float moves it by at most 2^-24 theta |c_l|,
// and |Psi_l| <= 4 on the reference triangle for every l <= 5, so a point value
// moves by at most 4 * 2^-24 * theta * sum_{l>=1} |c_l|; the limiter aims twice that
// above the floor.
constexpr double kMixMargin = 8.0 * 0x1p-24;

// ------------------------------------------------------------------------- basis

template <int K>
__device__ __forceinline__ void psi(double x, double e, double* p) {
    p[0] = 1.0;
    p[1] = 4.0 * x + 2.0 * e - 2.0;
    p[2] = 3.0 * e - 1.0;
    if constexpr (K == 2) {
        p[3] = 24.0 * x * x + 24.0 * x * e + 4.0 * e * e - 24.0 * x - 8.0 * e + 4.0;
        p[4] = 20.0 * x * e + 10.0 * e * e - 4.0 * x - 12.0 * e + 2.0;
        p[5] = 10.0 * e * e - 8.0 * e + 1.0;
    }
}

// At the reference vertices (0,0), (1,0), (0,1) every basis function and its
// first derivatives are affine in the vertex's coordinates (sx, se) (there
// x^2 = x, e^2 = e, xe = 0).  Returns sum_{l>=1} u_l Psi_l and the reference
// derivatives of sum_l u_l Psi_l at vertex (sx, se).
template <int K, typename T>
__device__ __forceinline__ void vertex_eval(const T* u, T sx, T se, T& qh, T& dx, T& de) {
    if constexpr (K == 1) {
        qh = fma((T)4.0 * u[1], sx, fma((T)2.0 * u[1] + (T)3.0 * u[2], se, (T)-2.0 * u[1] - u[2]));
        dx = (T)4.0 * u[1];
        de = (T)2.0 * u[1] + (T)3.0 * u[2];
    } else {
        const T a = (T)-2.0 * u[1] - u[2] + (T)4.0 * u[3] + (T)2.0 * u[4] + u[5];
        const T b = (T)4.0 * u[1] - (T)4.0 * u[4];
        const T c = (T)2.0 * u[1] + (T)3.0 * u[2] - (T)4.0 * u[3] - (T)2.0 * u[4] + (T)2.0 * u[5];
        qh = fma(b, sx, fma(c, se, a));
        const T ax = (T)4.0 * u[1] - (T)24.0 * u[3] - (T)4.0 * u[4];
        dx = fma((T)48.0 * u[3], sx, fma((T)24.0 * u[3] + (T)20.0 * u[4], se, ax));
        const T ae = (T)2.0 * u[1] + (T)3.0 * u[2] - (T)8.0 * u[3] - (T)12.0 * u[4] - (T)8.0 * u[5];
        const T bc = (T)24.0 * u[3] + (T)20.0 * u[4];
        de = fma(bc, sx, fma((T)8.0 * u[3] + (T)20.0 * u[4] + (T)20.0 * u[5], se, ae));
    }
}

// The restriction of sum_l u_l Psi_l to local edge j (from vertex j+1 to vertex
// j+2, parameter s in [0, 1]) has degree K in s, so it is the Lagrange
// interpolant of its values at the edge's ends (q0 at s = 0, q1 at s = 1) and,
// for K = 2, its midpoint (qm).  The midpoints (1/2,1/2), (0,1/2), (1/2,0) of
// edges 0, 1, 2 give affine forms in the indicators i1 = [j==1], i2 = [j==2].
template <int K, typename T>
__device__ __forceinline__ void edge_trace_nodes(const T* u, int j, T& q0, T& qm, T& q1) {
    const int sv = j == 2 ? 0 : j + 1, ev = j == 0 ? 2 : j - 1;   // (j+1) % 3, (j+2) % 3
    T qh0, qh1, dx, de;
    vertex_eval<K, T>(u, sv == 1 ? (T)1.0 : (T)0.0, sv == 2 ? (T)1.0 : (T)0.0, qh0, dx, de);
    vertex_eval<K, T>(u, ev == 1 ? (T)1.0 : (T)0.0, ev == 2 ? (T)1.0 : (T)0.0, qh1, dx, de);
    q0 = u[0] + qh0;
    q1 = u[0] + qh1;
    qm = (T)0.0;
    if constexpr (K == 2) {
        // Psi_1..5 at the midpoints: edge 0 (1, 1/2, 1, 3/2, -1/2), edge 1 (-1, 1/2,
        // 1, -3/2, -1/2), edge 2 (0, -1, -2, 0, 1)
        const T i1 = j == 1 ? (T)1.0 : (T)0.0, i2 = j == 2 ? (T)1.0 : (T)0.0;
        const T m0 = u[0] + u[1] + (T)0.5 * u[2] + u[3] + (T)1.5 * u[4] - (T)0.5 * u[5];
        const T m1 = (T)-2.0 * u[1] - (T)3.0 * u[4];
        const T m2 = -u[1] - (T)1.5 * u[2] - (T)3.0 * u[3] - (T)1.5 * u[4] + (T)1.5 * u[5];
        qm = fma(i1, m1, fma(i2, m2, m0));
    }
}

// Basis values at the fixed points of a stage, in constant memory: the point loops
// run with a wave-uniform index, so these become scalar loads instead of registers.
template <int K, typename T>
struct Tab {
    static constexpr int NM = Rule<K>::NM, NQ = Rule<K>::NQ, NE = Rule<K>::NE;
    T vp[NQ][NM], vdx[NQ][NM], vde[NQ][NM];   // volume points: Psi, dPsi/dxi, dPsi/deta
    T vw[NQ];                                 // volume weights
    T ep[3 * NE][NM];                         // own edge Gauss points (edge i, node nu)
    T nbw[NE][3];   // Lagrange weights (end 0, midpoint, end 1) of the neighbour's trace at its
                    // parameter 1 - s_nu = s_{NE-1-nu}
    double zr[NM];  // classical decomposition: u* = sum_l zr_l u_l (P2; Sec. 4.4, classical branch)
};

template <typename T>
constexpr void basis_at(int nm, double x, double e, T* p, T* dx, T* de) {
    const double P[6] = {1.0, 4.0 * x + 2.0 * e - 2.0, 3.0 * e - 1.0,
                         24.0 * x * x + 24.0 * x * e + 4.0 * e * e - 24.0 * x - 8.0 * e + 4.0,
                         20.0 * x * e + 10.0 * e * e - 4.0 * x - 12.0 * e + 2.0, 10.0 * e * e - 8.0 * e + 1.0};
    const double X[6] = {0.0, 4.0, 0.0, 48.0 * x + 24.0 * e - 24.0, 20.0 * e - 4.0, 0.0};
    const double E[6] = {0.0, 2.0, 3.0, 24.0 * x + 8.0 * e - 8.0, 20.0 * x + 20.0 * e - 12.0, 20.0 * e - 8.0};
    for (int l = 0; l < nm; ++l) {
        p[l] = (T)P[l];
        dx[l] = (T)X[l];
        de[l] = (T)E[l];
    }
}

template <int K, typename T>
constexpr Tab<K, T> make_tab() {
    using R = Rule<K>;
    Tab<K, T> t{};
    T scratch[6] = {}, scratch2[6] = {};
    for (int m = 0; m < R::NQ; ++m) {
        basis_at<T>(R::NM, R::xi[m], R::eta[m], t.vp[m], t.vdx[m], t.vde[m]);
        t.vw[m] = (T)R::w[m];
    }
    for (int i = 0; i < 3; ++i)
        for (int nu = 0; nu < R::NE; ++nu) {
            const double s = R::s[nu];
            const double x = i == 0 ? 1.0 - s : (i == 1 ? 0.0 : s);
            const double e = i == 0 ? s : (i == 1 ? 1.0 - s : 0.0);
            basis_at<T>(R::NM, x, e, t.ep[i * R::NE + nu], scratch, scratch2);
        }
    // u* = (ubar - sum_i w_i sum_nu w_nu u(x_i,nu)) / (1 - sum_i w_i) with the
    // Zhang-Xia-Shu edge weights w_i = 2 w1^GL / 3, w1^GL = 1/(L(L-1)),
    // L = ceil((k+3)/2) (Sec. 4.2); a linear form in the modes.  P1 has no internal
    // nodes (the edge weights sum to one) and no u*.
    if constexpr (K == 2) {
        constexpr int L = (K + 4) / 2;
        const double wi = 2.0 / (3.0 * L * (L - 1));
        double acc[6] = {};
        double pp[6] = {}, px[6] = {}, pe[6] = {};
        for (int i = 0; i < 3; ++i)
            for (int nu = 0; nu < R::NE; ++nu) {
                const double s = R::s[nu];
                const double x = i == 0 ? 1.0 - s : (i == 1 ? 0.0 : s);
                const double e = i == 0 ? s : (i == 1 ? 1.0 - s : 0.0);
                basis_at<double>(R::NM, x, e, pp, px, pe);
                for (int l = 0; l < R::NM; ++l) acc[l] += wi * R::ws[nu] * pp[l];
            }
        for (int l = 0; l < R::NM; ++l) t.zr[l] = ((l == 0 ? 1.0 : 0.0) - acc[l]) / (1.0 - 3.0 * wi);
    }
    for (int nu = 0; nu < R::NE; ++nu) {
        const double s = R::s[R::NE - 1 - nu];
        t.nbw[nu][0] = (T)(K == 2 ? (1.0 - s) * (1.0 - 2.0 * s) : 1.0 - s);
        t.nbw[nu][1] = (T)(K == 2 ? 4.0 * s * (1.0 - s) : 0.0);
        t.nbw[nu][2] = (T)(K == 2 ? s * (2.0 * s - 1.0) : s);
    }
    return t;
}

__constant__ Tab<1, double> kTab1d = make_tab<1, double>();
__constant__ Tab<2, double> kTab2d = make_tab<2, double>();
__constant__ Tab<1, float> kTab1f = make_tab<1, float>();
__constant__ Tab<2, float> kTab2f = make_tab<2, float>();
template <int K, typename T>
__device__ __forceinline__ const Tab<K, T>& tab() {
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (K == 1) return kTab1f;
        else return kTab2f;
    } else {
        if constexpr (K == 1) return kTab1d;
        else return kTab2d;
    }
}

template <int NM, typename T>
__device__ __forceinline__ T dot(const T* u, const T* p) {
    T s = u[0] * p[0];
#pragma unroll
    for (int l = 1; l < NM; ++l) s = fma(u[l], p[l], s);
    return s;
}
// sum over the modes l >= 1 of |u_l|
template <int NM>
__device__ __forceinline__ double abs_sum_hi(const double* u) {
    double s = fabs(u[1]);
#pragma unroll
    for (int l = 2; l < NM; ++l) s += fabs(u[l]);
    return s;
}

// ------------------------------------------------------------------------- fast arithmetic

// 1/x from v_rcp_f64 and two Newton steps (about 1 ulp; not correctly rounded)
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(x) for x >= 0 from v_rsq_f64, one Goldschmidt step and one Newton
// correction.  v_rsq_f64 is within 2^-23 relative; the Goldschmidt step squares
// that error and the correction squares it again, below the rounding of the last
// FMA, so the result is within 1 ulp (correctly rounded in a 4M-sample check on
// gfx950, where v_rsq_f64 stayed within 2^-24).  Arguments below 1e-300 (zero, and
// NaN) give 1e-150: every use adds the root to O(1) terms or scales a damping rate,
// where that is exactly nothing, and it spares the zero test and its selects.
__device__ __forceinline__ double fsqrt(double x) {
    const double xs = fmax(x, 1e-300);
    const double y = __builtin_amdgcn_rsq(xs);
    double g = xs * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, xs);
    return fma(d, h, g);
}

// reciprocal, square root (0 for x <= 0), exponential and quotient in the bulk type
template <typename T>
struct Fp;
template <>
struct Fp<double> {
    static __device__ __forceinline__ double rcp(double x) { return frcp(x); }
    static __device__ __forceinline__ double sqrt(double x) { return fsqrt(x); }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double div(double x, double y) { return x / y; }
};
template <>
struct Fp<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }   // 1 ulp
    // v_sqrt_f32 itself (1 ulp) instead of the correctly rounded expansion: about 17
    // instructions fewer per call in the mixed OE
    static __device__ __forceinline__ float sqrt(float x) { return x > 0.0f ? __builtin_amdgcn_sqrtf(x) : 0.0f; }
    // 2^(x log2 e) with v_exp_f32: a few ulp, results below the normal range flush to 0
    static __device__ __forceinline__ float exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
    static __device__ __forceinline__ float div(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
};

// ------------------------------------------------------------------------- quad exchanges

// DPP quad_perm move: lane q of every quad receives lane perm[q]'s value (every
// source lane of a quad permutation exists, so the destination's old value is
// never kept and needs no initialisation)
template <int CTRL>
__device__ __forceinline__ double qperm(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float qperm(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}
template <int L, typename T>
__device__ __forceinline__ T qget(T x) { return qperm<L * 0x55>(x); }   // broadcast lane L
template <typename T>
__device__ __forceinline__ T qswap12(T x) { return qperm<0xD8>(x); }   // [0,2,1,3]
template <typename T>
__device__ __forceinline__ T qxor1(T x) { return qperm<0xB1>(x); }     // [1,0,3,2]
template <typename T>
__device__ __forceinline__ T qxor2(T x) { return qperm<0x4E>(x); }     // [2,3,0,1]
template <typename T>
__device__ __forceinline__ T qmax(T x) {
    x = fmax(x, qxor1(x));
    return fmax(x, qxor2(x));
}
template <typename T>
__device__ __forceinline__ T qmin(T x) {
    x = fmin(x, qxor1(x));
    return fmin(x, qxor2(x));
}
// 4x4 transpose inside a quad through LDS: lane w holds x[c] = (its variable w at
// state c); on return q[w] = variable w at state v, where v is the calling lane.
// Each lane stores its four entries and reads the four it needs (8 LDS operations
// instead of three quad rotations and their select chains).
// Layout [entry][thread] keeps both the stores and the loads free of bank
// conflicts; LDS executes a wave's operations in order, and the wave barriers keep
// the compiler from moving the loads above the stores or the next stores above
// these loads.
template <typename T>
__device__ __forceinline__ void quad_transpose(int v, const T (&x)[4], T (&q)[4]) {
    __shared__ T buf[4][kBlock];
    const int t = threadIdx.x, quad = t & ~3;
#pragma unroll
    for (int c = 0; c < 4; ++c) buf[c][t] = x[c];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int w = 0; w < 4; ++w) q[w] = buf[v][quad + w];
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------------- Euler

// component v of F(q).n for the lane's variable; (nx, ny) may be a scaled normal,
// sn is the lane's component of it (nx on lane 1, ny on lane 2, else 0) and
// s3 = [v == 3]
template <typename T>
__device__ __forceinline__ T lane_flux(T qv, T q0, T q1, T q2, T q3, T nx, T ny, T gm1, T sn, T s3) {
    const T ir = Fp<T>::rcp(q0);
    const T mn = q1 * nx + q2 * ny;
    const T vn = mn * ir;
    const T p = gm1 * (q3 - (T)0.5 * (q1 * q1 + q2 * q2) * ir);
    return qv * vn + p * (sn + s3 * vn);
}

// spectral radius |v.n| + c of F'(u).n (Example ex:euler); guarded so that a
// pre-limiter state with rho <= 0 or p < 0 still gives a finite value
template <typename T>
__device__ __forceinline__ T spectral_radius(T q0, T q1, T q2, T q3, T nx, T ny, T gamma) {
    const T ir = Fp<T>::rcp(fmax(q0, (T)kEpsBP));
    const T p = (gamma - (T)1.0) * (q3 - (T)0.5 * (q1 * q1 + q2 * q2) * ir);
    return fabs(q1 * nx + q2 * ny) * ir + Fp<T>::sqrt(gamma * fmax(p, (T)0.0) * ir);
}

// ------------------------------------------------------------------------- work distribution

// Workgroup b of a pass with G workgroups (G a multiple of 8) runs on XCD b % 8;
// XCD x owns the contiguous tile range [x T, (x+1) T), T = ceil(n_tiles / 8), which
// its G/8 workgroups walk in dispatch order.
struct TileWalk {
    int first, end, stride;
};
__device__ __forceinline__ TileWalk tile_walk(int n_tiles) {
    const int per_x = gridDim.x >> 3;
    const int x = blockIdx.x & 7, r = blockIdx.x >> 3;
    const int T = (n_tiles + 7) >> 3;
    const int lo = x * T;
    return {lo + r, min(lo + T, n_tiles), per_x};
}

// The batched passes: XCD x owns the chunk range [cs.b[x], cs.b[x+1]) (ranges of
// equal estimated cost over the instances' cells in order).
__device__ __forceinline__ TileWalk chunk_walk(const ChunkSplit& cs) {
    const int per_x = gridDim.x >> 3;
    const int x = blockIdx.x & 7, r = blockIdx.x >> 3;
    return {cs.b[x] + r, cs.b[x + 1], per_x};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Addresses of variable v in a state view: its FP64 average and its higher modes
// (mode l at hi[(l - 1) * n_cell]).  The FP64 form is the plain [var][mode][cell]
// array, so its higher modes follow the average at a fixed offset.
template <int NM, typename T>
struct VarPtr {
    double* avg;
    T* hi;
};
template <int NM, typename T>
__device__ __forceinline__ VarPtr<NM, T> var_ptr(const StateView& sv, const StageArgs& a, int v, size_t snc) {
    if constexpr (std::is_same<T, double>::value) {
        double* av = sv.avg + (size_t)v * NM * snc;
        return {av, av + snc};
    } else {
        return {sv.avg + v * a.avs, (T*)sv.hi + v * a.hvs};
    }
}

// a wave-uniform double moved to scalar registers
__device__ __forceinline__ double uniform(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

// ------------------------------------------------------------------------- pass 1: residual

// Reduces the lanes' (sum |K| ubar, min, max) over the workgroup, per variable, and
// writes entry t = 4 k + v (k: sum, min, max) to dst[t * stride].  `pacc` holds the
// count of inadmissible averages on lane 0 of each quad and the max of |m - mbar|^2
// on lane 1; they go to dst[kColBad * stride] and dst[kNumPartial * stride].
__device__ __forceinline__ void residual_flush(double psum, double pmin, double pmax, double pacc, double* dst,
                                               size_t stride) {
    const int v = threadIdx.x & 3;
    double nbad = v == 0 ? pacc : 0.0, pnm = v == 1 ? pacc : 0.0;
    // over the lanes holding the same variable (xor of lane ids >= 4), then waves
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) {
        psum += __shfl_xor(psum, o, 64);
        pmin = fmin(pmin, __shfl_xor(pmin, o, 64));
        pmax = fmax(pmax, __shfl_xor(pmax, o, 64));
    }
    nbad = wave_sum(nbad);
    pnm = wave_max(pnm);
    __shared__ double lds[kBlock / 64][3][4];
    __shared__ double lds_bad[kBlock / 64][2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane < 4) {
        lds[wid][0][lane] = psum;
        lds[wid][1][lane] = pmin;
        lds[wid][2][lane] = pmax;
    }
    if (lane == 0) {
        lds_bad[wid][0] = nbad;
        lds_bad[wid][1] = pnm;
    }
    __syncthreads();
    if (threadIdx.x < kNumPartial) {
        const int k = threadIdx.x >> 2, vv = threadIdx.x & 3;
        double acc = lds[0][k][vv];
        for (int w2 = 1; w2 < kBlock / 64; ++w2) {
            const double x = lds[w2][k][vv];
            acc = k == 0 ? acc + x : (k == 1 ? fmin(acc, x) : fmax(acc, x));
        }
        dst[(size_t)threadIdx.x * stride] = acc;
    } else if (threadIdx.x == kNumPartial) {
        double acc = lds_bad[0][0];
        for (int w2 = 1; w2 < kBlock / 64; ++w2) acc += lds_bad[w2][0];
        dst[(size_t)kColBad * stride] = acc;
    } else if (threadIdx.x == kNumPartial + 1) {
        double acc = lds_bad[0][1];
        for (int w2 = 1; w2 < kBlock / 64; ++w2) acc = fmax(acc, lds_bad[w2][1]);
        dst[(size_t)kNumPartial * stride] = acc;
    }
}

// Per-lane accumulators of the filter pass: the max wave speed, counts and sum
// |K| ubar of the lane's variable in registers; the boundary momentum flux A_1,
// A_2, B_1, B_2 at the lane's edge points (rarely touched) in LDS, one slot per
// thread, so that it holds no register through the OE.
struct FilterAcc {
    double amax = 0.0, n_lim = 0.0, n_bad = 0.0, n_flat = 0.0, msum = 0.0;
};
constexpr int kBookCols = 4;

// Reduces the lanes' accumulators over the workgroup and writes entry k to
// dst[k * stride]: max wave speed, limited, bad and flattened counts, sum |K| m1bar,
// sum |K| m2bar, A_1, A_2, B_1, B_2.
__device__ __forceinline__ void filter_flush(const FilterAcc& f, const double (&book)[kBookCols][kBlock], double* dst,
                                             size_t stride) {
    const int v = threadIdx.x & 3, t = threadIdx.x;
    double x[kFilterCols] = {f.amax, f.n_lim, f.n_bad, f.n_flat, v == 1 ? f.msum : 0.0,
                             v == 2 ? f.msum : 0.0, book[0][t], book[1][t], book[2][t], book[3][t]};
    x[0] = wave_max(x[0]);
#pragma unroll
    for (int k = 1; k < kFilterCols; ++k) x[k] = wave_sum(x[k]);
    __shared__ double lds[kBlock / 64][kFilterCols];
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < kFilterCols; ++k) lds[threadIdx.x >> 6][k] = x[k];
    }
    __syncthreads();
    if (threadIdx.x < kFilterCols) {
        const int k = threadIdx.x;
        double acc = lds[0][k];
        for (int w2 = 1; w2 < kBlock / 64; ++w2) acc = k == 0 ? fmax(acc, lds[w2][k]) : acc + lds[w2][k];
        dst[(size_t)k * stride] = acc;
    }
}

// Batched passes: workgroup b walks its XCD's range of the chunk table; each
// chunk is a run of reduction groups [g0, g1) of instance desc[chunk.inst], given
// to run(a, g0, g1).
template <typename F>
__device__ __forceinline__ void for_each_chunk(const StageArgs* desc, const Chunk* chunks, const ChunkSplit& cs,
                                               F run) {
    const TileWalk w = chunk_walk(cs);
    for (int ci = w.first; ci < w.end; ci += w.stride) {
        const Chunk ch = chunks[ci];
        const StageArgs& a = desc[ch.inst];
        if (!a.g->active || a.g->skip) continue;
        run(a, ch.g0, ch.g1);
    }
}

template <int K, typename T, bool kBatch>
__device__ __forceinline__ void residual_run(const StageArgs& a, int g0, int g1) {
    using R = Rule<K>;
    constexpr int NM = R::NM;
    const Glob* g = a.g;
    const int nc = a.m.n_cell;
    const size_t snc = (size_t)nc;
    const int v = threadIdx.x & 3;
    const T s3 = v == 3 ? 1.0 : 0.0;
    const T gm1 = (T)(a.gamma - 1.0);
    const double alpha = g->alpha, dt = g->dt;
    const double sa = a.stage == 0 ? 0.0 : (a.stage == 1 ? 0.75 : 1.0 / 3.0);
    const double sb = a.stage == 0 ? 1.0 : (a.stage == 1 ? 0.25 : 2.0 / 3.0);
    // this lane's variable: FP64 average and bulk-type higher modes
    const VarPtr<NM, T> up = var_ptr<NM, T>(a.uin, a, v, snc);
    const VarPtr<NM, T> u0p = var_ptr<NM, T>(a.u0, a, v, snc);
    const VarPtr<NM, T> wp = var_ptr<NM, T>(a.w, a, v, snc);
    const double* ua_p = up.avg;
    const T* uh_p = up.hi;
    const double* u0a_p = u0p.avg;
    const T* u0h_p = u0p.hi;
    double* wa_p = wp.avg;
    T* wh_p = wp.hi;
    const Tab<K, T>& TB = tab<K, T>();
    // The domain average of the momentum of the state this pass writes, known before
    // it is written: the discrete divergence form conserves sum_K |K| ubar_K up to
    // the flux through the boundary (each interior edge's flux enters its two cells
    // with opposite signs), so
    //   sum |K| mbar(w) = sa sum |K| mbar(u^n) + sb (sum |K| mbar(u_in) - dt (A + alpha B))
    // with the sums and the boundary flux A + alpha B of the inputs recorded by the
    // filter pass that produced them (sa = 0, sb = 1 in the first stage).  The pass
    // then forms ||| m - mbar |||_inf of eq. normOmg at its own volume points, which
    // saves a pass over the state; the result equals the direct average up to the
    // rounding of the interior fluxes' cancellation.
    // mbar is wave-uniform: moved to scalar registers, it holds no vector register
    // through the flux loops
    double mb[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const bool first = a.stage == 0;
        const double s_in = first ? g->mom_n[j] : g->mom_c[j];
        const double b_in = first ? g->bfa_n[j] + alpha * g->bfb_n[j] : g->bfa_c[j] + alpha * g->bfb_c[j];
        const double s_w = s_in - dt * b_in;
        mb[j] = uniform((first ? s_w : sa * g->mom_n[j] + sb * s_w) / g->area_sum);
    }

    // one cell, owned by a quad of lanes: residual, SSP combination, partials
    // pacc: lane 0 counts inadmissible averages, lane 1 keeps the max of |m - mbar|^2
    auto cell = [&](int c, double& psum, double& pmin, double& pmax, double& pacc) __attribute__((always_inline)) {
        const double ua = ua_p[c];
        T u[NM];
        u[0] = (T)ua;
#pragma unroll
        for (int l = 1; l < NM; ++l) u[l] = uh_p[(l - 1) * snc + c];
        const T xx = (T)a.m.jinv[c], xy = (T)a.m.jinv[snc + c];
        const T ex = (T)a.m.jinv[2 * snc + c], ey = (T)a.m.jinv[3 * snc + c];
        const double area = a.m.area[c];
        const T areaT = (T)area;
        // edge links and lengths with the cell's own data, so that each edge's
        // neighbour loads issue at once (holding a neighbour ahead of its use costs
        // occupancy and measured slower); at a transmissive boundary the own cell is
        // fetched and not used
        int lk[3];
        double ln[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lk[i] = a.m.link[i * snc + c];
            ln[i] = a.m.len[i * snc + c];
        }
        auto fetch = [&](int link, T (&d)[NM]) __attribute__((always_inline)) {
            const int nb = link >= 0 ? (link >> 2) : c;
            d[0] = (T)ua_p[nb];
#pragma unroll
            for (int l = 1; l < NM; ++l) d[l] = uh_p[(l - 1) * snc + nb];
        };

        // mode 0 accumulates in FP64 in both forms (its volume term is zero)
        double r0 = 0.0;
        T r[NM];
#pragma unroll
        for (int l = 0; l < NM; ++l) r[l] = (T)0.0;

        // volume term |K| sum_mu w_mu F(u).grad Psi_l with grad Psi = J^{-T} grad_ref Psi,
        // i.e. dPsi/dxi (F.grad xi) + dPsi/deta (F.grad eta)
#pragma unroll
        for (int m = 0; m < R::NQ; ++m) {
            const T* p = TB.vp[m];
            const T* dx = TB.vdx[m];
            const T* de = TB.vde[m];
            const T qv = dot<NM>(u, p);
            const T q0 = qget<0>(qv), q1 = qget<1>(qv), q2 = qget<2>(qv), q3 = qget<3>(qv);
            const T wa = TB.vw[m] * areaT;
            const T g1 = wa * lane_flux(qv, q0, q1, q2, q3, xx, xy, gm1, v == 1 ? xx : (v == 2 ? xy : (T)0.0), s3);
            const T g2 = wa * lane_flux(qv, q0, q1, q2, q3, ex, ey, gm1, v == 1 ? ex : (v == 2 ? ey : (T)0.0), s3);
#pragma unroll
            for (int l = 1; l < NM; ++l) r[l] = fma(dx[l], g1, fma(de[l], g2, r[l]));
        }

        // surface term - sum_i l_i sum_nu w_nu Fhat(u_int, u_ext, n_i) Psi_l; the scaled
        // normal l_i n_i equals -2|K| grad(lambda_i) of the barycentric coordinate
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
            const T gx = i == 0 ? -(xx + ex) : (i == 1 ? xx : ex);
            const T gy = i == 0 ? -(xy + ey) : (i == 1 ? xy : ey);
            const T lnx = (T)-2.0 * areaT * gx, lny = (T)-2.0 * areaT * gy;
            const T sn = v == 1 ? lnx : (v == 2 ? lny : (T)0.0);   // the lane's normal component
            const T al = (T)(alpha * (i == 0 ? ln[0] : (i == 1 ? ln[1] : ln[2])));
            const int link = i == 0 ? lk[0] : (i == 1 ? lk[1] : lk[2]);
            const bool has = link >= 0;
            const bool wall = link == kLinkWall;
            const int j = link & 3;
            T un[NM];
            fetch(link, un);
            // the exterior trace from its ends and midpoint: the neighbour's along its
            // local edge j, or at a reflective wall the mirrored own trace
            const bool ext = has || wall;
            T n0 = (T)0.0, nm = (T)0.0, n1 = (T)0.0;
            if (ext) edge_trace_nodes<K, T>(un, has ? j : i, n0, nm, n1);
            if (wall) {
                // reflective wall (un holds the own cell): the exterior trace is the own
                // trace with its normal momentum reversed, m - 2 (m.n) n, again of degree
                // K along the edge; its end and midpoint values stand in for the
                // neighbour's, ends swapped (the neighbour's parameter runs the other way)
                const T il = (T)frcp(i == 0 ? ln[0] : (i == 1 ? ln[1] : ln[2]));
                const T nxu = lnx * il, nyu = lny * il;
                const T cn = (T)-2.0 * (sn * il);   // this lane's share of -2n
                const T b0 = fma(cn, fma(qget<1>(n1), nxu, qget<2>(n1) * nyu), n1);
                const T bm = fma(cn, fma(qget<1>(nm), nxu, qget<2>(nm) * nyu), nm);
                const T b1 = fma(cn, fma(qget<1>(n0), nxu, qget<2>(n0) * nyu), n0);
                n0 = b0;
                nm = bm;
                n1 = b1;
            }
#pragma unroll
            for (int nu = 0; nu < R::NE; ++nu) {
                const T* p = TB.ep[i * R::NE + nu];
                const T wsn = (T)(nu == 0 ? R::ws[0] : (nu == 1 ? R::ws[1] : R::ws[2]));
                const T qi = dot<NM>(u, p);
                T qe = qi;
                if (ext) {
                    // the neighbour runs the shared edge the other way: its parameter is
                    // 1 - s_nu = s_{NE-1-nu} (symmetric Gauss nodes)
                    const T* lw = TB.nbw[nu];
                    qe = fma(lw[0], n0, fma(lw[1], nm, lw[2] * n1));
                }
                const T fi = lane_flux(qi, qget<0>(qi), qget<1>(qi), qget<2>(qi), qget<3>(qi), lnx, lny, gm1, sn, s3);
                const T fe = lane_flux(qe, qget<0>(qe), qget<1>(qe), qget<2>(qe), qget<3>(qe), lnx, lny, gm1, sn, s3);
                const T fh = wsn * (T)0.5 * (fi + fe - al * (qe - qi));
                r0 -= (double)fh;
#pragma unroll
                for (int l = 1; l < NM; ++l) r[l] = fma(-fh, p[l], r[l]);
            }
        }

        // diagonal mass a_K^(l) = |K| (a_l/|K|), then the SSP-RK3 combination; the
        // average in FP64, the higher modes in the bulk type
        const double ia = frcp(area);
        const double adv0 = ua + dt * (r0 * ia * kInvMass[0]);
        const double w0 = a.stage == 0 ? adv0 : sa * u0a_p[c] + sb * adv0;
        wa_p[c] = w0;
        if (a.bp_enable) {
            // the OE filter and the limiter keep every average: an inadmissible one
            // here ends the step's attempt (it is retried with half the time step)
            const double q0 = qget<0>(w0), q1 = qget<1>(w0), q2 = qget<2>(w0), q3 = qget<3>(w0);
            if (v == 0 && !(q0 > 0.0 && q3 - 0.5 * (q1 * q1 + q2 * q2) / q0 > 0.0)) pacc += 1.0;
        }
        const T iaT = (T)ia, dtT = (T)dt, saT = (T)sa, sbT = (T)sb;
        T w[NM];
        w[0] = (T)w0;
#pragma unroll
        for (int l = 1; l < NM; ++l) {
            const T adv = u[l] + dtT * (r[l] * iaT * (T)kInvMass[l]);
            w[l] = a.stage == 0 ? adv : saT * u0h_p[(l - 1) * snc + c] + sbT * adv;
            wh_p[(l - 1) * snc + c] = w[l];
        }
        psum += area * w0;
        // |m - mbar|^2 at the volume points, in the bulk type like the point values
        const T mb0 = (T)mb[0], mb1 = (T)mb[1];
        T cnm = (T)0.0;
#pragma unroll 1
        for (int m = 0; m < R::NQ; ++m) {
            const T qt = dot<NM>(w, TB.vp[m]);
            const double q = (double)qt;
            pmin = fmin(pmin, q);
            pmax = fmax(pmax, q);
            const T d1 = qget<1>(qt) - mb0, d2 = qget<2>(qt) - mb1;
            cnm = fmax(cnm, fma(d1, d1, d2 * d2));
        }
        pacc = v == 1 ? fmax(pacc, (double)cnm) : pacc;
    };
    if constexpr (!kBatch) {
        double psum = 0.0, pmin = INFINITY, pmax = -INFINITY, pacc = 0.0;
        const TileWalk tw = tile_walk((nc + kCellsPerTile - 1) / kCellsPerTile);
        for (int tile = tw.first; tile < tw.end; tile += tw.stride) {
            const int c = tile * kCellsPerTile + (threadIdx.x >> 2);
            if (c < nc) cell(c, psum, pmin, pmax, pacc);   // whole quad
        }
        residual_flush(psum, pmin, pmax, pacc, a.part + blockIdx.x, kMaxBlocks);
    } else {
        for (int gi = g0; gi < g1; ++gi) {
            double psum = 0.0, pmin = INFINITY, pmax = -INFINITY, pacc = 0.0;
#pragma unroll 1
            for (int tile = 0; tile < kGroupCells / kCellsPerTile; ++tile) {
                const int c = gi * kGroupCells + tile * kCellsPerTile + (threadIdx.x >> 2);
                if (c < nc) cell(c, psum, pmin, pmax, pacc);
            }
            residual_flush(psum, pmin, pmax, pacc, a.part + a.gbase + gi, a.gstride);
            __syncthreads();   // the flush's LDS is reused by the next group
        }
    }
}

template <int K, typename T>
__global__ __launch_bounds__(kBlock) void k_residual(StageArgs a) {
    if (!a.g->active || a.g->skip) return;
    residual_run<K, T, false>(a, 0, 0);
}
// KM: degrees present in the launch (1: P1, 2: P2, 3: both)
template <int KM, typename T>
__global__ __launch_bounds__(kBlock) void k_residual_batch(const StageArgs* desc, const Chunk* chunks, ChunkSplit cs) {
    for_each_chunk(desc, chunks, cs, [](const StageArgs& a, int g0, int g1) {
        if constexpr (KM != 3) residual_run<KM, T, true>(a, g0, g1);
        else if (a.k == 1) residual_run<1, T, true>(a, g0, g1);
        else residual_run<2, T, true>(a, g0, g1);
    });
}

// ------------------------------------------------------------------------- pass 2: OE, limiter, alpha

// P2 physical Hessian (xx, xy, yy) of one variable with modes u[0..5] (constant per cell)
template <typename T>
__device__ __forceinline__ void hessian(const T* u, T xx, T xy, T ex, T ey, T* h) {
    const T hxx = (T)48.0 * u[3];
    const T hxe = (T)24.0 * u[3] + (T)20.0 * u[4];
    const T hee = (T)8.0 * u[3] + (T)20.0 * u[4] + (T)20.0 * u[5];
    h[0] = hxx * xx * xx + (T)2.0 * hxe * xx * ex + hee * ex * ex;
    h[1] = hxx * xx * xy + hxe * (xx * ey + xy * ex) + hee * ex * ey;
    h[2] = hxx * xy * xy + (T)2.0 * hxe * xy * ey + hee * ey * ey;
}

// rho e = E - |m|^2 / (2 rho) of a point value
__device__ __forceinline__ double internal_energy(const double (&q)[4]) {
    return q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) * frcp(q[0]);
}

// The full state (all four variables, FP64) at this lane's limiter points t = v,
// v+4, v+8 of the NP-point node set.  Each lane evaluates its own variable (average
// wa, modes w) at every point of the set, with wave-uniform basis rows for the edge
// points, and three quad transposes then hand lane v the four variables at its
// points; no lane holds the whole cell's coefficients.  Classical decomposition
// (zxs): the two extra slots repeat edge points 0 and 1 (P1: no internal nodes) or
// hold u* (P2), which leaves every minimum over the set unchanged.  The u* form of
// the optimal decomposition (ustar, P2) holds u* = the mean of its two internal
// nodes (equal node weights) in both slots.
template <int K, int NM, typename T>
__device__ __forceinline__ void node_values_t(int v, double wa, const T (&w)[NM], double n0x, double n0e,
                                              double n1x, double n1e, bool zxs, bool ustar, double (&pv)[3][4]) {
    constexpr int NE3 = 3 * Rule<K>::NE, NP = NE3 + 2;
    const Tab<K, double>& TD = tab<K, double>();
    double wd[NM];
    wd[0] = wa;
#pragma unroll
    for (int l = 1; l < NM; ++l) wd[l] = (double)w[l];
    double y[12];
#pragma unroll
    for (int t = 0; t < NE3; ++t) y[t] = dot<NM>(wd, TD.ep[t]);   // edge i = t / NE, node nu = t % NE
    if (zxs) {
        if constexpr (K == 1) {
            y[NE3] = y[0];
            y[NE3 + 1] = y[1];
        } else {
            y[NE3] = dot<NM>(wd, TD.zr);
            y[NE3 + 1] = y[NE3];
        }
    } else {
        double p[NM];
        psi<K>(n0x, n0e, p);
        y[NE3] = dot<NM>(wd, p);
        psi<K>(n1x, n1e, p);
        y[NE3 + 1] = dot<NM>(wd, p);
        if constexpr (K == 2) {
            if (ustar) y[NE3] = y[NE3 + 1] = 0.5 * (y[NE3] + y[NE3 + 1]);
        }
    }
#pragma unroll
    for (int t = NP; t < 12; ++t) y[t] = y[0];   // slots past the set (not used)
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const double x[4] = {y[4 * kk], y[4 * kk + 1], y[4 * kk + 2], y[4 * kk + 3]};
        quad_transpose(v, x, pv[kk]);
    }
}

template <int K, typename T, bool kBatch>
__device__ __forceinline__ void filter_run(const StageArgs& a, int g0, int g1) {
    using R = Rule<K>;
    using F = Fp<T>;
    constexpr int NM = R::NM;
    constexpr int NE = R::NE;
    constexpr int NP = 3 * NE + 2;   // limiter node set size
    constexpr bool kMixed = std::is_same<T, float>::value;
    const Glob* g = a.g;
    const int nc = a.m.n_cell;
    const size_t snc = (size_t)nc;
    const double gamma = a.gamma;
    const T gammaT = (T)gamma;
    const int v = threadIdx.x & 3;
    const bool oe = a.oe_enable && a.stage >= 0;
    const bool ri = a.oe_mode == 0;
    const T dt = (T)g->dt;
    // inverse L-infinity norm of this lane's quantity (0 in the zero branch)
    const T inv_my =
        (T)(v == 0 ? g->inv_nrm[0] : (v == 3 ? g->inv_nrm[3] : (ri ? g->inv_nrm_m : g->inv_nrm[v])));
    const VarPtr<NM, T> wp = var_ptr<NM, T>(a.w, a, v, snc);
    const VarPtr<NM, T> op = var_ptr<NM, T>(a.uout, a, v, snc);
    const double* wa_p = wp.avg;
    const T* wh_p = wp.hi;
    double* oa_p = op.avg;
    T* oh_p = op.hi;
    const Tab<K, T>& TB = tab<K, T>();
    __shared__ double book[kBookCols][kBlock];   // the output's momentum bookkeeping (FilterAcc)

    // one cell, owned by a quad of lanes: OE, limiter, wave speed of the result
    auto cell = [&](int c, FilterAcc& f) __attribute__((always_inline)) {
        const double wa = wa_p[c];   // the average: untouched by the OE (eq. OE:m0) and the limiter
        T w[NM];
        w[0] = (T)wa;
#pragma unroll
        for (int l = 1; l < NM; ++l) w[l] = wh_p[(l - 1) * snc + c];
        int lk[3];   // edge links, loaded with the cell's own data (one round trip less per edge)
#pragma unroll
        for (int i = 0; i < 3; ++i) lk[i] = a.m.link[i * snc + c];
        const T xx = (T)a.m.jinv[c], xy = (T)a.m.jinv[snc + c];
        const T ex = (T)a.m.jinv[2 * snc + c], ey = (T)a.m.jinv[3 * snc + c];
        const double area_d = a.m.area[c];
        const T area = (T)area_d;
        // unit outward normals n_i = l_i n_i / l_i with l_i n_i = -2|K| grad(lambda_i)
        T nxs[3], nys[3], ils[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T gx = i == 0 ? -(xx + ex) : (i == 1 ? xx : ex);
            const T gy = i == 0 ? -(xy + ey) : (i == 1 ? xy : ey);
            ils[i] = F::rcp((T)a.m.len[i * snc + c]);
            nxs[i] = (T)-2.0 * area * gx * ils[i];
            nys[i] = (T)-2.0 * area * gy * ils[i];
        }

        if (oe) {
            T sig[K + 1];
#pragma unroll
            for (int jj = 0; jj <= K; ++jj) sig[jj] = (T)0.0;
            T ho[3] = {(T)0.0, (T)0.0, (T)0.0};
            if constexpr (K == 2) hessian(w, xx, xy, ex, ey, ho);
            // own value (higher modes) and reference gradient at the three vertices
            T oh[3], ox[3], oe[3];
#pragma unroll
            for (int vt = 0; vt < 3; ++vt)
                vertex_eval<K, T>(w, vt == 1 ? (T)1.0 : (T)0.0, vt == 2 ? (T)1.0 : (T)0.0, oh[vt], ox[vt], oe[vt]);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int link = lk[i];
                if (link < 0) continue;   // transmissive boundary: zero jump (whole quad)
                const int nb = link >> 2, j = link & 3;
                const double wna = wa_p[nb];
                T wn[NM];
                wn[0] = (T)wna;
#pragma unroll
                for (int l = 1; l < NM; ++l) wn[l] = wh_p[(l - 1) * snc + nb];
                const T nxx = (T)a.m.jinv[nb], nxy = (T)a.m.jinv[snc + nb];
                const T nex = (T)a.m.jinv[2 * snc + nb], ney = (T)a.m.jinv[3 * snc + nb];
                const T nx = i == 0 ? nxs[0] : (i == 1 ? nxs[1] : nxs[2]);
                const T ny = i == 0 ? nys[0] : (i == 1 ? nys[1] : nys[2]);
                const T h = (T)2.0 * area * (i == 0 ? ils[0] : (i == 1 ? ils[1] : ils[2]));
                // momentum lanes see m_n = m.n (lane 1) and m_t = m.(-n_y, n_x) (lane 2)
                const T ca = (ri && (v == 1 || v == 2)) ? nx : (T)1.0;
                const T cb = ri ? (v == 1 ? ny : (v == 2 ? -ny : (T)0.0)) : (T)0.0;
                T S[K + 1];
#pragma unroll
                for (int jj = 0; jj <= K; ++jj) S[jj] = (T)0.0;
                T xs[4];   // own variable at: own end 0, neighbour end 0, own end 1, neighbour end 1
#pragma unroll
                for (int end = 0; end < 2; ++end) {
                    // own vertex i+1 (then i+2) meets the neighbour's vertex j+2 (then j+1)
                    const int ov = (i + 1 + end) % 3, nv = (j + 2 - end) % 3;
                    T q, r, jv;
                    // the neighbour's vertex nv, a per-lane index: closed form
                    T rh, tx, te;
                    vertex_eval<K, T>(wn, nv == 1 ? (T)1.0 : (T)0.0, nv == 2 ? (T)1.0 : (T)0.0, rh, tx, te);
                    const T qh = oh[ov];
                    q = w[0] + qh;
                    r = wn[0] + rh;
                    if constexpr (kMixed) {
                        // value jump from the FP64 averages plus the float higher modes
                        jv = (T)(wna - wa) + (rh - qh);
                    } else {
                        jv = r - q;
                    }
                    const T sx = ox[ov], se = oe[ov];
                    const T qx = sx * xx + se * ex, qy = sx * xy + se * ey;
                    const T rx = tx * nxx + te * nex, ry = tx * nxy + te * ney;
                    xs[2 * end] = q;
                    xs[2 * end + 1] = r;
                    T jx = rx - qx, jy = ry - qy;
                    if (ri) {
                        jv = ca * jv + cb * qswap12(jv);
                        jx = ca * jx + cb * qswap12(jx);
                        jy = ca * jy + cb * qswap12(jy);
                    }
                    S[0] = fma(jv, jv, S[0]);
                    S[1] = fma(jx, jx, fma(jy, jy, S[1]));
                }
                if constexpr (K == 2) {
                    // second derivatives are constant per cell: both endpoints carry the
                    // same jump, 2 (jxx^2 + 2 jxy^2 + jyy^2)
                    T hn[3];
                    hessian(wn, nxx, nxy, nex, ney, hn);
                    T d0 = hn[0] - ho[0], d1 = hn[1] - ho[1], d2 = hn[2] - ho[2];
                    if (ri) {
                        d0 = ca * d0 + cb * qswap12(d0);
                        d1 = ca * d1 + cb * qswap12(d1);
                        d2 = ca * d2 + cb * qswap12(d2);
                    }
                    S[2] = (T)2.0 * (d0 * d0 + (T)2.0 * d1 * d1 + d2 * d2);
                }
                // beta^(i): max spectral radius over both endpoints and both sides; lane v
                // evaluates state v of the four
                T st[4];
                quad_transpose(v, xs, st);
                const T beta = qmax(spectral_radius(st[0], st[1], st[2], st[3], nx, ny, gammaT));
                const T bh = F::div(beta, h);
                T hj = (T)1.0;
#pragma unroll
                for (int jj = 0; jj <= K; ++jj) {
                    T d = (T)kA[K][jj] * hj * inv_my * F::sqrt((T)0.5 * S[jj]);
                    if (ri) d = fmax(d, qswap12(d));   // delta(m) = max(delta(m_n), delta(m_t))
                    sig[jj] = fma(bh, d, sig[jj]);
                    hj *= h;
                }
            }
            // exact solution of the damping ODE: degree-m modes scaled by
            // exp(-dt sum_{j<=m} sigma^j); the cell average is untouched (eq. OE:m0)
            T acc = sig[0];
#pragma unroll
            for (int m = 1; m <= K; ++m) {
                acc += sig[m];
                const T f = F::exp(-dt * acc);
#pragma unroll
                for (int l = m * (m + 1) / 2; l < (m + 1) * (m + 2) / 2; ++l) w[l] *= f;
            }
        }

        // the full state in FP64 at this lane's share of the limiter points, t = v,
        // v+4, v+8
        const double n0x = a.m.node_ref[c], n0e = a.m.node_ref[snc + c];
        const double n1x = a.m.node_ref[2 * snc + c], n1e = a.m.node_ref[3 * snc + c];
        double pv[3][4];
        node_values_t<K, NM, T>(v, wa, w, n0x, n0e, n1x, n1e, a.zxs, a.ustar, pv);
        bool pin[3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) pin[kk] = v + 4 * kk < NP;
        const double ub0 = qget<0>(wa), ub1 = qget<1>(wa), ub2 = qget<2>(wa), ub3 = qget<3>(wa);
        double th1 = 1.0, th2 = 1.0;
        if (a.bp_enable) {
            // step 1: density (Sec. 4.4, eq. 1944)
            double rloc = INFINITY;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
                if (pin[kk]) rloc = fmin(rloc, pv[kk][0]);
            const double rmin = qmin(rloc);
            const double e1 = fmin(ub0, kEpsBP);
            th1 = rmin >= e1 ? 1.0 : fmin((ub0 - e1) / (ub0 - rmin), 1.0);
            // factor of the stored density modes: in the mixed form it aims above the
            // floor by the rounding bound; theta_2 below still comes from the density
            // pinned at eps_1 (rho e grows with rho at nodes below the average, so
            // that theta_2 is the smaller one), which keeps it at the FP64 value
            double th1s = th1;
            // mixed form: sum_{l>=1} |c_l| of each variable (lane v forms its own)
            double as0 = 0.0, as1 = 0.0, as2 = 0.0, as3 = 0.0;
            if constexpr (kMixed) {
                double wd[NM];
                wd[0] = 0.0;
#pragma unroll
                for (int l = 1; l < NM; ++l) wd[l] = (double)w[l];
                const double as = abs_sum_hi<NM>(wd);
                as0 = qget<0>(as);
                as1 = qget<1>(as);
                as2 = qget<2>(as);
                as3 = qget<3>(as);
                const double t1 = e1 + kMixMargin * as0;
                th1s = rmin >= t1 ? 1.0 : fmax(fmin((ub0 - t1) / (ub0 - rmin), 1.0), 0.0);
            }
            // step 2: internal energy E - |m|^2 / (2 rho) of the density-scaled state (eq. 1981)
            const double eb = ub3 - 0.5 * (ub1 * ub1 + ub2 * ub2) / ub0;
            const double e2 = fmin(eb, kEpsBP);
            double eloc = INFINITY;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                pv[kk][0] = ub0 + th1 * (pv[kk][0] - ub0);
                if (pin[kk])
                    eloc = fmin(eloc, pv[kk][3] - 0.5 * (pv[kk][1] * pv[kk][1] + pv[kk][2] * pv[kk][2]) *
                                                      frcp(pv[kk][0]));
            }
            const double emin = qmin(eloc);
            th2 = emin >= e2 ? 1.0 : fmin((eb - e2) / (eb - emin), 1.0);
            if constexpr (kMixed) {
                // Rounding the scaled modes moves rho e at a node by at most, to first
                // order, |dE| + |v| (|dm1| + |dm2|) + |v|^2/2 |drho|, with v the
                // velocity of the limited state there and each |d.| <= margin * theta
                // * sum_l |c_l|; theta_2 aims that far above the floor.
                double vloc = 0.0;
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    if (pin[kk]) {
                        const double q0 = ub0 + th2 * (pv[kk][0] - ub0);
                        const double q1 = ub1 + th2 * (pv[kk][1] - ub1), q2 = ub2 + th2 * (pv[kk][2] - ub2);
                        vloc = fmax(vloc, (q1 * q1 + q2 * q2) * frcp(q0 * q0));
                    }
                }
                const double vm = fsqrt(qmax(vloc));
                const double t2 = e2 + kMixMargin * th2 *
                                           (as3 + vm * (as1 + as2) + 0.5 * vm * vm * th1 * as0);
                th2 = emin >= t2 ? 1.0 : fmax(fmin((eb - t2) / (eb - emin), 1.0), 0.0);
                th1 = th1s;
                const double f = v == 0 ? th1 * th2 : th2;
                if (f < 1.0) {
#pragma unroll
                    for (int l = 1; l < NM; ++l) w[l] = (T)((double)w[l] * f);
                }
            } else {
#pragma unroll
                for (int l = 1; l < NM; ++l) {
                    if (v == 0) w[l] *= th1;
                    w[l] *= th2;
                }
            }
            if (v == 0) {
                f.n_lim += (th1 < 1.0 || th2 < 1.0) ? 1.0 : 0.0;
                f.n_bad += (ub0 > 0.0 && eb > 0.0) ? 0.0 : 1.0;
            }
            if constexpr (kMixed) {
                if (th1 < 1.0 || th2 < 1.0) {   // the same in the four lanes of the quad
                    // check the coefficients as stored (rounded to float)
                    node_values_t<K, NM, T>(v, wa, w, n0x, n0e, n1x, n1e, a.zxs, a.ustar, pv);
                    double ok = 1.0;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk)
                        if (pin[kk] && !(pv[kk][0] >= 0.5 * e1 && internal_energy(pv[kk]) >= 0.5 * e2)) ok = 0.0;
                    if (qmin(ok) == 0.0) {
                        // keep the average only: admissible whenever the average is
#pragma unroll
                        for (int l = 1; l < NM; ++l) w[l] = (T)0.0;
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk) {
                            pv[kk][0] = ub0;
                            pv[kk][1] = ub1;
                            pv[kk][2] = ub2;
                            pv[kk][3] = ub3;
                        }
                        if (v == 0) f.n_flat += 1.0;
                    }
                }
            }
        }

        // max wave speed over the edge Gauss points of the limited state (eq. 1250);
        // in the mixed form pv already holds the stored state's values.  At a
        // boundary edge the point also adds its momentum flux l w_nu F.n, as the
        // next residual pass will take it, to the output's bookkeeping:
        // transmissive F(u).n; reflective ((m.n)^2/rho + p) n plus alpha (m.n) n.
        const double ta = kMixed ? 1.0 : th2;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            const int t = v + 4 * kk;
            if (t < 3 * NE) {
                const int i = t / NE;
                const double nx = (double)(i == 0 ? nxs[0] : (i == 1 ? nxs[1] : nxs[2]));
                const double ny = (double)(i == 0 ? nys[0] : (i == 1 ? nys[1] : nys[2]));
                const double rr = spectral_radius(ub0 + ta * (pv[kk][0] - ub0), ub1 + ta * (pv[kk][1] - ub1),
                                                  ub2 + ta * (pv[kk][2] - ub2), ub3 + ta * (pv[kk][3] - ub3), nx,
                                                  ny, gamma);
                f.amax = (rr > f.amax || rr != rr) ? rr : f.amax;
            }
        }
        if (lk[0] < 0 || lk[1] < 0 || lk[2] < 0) {
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                const int t = v + 4 * kk;
                const int i = t / NE;
                const int link = i == 0 ? lk[0] : (i == 1 ? lk[1] : lk[2]);
                if (t < 3 * NE && link < 0) {
                    const double nx = (double)(i == 0 ? nxs[0] : (i == 1 ? nxs[1] : nxs[2]));
                    const double ny = (double)(i == 0 ? nys[0] : (i == 1 ? nys[1] : nys[2]));
                    const double q0 = ub0 + ta * (pv[kk][0] - ub0), q1 = ub1 + ta * (pv[kk][1] - ub1);
                    const double q2 = ub2 + ta * (pv[kk][2] - ub2), q3 = ub3 + ta * (pv[kk][3] - ub3);
                    const int nu = t - i * NE, th = threadIdx.x;
                    const double lw = a.m.len[i * snc + c] * (nu == 0 ? R::ws[0] : (nu == 1 ? R::ws[1] : R::ws[2]));
                    const double ir = frcp(q0);
                    const double mn = q1 * nx + q2 * ny;
                    const double p = (gamma - 1.0) * (q3 - 0.5 * (q1 * q1 + q2 * q2) * ir);
                    if (link == kLinkWall) {
                        const double ca = lw * (mn * mn * ir + p), cb = lw * mn;
                        book[0][th] += ca * nx;
                        book[1][th] += ca * ny;
                        book[2][th] += cb * nx;
                        book[3][th] += cb * ny;
                    } else {
                        book[0][th] += lw * (q1 * mn * ir + p * nx);
                        book[1][th] += lw * (q2 * mn * ir + p * ny);
                    }
                }
            }
        }
        f.msum = fma(area_d, wa, f.msum);   // sum |K| ubar of this lane's variable
        oa_p[c] = wa;
#pragma unroll
        for (int l = 1; l < NM; ++l) oh_p[(l - 1) * snc + c] = w[l];
    };
    if constexpr (!kBatch) {
        FilterAcc f;
#pragma unroll
        for (int k = 0; k < kBookCols; ++k) book[k][threadIdx.x] = 0.0;
        const TileWalk tw = tile_walk((nc + kCellsPerTile - 1) / kCellsPerTile);
        for (int tile = tw.first; tile < tw.end; tile += tw.stride) {
            const int c = tile * kCellsPerTile + (threadIdx.x >> 2);
            if (c < nc) cell(c, f);   // whole quad
        }
        filter_flush(f, book, a.part + (size_t)(kNumPartial + 1) * kMaxBlocks + blockIdx.x, kMaxBlocks);
    } else {
        for (int gi = g0; gi < g1; ++gi) {
            FilterAcc f;
#pragma unroll
            for (int k = 0; k < kBookCols; ++k) book[k][threadIdx.x] = 0.0;
#pragma unroll 1
            for (int tile = 0; tile < kGroupCells / kCellsPerTile; ++tile) {
                const int c = gi * kGroupCells + tile * kCellsPerTile + (threadIdx.x >> 2);
                if (c < nc) cell(c, f);
            }
            filter_flush(f, book, a.part + (size_t)(kNumPartial + 1) * a.gstride + a.gbase + gi, a.gstride);
            __syncthreads();
        }
    }
}
// three waves per SIMD: the allocator then keeps the P2 instantiations within 168 VGPRs
template <int K, typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_filter(StageArgs a) {
    if (!a.g->active || a.g->skip) return;
    filter_run<K, T, false>(a, 0, 0);
}
// FP64: no occupancy request (with the chunk indirection a 168-VGPR budget spills
// heavily); mixed: three waves per SIMD
template <int KM, typename T>
__device__ __forceinline__ void filter_batch_body(const StageArgs* desc, const Chunk* chunks, const ChunkSplit& cs) {
    for_each_chunk(desc, chunks, cs, [](const StageArgs& a, int g0, int g1) {
        if constexpr (KM != 3) filter_run<KM, T, true>(a, g0, g1);
        else if (a.k == 1) filter_run<1, T, true>(a, g0, g1);
        else filter_run<2, T, true>(a, g0, g1);
    });
}
template <int KM, typename T>
__global__ __launch_bounds__(kBlock) void k_filter_batch(const StageArgs* desc, const Chunk* chunks, ChunkSplit cs) {
    filter_batch_body<KM, T>(desc, chunks, cs);
}
template <int KM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_filter_batch_mixed(
    const StageArgs* desc, const Chunk* chunks, ChunkSplit cs) {
    filter_batch_body<KM, float>(desc, chunks, cs);
}

// ------------------------------------------------------------------------- finalize (one workgroup)

constexpr int kFinThreads = 1024;

// Reduces NC columns base[col(k) * cstride + b], b < G, in a fixed order, where
// col(k) = col0 + k except that the last column is colN when colN >= 0; column k
// with op (opbits >> 2k) & 3 (0 sum, 1 min, 2 max).  Each column gets 16/NC waves
// that stride over the records with kBatchLoads independent loads in flight per
// lane, so the loads are coalesced and the pass is not a chain of load
// latencies.  The results are valid in thread 0.
constexpr int kBatchLoads = 8;
template <int NC>
__device__ __forceinline__ void reduce_columns(const double* base, size_t cstride, int G, int col0, unsigned opbits,
                                               double (&out)[NC], int colN = -1) {
    constexpr int kWaves = kFinThreads / 64, kPer = kWaves / NC;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = w / kPer, sub = w - k * kPer;
    __shared__ double lds[kWaves];
    if (k < NC) {
        const int op = (opbits >> (2 * k)) & 3;
        const int c = (k == NC - 1 && colN >= 0) ? colN : col0 + k;
        const double* col = base + (size_t)c * cstride;
        const double ident = op == 0 ? 0.0 : (op == 1 ? INFINITY : -INFINITY);
        double acc = ident;
        constexpr int kStride = kPer * 64;
        for (int b0 = sub * 64 + lane; b0 < G; b0 += kBatchLoads * kStride) {
            double x[kBatchLoads];
#pragma unroll
            for (int i = 0; i < kBatchLoads; ++i) x[i] = b0 + i * kStride < G ? col[b0 + i * kStride] : ident;
#pragma unroll
            for (int i = 0; i < kBatchLoads; ++i)
                acc = op == 0 ? acc + x[i] : (op == 1 ? fmin(acc, x[i]) : fmax(acc, x[i]));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double y = __shfl_xor(acc, o, 64);
            acc = op == 0 ? acc + y : (op == 1 ? fmin(acc, y) : fmax(acc, y));
        }
        if (lane == 0) lds[w] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int kk = 0; kk < NC; ++kk) {
            const int op = (opbits >> (2 * kk)) & 3;
            double v = lds[kk * kPer];
            for (int s2 = 1; s2 < kPer; ++s2) {
                const double y = lds[kk * kPer + s2];
                v = op == 0 ? v + y : (op == 1 ? fmin(v, y) : fmax(v, y));
            }
            out[kk] = v;
        }
    }
}

// domain averages and L-infinity norms (eq. normOmg): ||u - ubar|| = max(max u - ubar, ubar - min u)
// An inadmissible average ends this attempt of the step: `skip` turns the rest
// of it into no-ops (u^n is untouched) until the third stage's finalize.
// and ||| m - mbar |||_inf (eqs. normOmg, RIOESys:Coef1) with its zero branch
__device__ __forceinline__ void fin_residual(const double* base, size_t cstride, int G, Glob* g) {
    // 4 sums, 4 mins, 4 maxima, the max of |m - mbar|^2, then the bad-average count
    double tot[kNumPartial + 2];
    reduce_columns<kNumPartial + 2>(base, cstride, G, 0, 0x2AA5500u, tot, kColBad);
    if (threadIdx.x == 0) {
        if (tot[kNumPartial + 1] > 0.0) g->skip = 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double ub = tot[v] / g->area_sum;
            const double n = fmax(tot[8 + v] - ub, ub - tot[4 + v]);
            g->ubar[v] = ub;
            g->nrm[v] = n;
            g->inv_nrm[v] = n <= kEpsOE * fmax(1.0, fabs(ub)) ? 0.0 : 1.0 / n;
        }
        const double n = sqrt(tot[kNumPartial]);
        const double mb = sqrt(g->ubar[1] * g->ubar[1] + g->ubar[2] * g->ubar[2]);
        g->nrm_m = n;
        g->inv_nrm_m = n <= kEpsOE * fmax(1.0, mb) ? 0.0 : 1.0 / n;
    }
}

// alpha of the stage output; after the third stage (or the initial limiter pass)
// t, the step count and Delta t = C_SSP/alpha min_K C^DCW_{K,k}|K|, clamped to t_end.
// After the third stage of a skipped attempt: the step is retried from u^n with
// half the time step, or the run stops once max_restarts retries are used.
__device__ __forceinline__ void fin_filter(const double* base, size_t cstride, int G, Glob* g, int stage) {
    const int skip = g->skip;
    __syncthreads();   // every thread has read `skip` before thread 0 may clear it
    if (skip) {
        if (threadIdx.x == 0 && stage == 2) {
            g->skip = 0;
            if (++g->restarts > g->max_restarts) {
                g->err = 1;
                g->active = 0;
            } else {
                g->dt *= 0.5;
                g->alpha = g->alpha_step;   // the retry's first stage starts from u^n again
                g->n_restarts += 1;
            }
        }
        return;
    }
    double r[kFilterCols];
    reduce_columns<kFilterCols>(base, cstride, G, kNumPartial + 1, 2u, r);   // max, then sums
    if (threadIdx.x != 0) return;
    const double alpha = r[0], lim = r[1], bad = r[2];
    // the output's momentum bookkeeping; after the third stage (or the initial
    // limiter pass) the output is u^n
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        g->mom_c[j] = r[4 + j];
        g->bfa_c[j] = r[6 + j];
        g->bfb_c[j] = r[8 + j];
        if (stage < 0 || stage == 2) {
            g->mom_n[j] = r[4 + j];
            g->bfa_n[j] = r[6 + j];
            g->bfb_n[j] = r[8 + j];
        }
    }
    g->n_limited += (long long)lim;
    g->n_bad += (long long)bad;
    g->n_flat += (long long)r[3];
    if (bad > 0) g->err = 1;
    if (stage < 2) {
        g->alpha = alpha;
        if (stage < 0) g->alpha_step = alpha;
        else if (alpha > g->alpha_step * (1.0 + 1e-12)) g->n_cfl_exc += 1;
    } else {
        g->t += g->dt;
        g->step += 1;
        g->alpha = alpha;
        g->alpha_step = alpha;
        g->restarts = 0;
    }
    if (stage < 0 || stage == 2) {
        double dt = g->c_ssp * g->minck / alpha;
        const double rem = g->t_end - g->t;
        if (rem < dt) dt = rem;
        g->dt = dt;
        if (!(isinf(g->t_end) || rem > 1e-12 * fmax(1.0, fabs(g->t_end)))) g->active = 0;
    }
    if (g->err) g->active = 0;
}

// One instance: the partials of the G workgroups of its passes.
__global__ __launch_bounds__(kFinThreads) void k_fin_residual(const double* part, int G, Glob* g) {
    if (g->active) fin_residual(part, kMaxBlocks, G, g);
}
__global__ __launch_bounds__(kFinThreads) void k_fin_filter(const double* part, int G, Glob* g, int stage) {
    if (g->active) fin_filter(part, kMaxBlocks, G, g, stage);
}

// A batch: workgroup i reduces the group records of instance desc[i].
__global__ __launch_bounds__(kFinThreads) void k_fin_residual_batch(const StageArgs* desc) {
    const StageArgs& a = desc[blockIdx.x];
    if (a.g->active) fin_residual(a.part + a.gbase, a.gstride, n_groups(a.m.n_cell), a.g);
}
__global__ __launch_bounds__(kFinThreads) void k_fin_filter_batch(const StageArgs* desc) {
    const StageArgs& a = desc[blockIdx.x];
    if (a.g->active) fin_filter(a.part + a.gbase, a.gstride, n_groups(a.m.n_cell), a.g, a.stage);
}

// ------------------------------------------------------------------------- initial data

struct ProblemParams {
    double p[20];
};

// 12-point degree-6 rule of tab:6th, as printed: barycentric (b1, b2, b3) and weight
__device__ constexpr double kQ12[12][4] = {
    {0.063089014491502, 0.063089014491502, 0.873821971016996, 0.050844906370207},
    {0.063089014491502, 0.873821971016996, 0.063089014491502, 0.050844906370207},
    {0.873821971016996, 0.063089014491502, 0.063089014491502, 0.050844906370207},
    {0.249286745170910, 0.249286745170910, 0.501426509658180, 0.116786275726379},
    {0.249286745170910, 0.501426509658180, 0.249286745170910, 0.116786275726379},
    {0.501426509658180, 0.249286745170910, 0.249286745170910, 0.116786275726379},
    {0.053145049844817, 0.636502499121399, 0.310352451033784, 0.082851075618374},
    {0.636502499121399, 0.053145049844817, 0.310352451033784, 0.082851075618374},
    {0.053145049844817, 0.310352451033784, 0.636502499121399, 0.082851075618374},
    {0.636502499121399, 0.310352451033784, 0.053145049844817, 0.082851075618374},
    {0.310352451033784, 0.053145049844817, 0.636502499121399, 0.082851075618374},
    {0.310352451033784, 0.636502499121399, 0.053145049844817, 0.082851075618374}};

__device__ __forceinline__ void problem_state(int kind, const ProblemParams& P, double gamma, double x, double y,
                                              double* q) {
    double r, u, v, p;
    if (kind == 0) {   // isentropic vortex
        const double xb = x - P.p[0], yb = y - P.p[1], r2 = xb * xb + yb * yb, eps = P.p[2];
        const double amp = eps / (2.0 * M_PI) * exp(0.5 * (1.0 - r2));
        const double T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * M_PI * M_PI) * exp(1.0 - r2);
        r = P.p[3] * pow(T, 1.0 / (gamma - 1.0));
        u = P.p[4] - amp * yb;
        v = P.p[5] + amp * xb;
        p = pow(r, gamma) * (P.p[6] / pow(P.p[3], gamma));
    } else if (kind == 1) {   // four quadrants
        const int qd = (x >= P.p[0] ? 1 : 0) + (y >= P.p[1] ? 2 : 0);
        r = P.p[2 + 4 * qd];
        u = P.p[3 + 4 * qd];
        v = P.p[4 + 4 * qd];
        p = P.p[5 + 4 * qd];
    } else {   // two states across a line
        const int side = ((x - P.p[0]) * P.p[2] + (y - P.p[1]) * P.p[3]) < 0.0 ? 0 : 1;
        r = P.p[4 + 4 * side];
        u = P.p[5 + 4 * side];
        v = P.p[6 + 4 * side];
        p = P.p[7 + 4 * side];
    }
    q[0] = r;
    q[1] = r * u;
    q[2] = r * v;
    q[3] = p / (gamma - 1.0) + 0.5 * r * (u * u + v * v);
}

// L2 projection (mass diagonal): u^(l) = sum_mu w_mu q(x_mu) Psi_l(x_mu) / (a_l/|K|),
// accumulated in FP64 and stored in the state view (higher modes rounded to T).
// vx holds the oriented vertex coordinates [6][cell]; for the blast, vx[6][cell]
// flags the cells that own the origin vertex and P.p[4] is their total area.
template <int K, typename T>
__global__ __launch_bounds__(kBlock) void k_project(StageArgs a, int kind, ProblemParams P, const double* vx) {
    constexpr int NM = Rule<K>::NM;
    const int nc = a.m.n_cell;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    const size_t snc = (size_t)nc;
    double acc[4][NM];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < NM; ++l) acc[v][l] = 0.0;
    if (kind == 2) {
        const bool hit = vx[6 * snc + c] != 0.0;
        acc[0][0] = P.p[2];
        acc[3][0] = hit ? P.p[0] / P.p[4] : P.p[1] / (a.gamma - 1.0);
    } else {
        double X[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) X[k] = vx[k * snc + c];
        for (int m = 0; m < 12; ++m) {
            const double b1 = kQ12[m][0], b2 = kQ12[m][1], b3 = kQ12[m][2], wm = kQ12[m][3];
            const double x = b1 * X[0] + b2 * X[2] + b3 * X[4];
            const double y = b1 * X[1] + b2 * X[3] + b3 * X[5];
            double q[4], p[NM];
            problem_state(kind, P, a.gamma, x, y, q);
            psi<K>(b2, b3, p);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int l = 0; l < NM; ++l) acc[v][l] = fma(wm * q[v], p[l], acc[v][l]);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) acc[v][l] *= kInvMass[l];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const VarPtr<NM, T> op = var_ptr<NM, T>(a.uout, a, v, snc);
        op.avg[c] = acc[v][0];
#pragma unroll
        for (int l = 1; l < NM; ++l) op.hi[(l - 1) * snc + c] = (T)acc[v][l];
    }
}

__global__ void k_set_end(Glob* g, double t_end) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    g->t_end = t_end;
    if (g->err) {
        g->active = 0;
        return;
    }
    double dt = g->c_ssp * g->minck / g->alpha_step;
    const double rem = t_end - g->t;
    if (rem < dt) dt = rem;
    g->dt = dt;
    g->active = (isinf(t_end) || rem > 1e-12 * fmax(1.0, fabs(t_end))) ? 1 : 0;
}

inline unsigned grid_for(int nc) { return (unsigned)((nc + kBlock - 1) / kBlock); }

__global__ void k_gather_status(const StageArgs* desc, int n, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Glob* g = desc[i].g;
    double* o = out + kStatusCols * i;
    o[0] = (double)g->active;
    o[1] = (double)g->err;
    o[2] = g->t;
    o[3] = (double)g->step;
    o[4] = g->dt;
    o[5] = g->t_end;
}

// host handles of the instantiations of one (degree, precision)
struct KernelSet {
    const void* pass[kNumPasses];   // residual, filter
    const void* project;
};
template <int K, typename T>
KernelSet kernel_set() {
    return {{reinterpret_cast<const void*>(&k_residual<K, T>), reinterpret_cast<const void*>(&k_filter<K, T>)},
            reinterpret_cast<const void*>(&k_project<K, T>)};
}
const KernelSet& kernels_for(int k, int mixed) {
    static const KernelSet sets[2][2] = {{kernel_set<1, double>(), kernel_set<1, float>()},
                                         {kernel_set<2, double>(), kernel_set<2, float>()}};
    return sets[k == 2 ? 1 : 0][mixed ? 1 : 0];
}

// host handles of the batched pass instantiations of one (degree mask, precision)
struct BatchSet {
    const void* pass[kNumPasses];   // residual, filter
};
template <int KM, typename T>
BatchSet batch_set() {
    const void* filter;
    if constexpr (std::is_same<T, float>::value) filter = reinterpret_cast<const void*>(&k_filter_batch_mixed<KM>);
    else filter = reinterpret_cast<const void*>(&k_filter_batch<KM, T>);
    return {{reinterpret_cast<const void*>(&k_residual_batch<KM, T>), filter}};
}
const BatchSet& batch_kernels(int kmask, int mixed) {
    static const BatchSet sets[3][2] = {{batch_set<1, double>(), batch_set<1, float>()},
                                        {batch_set<2, double>(), batch_set<2, float>()},
                                        {batch_set<3, double>(), batch_set<3, float>()}};
    return sets[kmask - 1][mixed ? 1 : 0];
}

// Grid of a pass: one workgroup per tile while the tiles fit on the GPU at once,
// otherwise as many workgroups as can be resident (occupancy x compute units),
// rounded down to a multiple of 8 so every XCD gets the same share; workgroups
// then stride over their XCD's tiles.  Bounded by kMaxBlocks (the partials).
int resident_blocks(const void* kernel) {
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 1, cus = cus > 0 ? cus : 256;
    const int g = std::min(kMaxBlocks, std::max(8, (cus * per_cu) / 8 * 8));
    cache[kernel] = g;
    return g;
}

int launch_pass(int which, int k, const StageArgs& a, void* stream) {
    StageArgs args = a;
    void* argv[] = {&args};
    const int grid = grid_for_pass(which, k, a.mixed, a.m.n_cell);
    return (int)hipLaunchKernel(kernels_for(k, a.mixed).pass[which], dim3(grid), dim3(kBlock), argv, 0,
                                (hipStream_t)stream);
}

// Partial records of dg_stage_noalloc: a file-scope device array, one copy per
// GPU at that GPU's own address.  Host code never uses its name as an address:
// scratch_address() asks the runtime for it once per device, with that device
// current, and the launches take the returned pointer.
static __device__ __align__(256) double scratch[kScratchDoubles];

}  // namespace

int scratch_address(int device, double** out) {
    static std::mutex mu;
    static std::unordered_map<int, double*> addr;
    std::lock_guard<std::mutex> lock(mu);
    *out = nullptr;
    auto it = addr.find(device);
    if (it != addr.end()) {
        *out = it->second;
        return 0;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return (int)e;
    if (cur != device) return (int)hipErrorInvalidDevice;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (p == nullptr) return (int)hipErrorInvalidSymbol;
    addr[device] = (double*)p;
    *out = (double*)p;
    return 0;
}

int grid_for_pass(int which, int k, int mixed, int n_cell) {
    const int tiles = (n_cell + kCellsPerTile - 1) / kCellsPerTile;
    const int want = std::max(8, ((tiles + 7) / 8) * 8);
    return std::min(want, resident_blocks(kernels_for(k, mixed).pass[which]));
}

int launch_residual(int k, const StageArgs& a, void* stream) { return launch_pass(kPassResidual, k, a, stream); }
int launch_filter(int k, const StageArgs& a, void* stream) { return launch_pass(kPassFilter, k, a, stream); }

int launch_finalize(int which, int k, const StageArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int G = grid_for_pass(which, k, a.mixed, a.m.n_cell);
    if (which == kPassResidual)
        hipLaunchKernelGGL(k_fin_residual, dim3(1), dim3(kFinThreads), 0, s, a.part, G, a.g);
    else
        hipLaunchKernelGGL(k_fin_filter, dim3(1), dim3(kFinThreads), 0, s, a.part, G, a.g, a.stage);
    return (int)hipGetLastError();
}

int launch_project(int k, const StageArgs& a, int kind, const double* dparams, int n_params, const double* vx,
                   void* stream) {
    ProblemParams P{};
    for (int i = 0; i < n_params && i < 20; ++i) P.p[i] = dparams[i];
    StageArgs args = a;
    void* argv[] = {&args, &kind, &P, &vx};
    return (int)hipLaunchKernel(kernels_for(k, a.mixed).project, dim3(grid_for(a.m.n_cell)), dim3(kBlock), argv, 0,
                                (hipStream_t)stream);
}

int resident_grid_batch(int which, int kmask, int mixed) {
    return std::max(8, resident_blocks(batch_kernels(kmask, mixed).pass[which]) / 8 * 8);
}

int launch_pass_batch(int which, int kmask, int mixed, const StageArgs* desc, const Chunk* chunks,
                      const ChunkSplit& cs, int grid, void* stream) {
    if (kmask < 1 || kmask > 3 || grid < 8 || (grid & 7) != 0) return (int)hipErrorInvalidValue;
    ChunkSplit split = cs;
    void* argv[] = {&desc, &chunks, &split};
    return (int)hipLaunchKernel(batch_kernels(kmask, mixed).pass[which], dim3(grid), dim3(kBlock), argv, 0,
                                (hipStream_t)stream);
}

int launch_finalize_batch(int which, const StageArgs* desc, int n_inst, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (which == kPassResidual) hipLaunchKernelGGL(k_fin_residual_batch, dim3(n_inst), dim3(kFinThreads), 0, s, desc);
    else hipLaunchKernelGGL(k_fin_filter_batch, dim3(n_inst), dim3(kFinThreads), 0, s, desc);
    return (int)hipGetLastError();
}

int launch_gather_status(const StageArgs* desc, int n, double* out, void* stream) {
    hipLaunchKernelGGL(k_gather_status, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, desc, n, out);
    return (int)hipGetLastError();
}

int launch_set_end(Glob* g, double t_end, void* stream) {
    hipLaunchKernelGGL(k_set_end, dim3(1), dim3(64), 0, (hipStream_t)stream, g, t_end);
    return (int)hipGetLastError();
}

}  // namespace oedg
