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
// Lane layout of the two passes: one lane per cell, all four conservative
// variables and their modes in that lane's registers, so every point value,
// 1/rho, pressure and flux is formed once.  A pass workgroup takes tiles of 256
// consecutive (Hilbert-ordered) cells, one per thread, and stages each tile with
// its halo of out-of-tile neighbours in LDS before computing it.  The residual's
// image holds every cell's averages, modes and geometry, from which a neighbour's
// traces at the edge Gauss points are formed with the basis rows of its local
// edge (the batched FP64 P2 pass uses the filter's image instead).  The filter's
// image holds every cell's polynomial as physical monomials about its vertex 0
// plus the two edge vectors from that vertex, so a neighbour's value, gradient
// and Hessian at a shared vertex cost a few FMAs.  The filter works every edge
// inside a tile once: the mesh precompute makes one cell of it the owner (at most
// two in-tile edges per cell, and in most waves at most two edges of any kind per
// lane), and the owner hands the other cell its damping rates through LDS once
// the image is no longer read.  Workgroups are spread so that each XCD walks a
// contiguous range of the tiles, which keeps neighbour gathers inside that XCD's
// L2.
//
// Edge fluxes are conservative to the last bit: both cells of an interior edge
// evaluate its LF flux from the same two traces (each cell's trace computed by the
// same arithmetic from the same basis rows, whichever lane asks), with the
// lower-index cell's scaled normal and length, and in a fixed operand order, so
// the two contributions are exact negatives of each other.  The file is compiled
// with FMA contraction off; every fused multiply-add is written out.
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

#pragma clang fp contract(off)

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
// derivatives of sum_l u_l Psi_l at vertex (sx, se), for a vertex known only at
// run time (a neighbour's).
template <int K, typename T>
__device__ __forceinline__ void vertex_eval(const T* u, T sx, T se, T& qh, T& dx, T& de) {
    if constexpr (K == 1) {
        const T b = (T)4.0 * u[1], c = fma((T)2.0, u[1], (T)3.0 * u[2]);
        qh = fma(b, sx, fma(c, se, fma((T)-2.0, u[1], -u[2])));
        dx = b;
        de = c;
    } else {
        const T a = fma((T)-2.0, u[1], fma((T)4.0, u[3], fma((T)2.0, u[4], u[5] - u[2])));
        const T b = (T)4.0 * (u[1] - u[4]);
        const T c = fma((T)2.0, u[1], fma((T)3.0, u[2], fma((T)-4.0, u[3], (T)2.0 * (u[5] - u[4]))));
        qh = fma(b, sx, fma(c, se, a));
        const T h1 = fma((T)24.0, u[3], (T)20.0 * u[4]);
        const T ax = fma((T)4.0, u[1] - u[4], (T)-24.0 * u[3]);
        dx = fma((T)48.0 * u[3], sx, fma(h1, se, ax));
        const T ae = fma((T)2.0, u[1], fma((T)3.0, u[2], fma((T)-8.0, u[3], fma((T)-12.0, u[4], (T)-8.0 * u[5]))));
        de = fma(h1, sx, fma(fma((T)8.0, u[3], (T)20.0 * (u[4] + u[5])), se, ae));
    }
}

// The same at a vertex VT known at compile time (the cell's own): no indicator terms.
template <int K, int VT, typename T>
__device__ __forceinline__ void vertex_eval_ct(const T* u, T& qh, T& dx, T& de) {
    if constexpr (K == 1) {
        const T b = (T)4.0 * u[1], c = fma((T)2.0, u[1], (T)3.0 * u[2]);
        const T a = fma((T)-2.0, u[1], -u[2]);
        qh = VT == 0 ? a : (VT == 1 ? a + b : a + c);
        dx = b;
        de = c;
    } else {
        const T a = fma((T)-2.0, u[1], fma((T)4.0, u[3], fma((T)2.0, u[4], u[5] - u[2])));
        const T h1 = fma((T)24.0, u[3], (T)20.0 * u[4]);
        const T ax = fma((T)4.0, u[1] - u[4], (T)-24.0 * u[3]);
        const T ae = fma((T)2.0, u[1], fma((T)3.0, u[2], fma((T)-8.0, u[3], fma((T)-12.0, u[4], (T)-8.0 * u[5]))));
        if constexpr (VT == 0) {
            qh = a;
            dx = ax;
            de = ae;
        } else if constexpr (VT == 1) {
            qh = fma((T)4.0, u[1] - u[4], a);
            dx = fma((T)48.0, u[3], ax);
            de = h1 + ae;
        } else {
            const T c = fma((T)2.0, u[1], fma((T)3.0, u[2], fma((T)-4.0, u[3], (T)2.0 * (u[5] - u[4]))));
            qh = c + a;
            dx = h1 + ax;
            de = fma((T)8.0, u[3], fma((T)20.0, u[4] + u[5], ae));
        }
    }
}

// Basis values at the fixed points of a stage, in constant memory: the point loops
// run with a wave-uniform index, so these become scalar loads instead of registers.
template <int K, typename T>
struct Tab {
    static constexpr int NM = Rule<K>::NM, NQ = Rule<K>::NQ, NE = Rule<K>::NE;
    T vp[NQ][NM], vdx[NQ][NM], vde[NQ][NM];   // volume points: Psi, dPsi/dxi, dPsi/deta
    T vw[NQ];                                 // volume weights
    T ep[3 * NE][NM];                         // edge Gauss points (edge i, node nu)
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

// sum_l u_l p_l with p_0 = Psi_0 = 1: the same operation sequence for every caller,
// whether the row comes from constant memory or from its copy in LDS
template <int NM, typename T>
__device__ __forceinline__ T dot(const T* u, const T* p) {
    T s = u[0];
#pragma unroll
    for (int l = 1; l < NM; ++l) s = fma(u[l], p[l], s);
    return s;
}
// sum over the modes l >= 1 (the point value minus the average)
template <int NM, typename T>
__device__ __forceinline__ T dot_hi(const T* u, const T* p) {
    T s = u[1] * p[1];
#pragma unroll
    for (int l = 2; l < NM; ++l) s = fma(u[l], p[l], s);
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
    // v_sqrt_f32 itself (1 ulp) instead of the correctly rounded expansion
    static __device__ __forceinline__ float sqrt(float x) { return x > 0.0f ? __builtin_amdgcn_sqrtf(x) : 0.0f; }
    // 2^(x log2 e) with v_exp_f32: a few ulp, results below the normal range flush to 0
    static __device__ __forceinline__ float exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
    static __device__ __forceinline__ float div(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
};

// ------------------------------------------------------------------------- Euler

// 1/rho and the pressure (gamma - 1)(E - |m|^2 / (2 rho)) of a point value
template <typename T>
__device__ __forceinline__ void euler_ip(const T (&q)[4], T gm1, T& ir, T& p) {
    ir = Fp<T>::rcp(q[0]);
    p = gm1 * fma((T)-0.5 * ir, fma(q[1], q[1], q[2] * q[2]), q[3]);
}

// F(q).n for the four conservative variables (Example ex:euler), (nx, ny) any
// (scaled) normal, with 1/rho and the pressure given
template <typename T>
__device__ __forceinline__ void euler_flux_n(const T (&q)[4], T ir, T p, T nx, T ny, T (&f)[4]) {
    const T mn = fma(q[1], nx, q[2] * ny);
    const T vn = mn * ir;
    f[0] = mn;
    f[1] = fma(q[1], vn, p * nx);
    f[2] = fma(q[2], vn, p * ny);
    f[3] = (q[3] + p) * vn;
}

// spectral radius |v.n| + c of F'(u).n (Example ex:euler); guarded so that a
// pre-limiter state with rho <= 0 or p < 0 still gives a finite value
template <typename T>
__device__ __forceinline__ T spectral_radius(T q0, T q1, T q2, T q3, T nx, T ny, T gamma) {
    const T ir = Fp<T>::rcp(fmax(q0, (T)kEpsBP));
    const T p = (gamma - (T)1.0) * fma((T)-0.5 * ir, fma(q1, q1, q2 * q2), q3);
    return fma(fabs(fma(q1, nx, q2 * ny)), ir, Fp<T>::sqrt(gamma * fmax(p, (T)0.0) * ir));
}

// l_e n_e = -2 |K| grad(lambda_e), the scaled outward normal of local edge e from
// the rows (xx, xy), (ex, ey) of J^-1: grad lambda_1 = (xx, xy), grad lambda_2 =
// (ex, ey), grad lambda_0 = -(both).  e may be a run-time (per-lane) index: the
// selects pick among the same three expressions, so the result does not depend on
// which cell's lane forms it.
template <typename T>
__device__ __forceinline__ void scaled_normal(T xx, T xy, T ex, T ey, T area, int e, T& nx, T& ny) {
    const T gx = e == 0 ? -(xx + ex) : (e == 1 ? xx : ex);
    const T gy = e == 0 ? -(xy + ey) : (e == 1 ? xy : ey);
    const T s = (T)-2.0 * area;
    nx = s * gx;
    ny = s * gy;
}

// the unit outward normal of local edge e, from J^-1, |K| and the edge's length l
template <typename T>
__device__ __forceinline__ void unit_normal(T xx, T xy, T ex, T ey, T area, int e, T len, T& nx, T& ny) {
    T lnx, lny;
    scaled_normal(xx, xy, ex, ey, area, e, lnx, lny);
    const T il = Fp<T>::rcp(len);
    nx = lnx * il;
    ny = lny * il;
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

// Wave reductions over the 64 lanes (all active) by DPP: within each row of 16
// lanes two quad permutes and two rotations leave the row's result in every lane,
// then the two row broadcasts of gfx9 carry rows 0 and 2 into rows 1 and 3 and
// rows 0-1 into rows 2-3, so lane 63 holds the result, which every lane reads.
// No LDS traffic, and a fixed order of operations (deterministic results).
// DPP moves 32 bits: a double goes as its two halves; the rows a broadcast does
// not write receive `fill`, the operation's identity.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_d(double v, double fill) {
    const long long b = __builtin_bit_cast(long long, v), f = __builtin_bit_cast(long long, fill);
    const int lo = __builtin_amdgcn_update_dpp((int)f, (int)b, Ctrl, RowMask, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(b >> 32), Ctrl, RowMask, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}
__device__ __forceinline__ double lane63(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, double ident, Op op) {
    v = op(v, dpp_d<0xB1, 0xF>(v, ident));    // quad_perm [1,0,3,2]
    v = op(v, dpp_d<0x4E, 0xF>(v, ident));    // quad_perm [2,3,0,1]
    v = op(v, dpp_d<0x124, 0xF>(v, ident));   // row_ror:4
    v = op(v, dpp_d<0x128, 0xF>(v, ident));   // row_ror:8
    v = op(v, dpp_d<0x142, 0xA>(v, ident));   // row_bcast:15 into rows 1 and 3
    v = op(v, dpp_d<0x143, 0xC>(v, ident));   // row_bcast:31 into rows 2 and 3
    return lane63(v);
}
__device__ __forceinline__ double wave_sum(double v) {
    return wave_reduce(v, 0.0, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_max(double v) {
    return wave_reduce(v, -INFINITY, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ double wave_min(double v) {
    return wave_reduce(v, INFINITY, [](double a, double b) { return fmin(a, b); });
}

// Raw buffer access.  Every load and store of the two passes goes through a
// resource descriptor in scalar registers plus a 32-bit per-lane byte offset (the
// cell index times the element size, shared by every array of a cell) and a
// wave-uniform offset (variable, mode, component), instead of a 64-bit address in
// vector registers per load.  num_records covers the array, so the hardware's
// range check never drops a valid access.
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcFlags = 0x00020000;   // dword 3 of a raw buffer resource on gfx9-family parts
__device__ __forceinline__ Rsrc make_rsrc(const void* p, size_t bytes) {
    const unsigned n = bytes > 0xffffffffull ? 0xffffffffu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, kRsrcFlags);
}
template <typename T>
__device__ __forceinline__ T bld(Rsrc r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double bld<double>(Rsrc r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ float bld<float>(Rsrc r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ int bld<int>(Rsrc r, unsigned voff, unsigned soff) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bst(double x, Rsrc r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bst(float x, Rsrc r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)voff, (int)soff, 0);
}

// One state buffer: the FP64 averages (variable v of the cell at byte offset
// c*8 + v*avs) and the higher modes in the bulk type (mode l of variable v at
// c*sizeof(T) + v*hvs + (l-1)*ms).  The FP64 form is one [var][mode][cell] array
// (both resources cover it); the mixed form has its averages and its float modes in
// two regions.
template <int NM, typename T>
struct SView {
    Rsrc avg, hi;
    unsigned avs, hvs, ms;
    __device__ __forceinline__ double a(int v, unsigned c8) const { return bld<double>(avg, c8, v * avs); }
    __device__ __forceinline__ T h(int v, int l, unsigned cT) const { return bld<T>(hi, cT, v * hvs + (l - 1) * ms); }
    __device__ __forceinline__ void put_a(int v, unsigned c8, double x) const { bst(x, avg, c8, v * avs); }
    __device__ __forceinline__ void put_h(int v, int l, unsigned cT, T x) const {
        bst(x, hi, cT, v * hvs + (l - 1) * ms);
    }
};
template <int NM, typename T>
__device__ __forceinline__ SView<NM, T> sview(const StateView& sv, const StageArgs& a) {
    const size_t nc = (size_t)a.m.n_cell;
    SView<NM, T> s;
    if constexpr (std::is_same<T, double>::value) {
        // [var][mode][cell]: sv.hi = sv.avg + n_cell, so mode l >= 1 of variable v is
        // at v*NM*nc + (l-1)*nc elements from sv.hi
        s.avg = make_rsrc(sv.avg, 4 * NM * nc * sizeof(double));
        s.hi = make_rsrc(sv.hi, (4 * NM - 1) * nc * sizeof(double));
        s.avs = s.hvs = (unsigned)(NM * nc * sizeof(double));
        s.ms = (unsigned)(nc * sizeof(double));
    } else {
        s.avg = make_rsrc(sv.avg, 4 * (size_t)a.avs * sizeof(double));
        s.hi = make_rsrc(sv.hi, 4 * (size_t)a.hvs * sizeof(float));
        s.avs = (unsigned)(a.avs * sizeof(double));
        s.hvs = (unsigned)(a.hvs * sizeof(float));
        s.ms = (unsigned)(nc * sizeof(float));
    }
    return s;
}
// cell c of a state: FP64 averages and bulk-type modes (mode 0 = the average in T)
template <int NM, typename T>
__device__ __forceinline__ void load_cell(const SView<NM, T>& s, int c, double (&avg)[4], T (&u)[4][NM]) {
    const unsigned c8 = (unsigned)c * 8u, cT = (unsigned)c * (unsigned)sizeof(T);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        avg[v] = s.a(v, c8);
        u[v][0] = (T)avg[v];
#pragma unroll
        for (int l = 1; l < NM; ++l) u[v][l] = s.h(v, l, cT);
    }
}
// The mesh arrays of an instance: J^-1 [4][cell], |K|, edge lengths [3][cell],
// edge links [3][cell], limiter-node reference coordinates [4][cell].
struct MView {
    Rsrc jinv, area, len, link, llink, node;
    unsigned n8, n4;   // byte strides of a component: n_cell * 8, n_cell * 4
    __device__ __forceinline__ double J(int k, unsigned c8) const { return bld<double>(jinv, c8, k * n8); }
    __device__ __forceinline__ double A(unsigned c8) const { return bld<double>(area, c8, 0); }
    __device__ __forceinline__ double L(int i, unsigned c8) const { return bld<double>(len, c8, i * n8); }
    __device__ __forceinline__ int link_of(int i, unsigned c4) const { return bld<int>(link, c4, i * n4); }
    __device__ __forceinline__ double N(int k, unsigned c8) const { return bld<double>(node, c8, k * n8); }
};
__device__ __forceinline__ MView mview(const DevMesh& m) {
    const size_t nc = (size_t)m.n_cell;
    MView v;
    v.jinv = make_rsrc(m.jinv, 4 * nc * 8);
    v.area = make_rsrc(m.area, nc * 8);
    v.len = make_rsrc(m.len, 3 * nc * 8);
    v.link = make_rsrc(m.link, 3 * nc * 4);
    v.llink = make_rsrc(m.llink, 3 * nc * 4);
    v.node = make_rsrc(m.node_ref, 4 * nc * 8);
    v.n8 = (unsigned)(nc * 8);
    v.n4 = (unsigned)(nc * 4);
    return v;
}

// a wave-uniform double moved to scalar registers
__device__ __forceinline__ double uniform(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

// The edge Gauss point rows of the basis in LDS, for the exterior trace: a
// neighbour's local edge is a per-lane index, so its rows cannot come from the
// scalar path.  Filled by the workgroup before the first cell.
template <int K, typename T>
struct EdgeRowsLds {
    T r[3 * Rule<K>::NE][Rule<K>::NM];
};
template <int K, typename T>
__device__ __forceinline__ void fill_edge_rows(EdgeRowsLds<K, T>& dst) {
    constexpr int N = 3 * Rule<K>::NE * Rule<K>::NM;
    const T* src = &tab<K, T>().ep[0][0];
    T* d = &dst.r[0][0];
    for (int t = threadIdx.x; t < N; t += blockDim.x) d[t] = src[t];
}

#ifndef OEDG_RES_WAVES
#define OEDG_RES_WAVES 2
#endif
#ifndef OEDG_FIL_WAVES
#define OEDG_FIL_WAVES 2
#endif

// ------------------------------------------------------------------------- tiles in LDS

// LDS image of a tile and its halo for one pass: per slot the four FP64 averages,
// the modes l >= 1 in the bulk type and NG geometry entries in the bulk type (the
// rows of J^-1, then |K| for the residual).  Slot s < kTileCells holds cell
// tile * kTileCells + s, slot kTileCells + h the tile's halo cell h.  SoA per
// entry, so a lane's slot reads are 8-byte (4-byte) strided accesses.
template <int K, typename T, int NG>
struct TileLds {
    static constexpr int NM = Rule<K>::NM, S = kTileCells + kHaloCap;
    double avg[4][S];
    T hi[4][NM - 1][S];
    T geo[NG][S];
};
template <int K, typename T, int NG>
__device__ __forceinline__ void stage_put(TileLds<K, T, NG>& L, int s, const double (&avg)[4],
                                          const T (&u)[4][Rule<K>::NM], const T (&geo)[NG]) {
    constexpr int NM = Rule<K>::NM;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        L.avg[v][s] = avg[v];
#pragma unroll
        for (int l = 1; l < NM; ++l) L.hi[v][l - 1][s] = u[v][l];
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) L.geo[g][s] = geo[g];
}
// the geometry entries of cell c (byte offset c8) in the bulk type
template <typename T, int NG>
__device__ __forceinline__ void geo_of(const MView& mv, unsigned c8, T (&geo)[NG]) {
#pragma unroll
    for (int g = 0; g < 4; ++g) geo[g] = (T)mv.J(g, c8);
    if constexpr (NG == 5) geo[4] = (T)mv.A(c8);
}
// The neighbour across an interior edge with llink value ll: its averages, modes and
// geometry, from the tile image or, beyond the halo cap, from global memory.
template <int K, typename T, int NG>
__device__ __forceinline__ void nb_get(const TileLds<K, T, NG>& L, int ll, const SView<Rule<K>::NM, T>& sv,
                                       const MView& mv, double (&avg)[4], T (&u)[4][Rule<K>::NM], T (&geo)[NG]) {
    constexpr int NM = Rule<K>::NM;
    if (ll & kLinkGlobal) {
        const int cell = (ll & ~kLinkGlobal) >> 3;
        load_cell<NM, T>(sv, cell, avg, u);
        geo_of<T, NG>(mv, (unsigned)cell * 8u, geo);
    } else {
        const int s = (ll >> 3) & kLinkSlotMask;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            avg[v] = L.avg[v][s];
            u[v][0] = (T)avg[v];
#pragma unroll
            for (int l = 1; l < NM; ++l) u[v][l] = L.hi[v][l - 1][s];
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) geo[g] = L.geo[g][s];
    }
}
// The residual's halo cell (hc >= 0): its loads, then its slot kTileCells + threadIdx.x
// of the modal image.
template <int K, typename T, int NG>
struct HaloCellG {
    double avg[4];
    T u[4][Rule<K>::NM];
    T geo[NG];
};
template <int K, typename T, int NG>
__device__ __forceinline__ void halo_load_g(HaloCellG<K, T, NG>& h, int hc, const SView<Rule<K>::NM, T>& sv,
                                            const MView& mv) {
    if (hc >= 0) {
        load_cell<Rule<K>::NM, T>(sv, hc, h.avg, h.u);
        geo_of<T, NG>(mv, (unsigned)hc * 8u, h.geo);
    }
}
template <int K, typename T, int NG>
__device__ __forceinline__ void halo_put_g(TileLds<K, T, NG>& L, const HaloCellG<K, T, NG>& h, int hc) {
    if (hc >= 0) stage_put<K, T, NG>(L, kTileCells + (int)threadIdx.x, h.avg, h.u, h.geo);
}

// P2 physical Hessian (xx, xy, yy) of one variable with modes u[0..5] (constant per
// cell): J^-T H_ref J^-1 with H_ref = (48 u3, 24 u3 + 20 u4, 8 u3 + 20 u4 + 20 u5)
template <typename T>
__device__ __forceinline__ void hessian(const T* u, T xx, T xy, T ex, T ey, T (&h)[3]) {
    const T hxx = (T)48.0 * u[3];
    const T hxe = fma((T)24.0, u[3], (T)20.0 * u[4]);
    const T hee = fma((T)8.0, u[3], (T)20.0 * (u[4] + u[5]));
    const T ax = fma(hxx, xx, hxe * ex), ae = fma(hxe, xx, hee * ex);   // (H_ref J^-1) column x
    const T bx = fma(hxx, xy, hxe * ey), be = fma(hxe, xy, hee * ey);   // column y
    h[0] = fma(xx, ax, ex * ae);
    h[1] = fma(xy, ax, ey * ae);
    h[2] = fma(xy, bx, ey * be);
}

// The filter's tile image: every cell's polynomial as physical monomials about its
// vertex 0 (the reference origin), u(x0 + X) = c0 + cX X + cY Y + cXX X^2 +
// cXY X Y + cYY Y^2 per variable (P2; P1 stops at the linear part), and
// the edge vectors d1 = x1 - x0, d2 = x2 - x0 that place its other two vertices.
// Values, physical gradients and the (constant) Hessian at a vertex then cost a
// few FMAs each, which is most of what the OE's jumps need; a slot takes as many
// bytes as modes plus J^-1 would.  FP64: c0 is the whole value at x0; mixed: c0
// is the higher modes' part (float) and the FP64 averages sit beside it, so a
// value jump is the FP64 difference of the averages plus the float one of the rest.
template <int K, typename T>
struct MonoLds {
    static constexpr int NC = K == 2 ? 6 : 3, S = kTileCells + kHaloCap;
    static constexpr bool kMixed = std::is_same<T, float>::value;
    double avg[kMixed ? 4 : 1][kMixed ? S : 1];
    T c[4][NC][S];
    T d[4][S];
};

// whether the cell receives the filter's edge work of this link from its partner: an
// in-tile edge that the partner owns (kLinkRecv is not a flag of global links, whose
// neighbour index covers that bit)
__device__ __forceinline__ bool link_recv(int ll) { return ll >= 0 && !(ll & kLinkGlobal) && (ll & kLinkRecv); }
// The filter's OE records: the damping rates that a lane forms for a partner cell
// (per variable, degree m - 1 and the partner's local edge, at the partner's slot),
// written over the image once no lane reads it any more.
template <int K, typename T>
__device__ __forceinline__ T (&oe_records(MonoLds<K, T>& L))[4][K][3][kTileCells] {
    static_assert(sizeof(T[4][K][3][kTileCells]) <= sizeof(MonoLds<K, T>), "records fit in the image");
    return *reinterpret_cast<T(*)[4][K][3][kTileCells]>(&L);
}

// the monomials of one variable (modes u, u[0] its average in T) from J^-1; with
// `full`, c0 includes the average
template <int K, typename T>
__device__ __forceinline__ void to_mono(const T (&u)[Rule<K>::NM], T xx, T xy, T ex, T ey, bool full,
                                        T (&c)[MonoLds<K, T>::NC]) {
    T a, dx, de;
    vertex_eval_ct<K, 0, T>(u, a, dx, de);
    c[0] = full ? u[0] + a : a;
    c[1] = fma(dx, xx, de * ex);
    c[2] = fma(dx, xy, de * ey);
    if constexpr (K == 2) {
        T h[3];
        hessian(u, xx, xy, ex, ey, h);
        c[3] = (T)0.5 * h[0];
        c[4] = h[1];
        c[5] = (T)0.5 * h[2];
    }
}
// d1 = J e1, d2 = J e2 from J^-1 = [[xx, xy], [ex, ey]]
template <typename T>
__device__ __forceinline__ void edge_vectors(T xx, T xy, T ex, T ey, T (&d)[4]) {
    const T id = Fp<T>::rcp(fma(xx, ey, -(xy * ex)));
    d[0] = ey * id;
    d[1] = -(ex * id);
    d[2] = -(xy * id);
    d[3] = xx * id;
}
// the offset P = (X, Y) of vertex vt (0, 1, 2; a per-lane index) from vertex 0 of a
// cell with edge vectors d
template <typename T>
__device__ __forceinline__ void vertex_point(const T (&d)[4], int vt, T (&P)[2]) {
    P[0] = vt == 0 ? (T)0.0 : (vt == 1 ? d[0] : d[2]);
    P[1] = vt == 0 ? (T)0.0 : (vt == 1 ? d[1] : d[3]);
}
// unit outward normal and length of local edge e (counter-clockwise, from vertex
// e+1 to e+2) of a cell with edge vectors d
template <typename T>
__device__ __forceinline__ void edge_normal(const T (&d)[4], int e, T& nx, T& ny, T& len) {
    T A[2], B[2];
    vertex_point(d, (e + 1) % 3, A);
    vertex_point(d, (e + 2) % 3, B);
    const T dx = B[0] - A[0], dy = B[1] - A[1];
    len = Fp<T>::sqrt(fma(dx, dx, dy * dy));
    const T il = Fp<T>::rcp(len);
    nx = dy * il;
    ny = -(dx * il);
}
// value (c0's part of it) and physical gradient at offset P
template <int K, typename T>
__device__ __forceinline__ void mono_at(const T (&c)[MonoLds<K, T>::NC], const T (&P)[2], T& val, T& gx, T& gy) {
    if constexpr (K == 2) {
        val = fma(P[0], fma(c[3], P[0], fma(c[4], P[1], c[1])), fma(P[1], fma(c[5], P[1], c[2]), c[0]));
        gx = fma(c[3], P[0] + P[0], fma(c[4], P[1], c[1]));
        gy = fma(c[5], P[1] + P[1], fma(c[4], P[0], c[2]));
    } else {
        val = fma(c[2], P[1], fma(c[1], P[0], c[0]));
        gx = c[1];
        gy = c[2];
    }
}
// a cell's slot of the image from its FP64 averages, modes and J^-1
template <int K, typename T>
__device__ __forceinline__ void mono_put(MonoLds<K, T>& L, int s, const double (&avg)[4],
                                         const T (&u)[4][Rule<K>::NM], const T (&geo)[4]) {
    constexpr int NC = MonoLds<K, T>::NC;
    constexpr bool kMixed = MonoLds<K, T>::kMixed;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        T c[NC];
        to_mono<K, T>(u[v], geo[0], geo[1], geo[2], geo[3], !kMixed, c);
        if constexpr (kMixed) L.avg[v][s] = avg[v];
#pragma unroll
        for (int k = 0; k < NC; ++k) L.c[v][k][s] = c[k];
    }
    T d[4];
    edge_vectors(geo[0], geo[1], geo[2], geo[3], d);
#pragma unroll
    for (int k = 0; k < 4; ++k) L.d[k][s] = d[k];
}
// The halo cell that thread threadIdx.x stages for a tile (halo index threadIdx.x),
// or -1.  Read one tile ahead, so that staging a tile waits on one round trip.
static_assert(kHaloCap <= kPassThreads, "one halo cell per thread");
__device__ __forceinline__ int halo_cell_of(const StageArgs& a, int tile) {
    const int h0 = a.m.halo_ptr[tile], hn = a.m.halo_ptr[tile + 1] - h0;
    return (int)threadIdx.x < hn ? a.m.halo_cell[h0 + (int)threadIdx.x] : -1;
}
// this thread's halo cell (hc >= 0): its loads, then its slot kTileCells + threadIdx.x
template <int K, typename T>
struct HaloCell {
    double avg[4];
    T u[4][Rule<K>::NM];
    T geo[4];
};
template <int K, typename T>
__device__ __forceinline__ void halo_load(HaloCell<K, T>& h, int hc, const SView<Rule<K>::NM, T>& sv,
                                          const MView& mv) {
    if (hc >= 0) {
        load_cell<Rule<K>::NM, T>(sv, hc, h.avg, h.u);
        geo_of<T, 4>(mv, (unsigned)hc * 8u, h.geo);
    }
}
template <int K, typename T>
__device__ __forceinline__ void halo_put(MonoLds<K, T>& L, const HaloCell<K, T>& h, int hc) {
    if (hc >= 0) mono_put<K, T>(L, kTileCells + (int)threadIdx.x, h.avg, h.u, h.geo);
}
// Running reductions of a pass workgroup over its tiles: after each tile every wave
// reduces its lanes' contributions (one cell each) and lane 0 combines the result
// into its wave's entry; the flush combines the waves in order.  op(k): 0 sum,
// 1 min, 2 max.  Two sets of entries, used by alternate tiles of a batched pass
// (each tile is a group with a record of its own): a set is reset again two tiles
// later, after a barrier that every wave reaches only once the flush has read it.
template <int NC>
struct WaveAcc {
    double x[2][kPassThreads / 64][NC];
};
__device__ __forceinline__ double acc_op(int op, double a, double b) {
    return op == 0 ? a + b : (op == 1 ? fmin(a, b) : fmax(a, b));
}
__device__ __forceinline__ double acc_ident(int op) { return op == 0 ? 0.0 : (op == 1 ? INFINITY : -INFINITY); }
template <int NC>
__device__ __forceinline__ void wave_acc_reset(WaveAcc<NC>& W, const int (&ops)[NC], int par) {
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) W.x[par][threadIdx.x >> 6][k] = acc_ident(ops[k]);
    }
}
// A sum column that is zero in every lane (counts and boundary fluxes, mostly) skips
// its reduction.
template <int NC>
__device__ __forceinline__ void wave_acc_add(WaveAcc<NC>& W, const int (&ops)[NC], const double (&val)[NC], int par) {
    double r[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if (ops[k] == 0)
            r[k] = __builtin_amdgcn_ballot_w64(val[k] != 0.0) != 0 ? wave_sum(val[k]) : 0.0;
        else
            r[k] = ops[k] == 1 ? wave_min(val[k]) : wave_max(val[k]);
    }
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < NC; ++k) W.x[par][w][k] = acc_op(ops[k], W.x[par][w][k], r[k]);
    }
}
// Writes entry k of the record to dst[col[k] * stride], dst the record's column 0
// and col[k] < kPartCols the absolute column (call with every thread).  sync: the
// workgroup synchronises before (the entries are complete) and after (they may be
// reset); a batched pass's tile already ends with a barrier and alternates sets.
template <int NC>
__device__ __forceinline__ void wave_acc_flush(const WaveAcc<NC>& W, const int (&ops)[NC], const int (&col)[NC],
                                               double* dst, size_t stride, int par, bool sync) {
    if (sync) __syncthreads();
    const int t = threadIdx.x;
    if (t < NC) {
        int op = 0, cl = 0;
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k == t) {
                op = ops[k];
                cl = col[k];
            }
        double v = W.x[par][0][t];
#pragma unroll
        for (int w = 1; w < kPassThreads / 64; ++w) v = acc_op(op, v, W.x[par][w][t]);
        dst[(size_t)cl * stride] = v;
    }
    if (sync) __syncthreads();
}

// Persistent walk of a pass: workgroup b takes its XCD's tiles in turn (single
// instance), or the tiles (= reduction groups) of its chunks (batch); body(tile, hc,
// par) computes one tile and ends with a barrier, hc the halo cell this thread
// stages for it, read while the previous tile was computed, par the set of
// reduction entries; flush(g, par) writes the record of group g (batch) or of the
// workgroup (g < 0).
template <bool kBatch, typename Body, typename Reset, typename Flush>
__device__ __forceinline__ void walk_tiles(const StageArgs& a, int g0, int g1, Body body, Reset reset, Flush flush) {
    if constexpr (!kBatch) {
        reset(0);
        const TileWalk tw = tile_walk(n_tiles_of(a.m.n_cell));
        int hc = tw.first < tw.end ? halo_cell_of(a, tw.first) : -1;
        for (int tile = tw.first; tile < tw.end; tile += tw.stride) {
            const int hn = tile + tw.stride < tw.end ? halo_cell_of(a, tile + tw.stride) : -1;
            body(tile, hc, 0);
            hc = hn;
        }
        flush(-1, 0);
    } else {
        int hc = g0 < g1 ? halo_cell_of(a, g0) : -1;
        for (int gi = g0; gi < g1; ++gi) {
            const int hn = gi + 1 < g1 ? halo_cell_of(a, gi + 1) : -1;
            const int par = (gi - g0) & 1;
            reset(par);
            body(gi, hc, par);
            flush(gi, par);
            hc = hn;
        }
    }
}

// ------------------------------------------------------------------------- pass 1: residual

constexpr int kResCols = 14;   // sums, minima, maxima (4 each), |m - mbar|^2 max, bad averages
__device__ constexpr int kResOps[kResCols] = {0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2, 2, 0};

// Img: TileLds<K, T, 5> (the modal image: averages, modes and geometry, the
// neighbour's traces from the basis rows er) or MonoLds<K, T> (monomials and edge
// vectors); the batched FP64 P2 pass takes the second, the others the first.
template <int K, typename T, bool kBatch, typename Img>
__device__ __forceinline__ void residual_run(const StageArgs& a, int g0, int g1, const EdgeRowsLds<K, T>& er, Img& L,
                                             WaveAcc<kResCols>& W) {
    constexpr bool kMono = std::is_same<Img, MonoLds<K, T>>::value;
    using R = Rule<K>;
    constexpr int NM = R::NM, NE = R::NE;
    constexpr bool kMixed = std::is_same<T, float>::value;
    const Glob* g = a.g;
    const int nc = a.m.n_cell;
    const T gm1 = (T)(a.gamma - 1.0);
    const double alpha = g->alpha, dt = g->dt;
    const double sa = a.stage == 0 ? 0.0 : (a.stage == 1 ? 0.75 : 1.0 / 3.0);
    const double sb = a.stage == 0 ? 1.0 : (a.stage == 1 ? 0.25 : 2.0 / 3.0);
    const SView<NM, T> up = sview<NM, T>(a.uin, a);
    const SView<NM, T> u0p = sview<NM, T>(a.u0, a);
    const SView<NM, T> wp = sview<NM, T>(a.w, a);
    const MView mv = mview(a.m);
    const Tab<K, T>& TB = tab<K, T>();
    const Tab<K, double>& TD = tab<K, double>();
    int ops[kResCols], cols[kResCols];
#pragma unroll
    for (int k = 0; k < kResCols; ++k) {
        ops[k] = kResOps[k];
        cols[k] = k == kResCols - 1 ? kColBad : k;
    }
    // The domain average of the momentum of the state this pass writes, known before
    // it is written: the discrete divergence form conserves sum_K |K| ubar_K up to
    // the flux through the boundary (each interior edge's flux enters its two cells
    // with opposite signs, exactly: see the surface term), so
    //   sum |K| mbar(w) = sa sum |K| mbar(u^n) + sb (sum |K| mbar(u_in) - dt (A + alpha B))
    // with the sums and the boundary flux A + alpha B of the inputs recorded by the
    // filter pass that produced them (sa = 0, sb = 1 in the first stage).  The pass
    // then forms ||| m - mbar |||_inf of eq. normOmg at its own volume points, which
    // saves a pass over the state.
    double mb[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const bool first = a.stage == 0;
        const double s_in = first ? g->mom_n[j] : g->mom_c[j];
        const double b_in = first ? g->bfa_n[j] + alpha * g->bfb_n[j] : g->bfa_c[j] + alpha * g->bfb_c[j];
        const double s_w = s_in - dt * b_in;
        mb[j] = uniform((first ? s_w : sa * g->mom_n[j] + sb * s_w) / g->area_sum);
    }

    auto tile_body = [&](int tile, int hc, int par) __attribute__((always_inline)) {
        const int c = tile * kTileCells + (int)threadIdx.x;
        const bool live = c < nc;
        const unsigned c8 = (unsigned)c * 8u, c4 = (unsigned)c * 4u, cT = (unsigned)c * (unsigned)sizeof(T);
        // the own cell (registers and the tile image), then the halo
        double ua[4];
        T u[4][NM];
        T geo[5];
        int lk[3];
        // both cells' loads are in flight before either is written to the image
        if constexpr (kMono) {
            HaloCell<K, T> hcell;
            halo_load<K, T>(hcell, hc, up, mv);
            if (live) {
                load_cell<NM, T>(up, c, ua, u);
                geo_of<T, 5>(mv, c8, geo);
#pragma unroll
                for (int i = 0; i < 3; ++i) lk[i] = bld<int>(mv.llink, c4, (unsigned)i * mv.n4);
                mono_put<K, T>(L, threadIdx.x, ua, u, reinterpret_cast<const T(&)[4]>(geo));
            }
            halo_put<K, T>(L, hcell, hc);
        } else {
            HaloCellG<K, T, 5> hcell;
            halo_load_g<K, T, 5>(hcell, hc, up, mv);
            if (live) {
                load_cell<NM, T>(up, c, ua, u);
                geo_of<T, 5>(mv, c8, geo);
#pragma unroll
                for (int i = 0; i < 3; ++i) lk[i] = bld<int>(mv.llink, c4, (unsigned)i * mv.n4);
                stage_put<K, T, 5>(L, threadIdx.x, ua, u, geo);
            }
            halo_put_g<K, T, 5>(L, hcell, hc);
        }
        __syncthreads();
        double part[kResCols];
#pragma unroll
        for (int k = 0; k < kResCols; ++k) part[k] = acc_ident(kResOps[k]);
        // mode 0 accumulates in FP64 in both forms (its volume term is zero)
        double r0[4] = {0.0, 0.0, 0.0, 0.0};
        T r[4][NM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) r[v][l] = (T)0.0;
        double area = 0.0;
        if (live) {
            const T xx = geo[0], xy = geo[1], ex = geo[2], ey = geo[3], areaT = geo[4];
            area = mv.A(c8);

            // volume term |K| sum_mu w_mu F(u).grad Psi_l with grad Psi = J^{-T} grad_ref Psi,
            // i.e. dPsi/dxi (F.grad xi) + dPsi/deta (F.grad eta)
#pragma unroll
            for (int m = 0; m < R::NQ; ++m) {
                T q[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) q[v] = dot<NM>(u[v], TB.vp[m]);
                T ir, p;
                euler_ip(q, gm1, ir, p);
                const T wa = TB.vw[m] * areaT;
                T g1[4], g2[4];
                euler_flux_n(q, ir, p, wa * xx, wa * xy, g1);
                euler_flux_n(q, ir, p, wa * ex, wa * ey, g2);
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int l = 1; l < NM; ++l)
                        r[v][l] = fma(TB.vdx[m][l], g1[v], fma(TB.vde[m][l], g2[v], r[v][l]));
            }

            if constexpr (kMono) {
                // surface term - sum_i l_i sum_nu w_nu Fhat(u_int, u_ext, n_i) Psi_l.  Both
                // cells of an interior edge form Fhat with the scaled normal l n of the
                // lower-index cell ("low") and l = |l n|, from the same two traces in
                // commuted order, so their contributions are exact negatives (sgn = +1 on the
                // low side):  Fhat_low = 1/2 (F(u_i).n + F(u_e).n - sgn alpha l (u_e - u_i)),
                // and the own cell adds -sgn w_nu Fhat_low Psi_l.  Every trace comes from the
                // cell's monomials in the tile image at its own offset of the Gauss point,
                // and every scaled normal from its edge vectors (l n = (dy, -dx) along the
                // counter-clockwise edge), by the same arithmetic whichever lane asks.
                constexpr int NC = MonoLds<K, T>::NC;
                T od[4];
    #pragma unroll
                for (int k2 = 0; k2 < 4; ++k2) od[k2] = L.d[k2][threadIdx.x];
                // the Gauss points of local edge e of a cell with edge vectors d: from
                // vertex e+1 towards e+2, parameter s_nu
                auto edge_pts = [&](const T (&d)[4], int e, T (&P)[NE][2], T& lnx, T& lny) __attribute__((always_inline)) {
                    T A[2], B[2];
                    vertex_point(d, (e + 1) % 3, A);
                    vertex_point(d, (e + 2) % 3, B);
                    const T dx = B[0] - A[0], dy = B[1] - A[1];
                    lnx = dy;
                    lny = -dx;
    #pragma unroll
                    for (int nu = 0; nu < NE; ++nu) {
                        P[nu][0] = fma((T)R::s[nu], dx, A[0]);
                        P[nu][1] = fma((T)R::s[nu], dy, A[1]);
                    }
                };
                auto trace = [&](const T (&cf)[NC], const T (&P)[2], T avg) __attribute__((always_inline)) {
                    T val, g0, g1;
                    mono_at<K, T>(cf, P, val, g0, g1);
                    return kMixed ? avg + val : val;
                };
    #pragma unroll 1
                for (int i = 0; i < 3; ++i) {
                    const int ll = i == 0 ? lk[0] : (i == 1 ? lk[1] : lk[2]);
                    const bool has = ll >= 0;
                    const bool wall = ll == kLinkWall;
                    const int j = has ? (ll & 3) : i;
                    const bool low = !has || (ll & 4) != 0;
                    const T sgn = low ? (T)1.0 : (T)-1.0;
                    T Po[NE][2], lnx_o, lny_o;
                    edge_pts(od, i, Po, lnx_o, lny_o);
                    // the own traces, then the neighbour's (the own cell's at a boundary,
                    // replaced below); the neighbour runs the shared edge the other way, so
                    // its point for nu is its own point NE-1-nu (symmetric Gauss nodes)
                    T qi[NE][4], qe[NE][4];
                    T lnx_n = lnx_o, lny_n = lny_o;
                    auto own_traces = [&]() __attribute__((always_inline)) {
    #pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            T co[NC];
    #pragma unroll
                            for (int k2 = 0; k2 < NC; ++k2) co[k2] = L.c[v][k2][threadIdx.x];
    #pragma unroll
                            for (int nu = 0; nu < NE; ++nu) qi[nu][v] = trace(co, Po[nu], u[v][0]);
                        }
                    };
                    own_traces();
                    if (has) {
                        auto nb_traces = [&](auto&& nbc, const T (&dn)[4]) __attribute__((always_inline)) {
                            T Pn[NE][2];
                            edge_pts(dn, j, Pn, lnx_n, lny_n);
    #pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                T cn[NC], na;
                                nbc(v, na, cn);
    #pragma unroll
                                for (int nu = 0; nu < NE; ++nu) qe[nu][v] = trace(cn, Pn[NE - 1 - nu], na);
                            }
                        };
                        if (ll & kLinkGlobal) {
                            // beyond the halo cap: the neighbour's coefficients from global memory
                            const int cell = (ll & ~kLinkGlobal) >> 3;
                            const unsigned n8 = (unsigned)cell * 8u, nT = (unsigned)cell * (unsigned)sizeof(T);
                            const T nxx = (T)mv.J(0, n8), nxy = (T)mv.J(1, n8), nex = (T)mv.J(2, n8), ney = (T)mv.J(3, n8);
                            T dn[4];
                            edge_vectors(nxx, nxy, nex, ney, dn);
                            nb_traces(
                                [&](int v, T& na, T (&cn)[NC]) __attribute__((always_inline)) {
                                    T un[NM];
                                    const double a0 = up.a(v, n8);
                                    un[0] = (T)a0;
    #pragma unroll
                                    for (int l = 1; l < NM; ++l) un[l] = up.h(v, l, nT);
                                    to_mono<K, T>(un, nxx, nxy, nex, ney, !kMixed, cn);
                                    na = un[0];
                                },
                                dn);
                        } else {
                            const int sl = (ll >> 3) & kLinkSlotMask;
                            T dn[4];
    #pragma unroll
                            for (int k2 = 0; k2 < 4; ++k2) dn[k2] = L.d[k2][sl];
                            nb_traces(
                                [&](int v, T& na, T (&cn)[NC]) __attribute__((always_inline)) {
                                    na = kMixed ? (T)L.avg[kMixed ? v : 0][kMixed ? sl : 0] : (T)0.0;
    #pragma unroll
                                    for (int k2 = 0; k2 < NC; ++k2) cn[k2] = L.c[v][k2][sl];
                                },
                                dn);
                        }
                    }
                    const T lnx = low ? lnx_o : lnx_n, lny = low ? lny_o : lny_n;
                    const T lc = Fp<T>::sqrt(fma(lnx, lnx, lny * lny));   // the edge length, from the same bits on both sides
                    const T al = (T)alpha * lc;
                    // unit normal of a reflective wall (own edge, so own is low)
                    const T il = Fp<T>::rcp(lc);
                    const T nxu = lnx * il, nyu = lny * il;
    #pragma unroll
                    for (int nu = 0; nu < NE; ++nu) {
                        const T* p = TB.ep[i * NE + nu];
                        if (!has) {
                            // transmissive: the exterior trace is the interior one; reflective:
                            // its normal momentum reversed, m - 2 (m.n) n
                            const T mn2 = (T)-2.0 * fma(qi[nu][1], nxu, qi[nu][2] * nyu);
                            qe[nu][0] = qi[nu][0];
                            qe[nu][1] = wall ? fma(mn2, nxu, qi[nu][1]) : qi[nu][1];
                            qe[nu][2] = wall ? fma(mn2, nyu, qi[nu][2]) : qi[nu][2];
                            qe[nu][3] = qi[nu][3];
                        }
                        T iri, pi, ire, pe;
                        euler_ip(qi[nu], gm1, iri, pi);
                        euler_ip(qe[nu], gm1, ire, pe);
                        T fi[4], fe[4];
                        euler_flux_n(qi[nu], iri, pi, lnx, lny, fi);
                        euler_flux_n(qe[nu], ire, pe, lnx, lny, fe);
                        const T wsn = (T)R::ws[nu];
    #pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const T d = qe[nu][v] - qi[nu][v];
                            const T fh = sgn * (wsn * ((T)0.5 * ((fi[v] + fe[v]) - sgn * (al * d))));
                            r0[v] -= (double)fh;
    #pragma unroll
                            for (int l = 1; l < NM; ++l) r[v][l] = fma(-fh, p[l], r[v][l]);
                        }
                    }
                }
            } else {
                // surface term - sum_i l_i sum_nu w_nu Fhat(u_int, u_ext, n_i) Psi_l.  Both
                // cells of an interior edge form Fhat with the scaled normal l n of the
                // lower-index cell ("low") and l = |l n|, from the same two traces in
                // commuted order, so their contributions are exact negatives (sgn = +1 on the
                // low side):  Fhat_low = 1/2 (F(u_i).n + F(u_e).n - sgn alpha l (u_e - u_i)),
                // and the own cell adds -sgn w_nu Fhat_low Psi_l.
    #pragma unroll 1
                for (int i = 0; i < 3; ++i) {
                    const int ll = i == 0 ? lk[0] : (i == 1 ? lk[1] : lk[2]);
                    const bool has = ll >= 0;
                    const bool wall = ll == kLinkWall;
                    const int j = has ? (ll & 3) : i;
                    const bool low = !has || (ll & 4) != 0;
                    const T sgn = low ? (T)1.0 : (T)-1.0;
                    // the neighbour (the own cell at a boundary, replaced below)
                    double una[4];
                    T un[4][NM];
                    T ng[5];
                    if (has) {
                        nb_get<K, T, 5>(L, ll, up, mv, una, un, ng);
                    } else {
    #pragma unroll
                        for (int v = 0; v < 4; ++v)
    #pragma unroll
                            for (int l = 0; l < NM; ++l) un[v][l] = u[v][l];
    #pragma unroll
                        for (int k2 = 0; k2 < 5; ++k2) ng[k2] = geo[k2];
                    }
                    // the exterior trace at the edge's Gauss points: the neighbour runs the
                    // shared edge the other way, so its parameter is 1 - s_nu = s_{NE-1-nu}
                    // (symmetric Gauss nodes)
                    T qe[NE][4];
    #pragma unroll
                    for (int v = 0; v < 4; ++v)
    #pragma unroll
                        for (int nu = 0; nu < NE; ++nu) qe[nu][v] = dot<NM>(un[v], er.r[j * NE + NE - 1 - nu]);
                    T lnx_o, lny_o, lnx_n, lny_n;
                    scaled_normal(xx, xy, ex, ey, areaT, i, lnx_o, lny_o);
                    scaled_normal(ng[0], ng[1], ng[2], ng[3], ng[4], j, lnx_n, lny_n);
                    const T lnx = low ? lnx_o : lnx_n, lny = low ? lny_o : lny_n;
                    const T lc = Fp<T>::sqrt(fma(lnx, lnx, lny * lny));   // the edge length, from the same bits on both sides
                    const T al = (T)alpha * lc;
                    // unit normal of a reflective wall (own edge, so own is low)
                    const T il = Fp<T>::rcp(lc);
                    const T nxu = lnx * il, nyu = lny * il;
    #pragma unroll
                    for (int nu = 0; nu < NE; ++nu) {
                        const T* p = TB.ep[i * NE + nu];
                        T qi[4];
    #pragma unroll
                        for (int v = 0; v < 4; ++v) qi[v] = dot<NM>(u[v], p);
                        if (!has) {
                            // transmissive: the exterior trace is the interior one; reflective:
                            // its normal momentum reversed, m - 2 (m.n) n
                            const T mn2 = (T)-2.0 * fma(qi[1], nxu, qi[2] * nyu);
                            qe[nu][0] = qi[0];
                            qe[nu][1] = wall ? fma(mn2, nxu, qi[1]) : qi[1];
                            qe[nu][2] = wall ? fma(mn2, nyu, qi[2]) : qi[2];
                            qe[nu][3] = qi[3];
                        }
                        T iri, pi, ire, pe;
                        euler_ip(qi, gm1, iri, pi);
                        euler_ip(qe[nu], gm1, ire, pe);
                        T fi[4], fe[4];
                        euler_flux_n(qi, iri, pi, lnx, lny, fi);
                        euler_flux_n(qe[nu], ire, pe, lnx, lny, fe);
                        const T wsn = (T)R::ws[nu];
    #pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const T d = qe[nu][v] - qi[v];
                            const T fh = sgn * (wsn * ((T)0.5 * ((fi[v] + fe[v]) - sgn * (al * d))));
                            r0[v] -= (double)fh;
    #pragma unroll
                            for (int l = 1; l < NM; ++l) r[v][l] = fma(-fh, p[l], r[v][l]);
                        }
                    }
                }
            }
        }
        // the tile's last read of the image: from here a wave may go on to the next
        // tile (a batched tile keeps its barrier at the end, before its record flush)
        if constexpr (!kBatch) __syncthreads();
        if (live) {
            // diagonal mass a_K^(l) = |K| (a_l/|K|), then the SSP-RK3 combination; the
            // average in FP64, the higher modes in the bulk type
            const double ia = frcp(area);
            double wavg[4];   // the pre-filter averages
            T w[4][NM];
            const T iaT = (T)ia, dtT = (T)dt, saT = (T)sa, sbT = (T)sb;
            // u^n of the second and third stages, all its loads in flight together
            double una[4] = {0.0, 0.0, 0.0, 0.0};
            T unh[4][NM] = {};
            if (a.stage != 0) load_cell<NM, T>(u0p, c, una, unh);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double adv0 = fma(dt, r0[v] * ia, ua[v]);
                const double w0 = a.stage == 0 ? adv0 : fma(sa, una[v], sb * adv0);
                wp.put_a(v, c8, w0);
                part[v] = area * w0;
                wavg[v] = w0;
                w[v][0] = (T)w0;
#pragma unroll
                for (int l = 1; l < NM; ++l) {
                    const T adv = fma(dtT, r[v][l] * iaT * (T)kInvMass[l], u[v][l]);
                    const T wl = a.stage == 0 ? adv : fma(saT, unh[v][l], sbT * adv);
                    w[v][l] = wl;
                    wp.put_h(v, l, cT, wl);
                }
            }
            if (a.bp_enable) {
                // the OE filter and the limiter keep every average: an inadmissible one
                // here ends the step's attempt (it is retried with half the time step)
                const double q0 = wavg[0], q1 = wavg[1], q2 = wavg[2], q3 = wavg[3];
                if (!(q0 > 0.0 && q3 - 0.5 * (q1 * q1 + q2 * q2) / q0 > 0.0)) part[13] = 1.0;
            }
            // min/max of every variable and |m - mbar|^2 at the volume points, in FP64: the
            // average plus the higher modes' part (formed in the bulk type), so a small
            // deviation from the domain average is not lost to the bulk type's rounding
            double cnm = 0.0;
#pragma unroll 1
            for (int m = 0; m < R::NQ; ++m) {
                double q[4], hv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if constexpr (kMixed) {
                        hv[v] = (double)dot_hi<NM>(w[v], TB.vp[m]);
                        q[v] = wavg[v] + hv[v];
                    } else {
                        q[v] = dot<NM>(w[v], TD.vp[m]);
                    }
                    part[4 + v] = fmin(part[4 + v], q[v]);
                    part[8 + v] = fmax(part[8 + v], q[v]);
                }
                double d1, d2;
                if constexpr (kMixed) {
                    d1 = (wavg[1] - mb[0]) + hv[1];
                    d2 = (wavg[2] - mb[1]) + hv[2];
                } else {
                    d1 = q[1] - mb[0];
                    d2 = q[2] - mb[1];
                }
                cnm = fmax(cnm, fma(d1, d1, d2 * d2));
            }
            part[12] = cnm;
        }
        wave_acc_add<kResCols>(W, ops, part, par);
        // a batched tile's record is flushed next, and the image rewritten by the next tile
        if constexpr (kBatch) __syncthreads();
    };
    walk_tiles<kBatch>(
        a, g0, g1, tile_body, [&](int par) { wave_acc_reset<kResCols>(W, ops, par); },
        [&](int gi, int par) {
            if (gi < 0) wave_acc_flush<kResCols>(W, ops, cols, a.part + blockIdx.x, kMaxBlocks, par, true);
            else wave_acc_flush<kResCols>(W, ops, cols, a.part + a.gbase + gi, a.gstride, par, false);
        });
}

template <int K, typename T>
__global__ __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(OEDG_RES_WAVES))) void k_residual(
    StageArgs a) {
    if (!a.g->active || a.g->skip) return;
    __shared__ EdgeRowsLds<K, T> er;
    __shared__ TileLds<K, T, 5> L;
    __shared__ WaveAcc<kResCols> W;
    fill_edge_rows<K, T>(er);
    __syncthreads();
    residual_run<K, T, false>(a, 0, 0, er, L, W);
}

// Batched passes: workgroup b walks its XCD's range of the chunk table; each
// chunk is a run of reduction groups [g0, g1) (tiles) of instance desc[chunk.inst],
// given to run(a, g0, g1).
template <typename F>
__device__ __forceinline__ void for_each_chunk(const StageArgs* desc, const Chunk* chunks, const ChunkSplit& cs,
                                               F run) {
    const TileWalk w = chunk_walk(cs);
    for (int ci = w.first; ci < w.end; ci += w.stride) {
        const Chunk ch = chunks[ci];
        // read as constant memory (as a kernel's own arguments are): the compiler may
        // load a field again where it would otherwise keep it in registers or spill it
        typedef const __attribute__((address_space(4))) unsigned ConstWord;
        static_assert(sizeof(StageArgs) % 4 == 0, "whole words");
        StageArgs a;
        ConstWord* src = (ConstWord*)(desc + ch.inst);
        unsigned* dst = reinterpret_cast<unsigned*>(&a);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(StageArgs) / 4); ++i) dst[i] = src[i];
        if (!a.g->active || a.g->skip) continue;
        run(a, ch.g0, ch.g1);
    }
}

// Batched passes over the chunks of the members of degree K (a batch of both
// degrees launches each).
template <int K, typename T>
__global__ __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(OEDG_RES_WAVES))) void k_residual_batch(
    const StageArgs* desc, const Chunk* chunks, ChunkSplit cs) {
    // FP64 P2: the monomial image (no slower here, and it spills less in the
    // batched kernel); P1 FP64: the modal image (three waves per SIMD instead of
    // two); mixed: the modal image, whose float traces keep the rounding within the
    // limiter's margin.  The P1 filters ask for three waves as well.
    using Img = typename std::conditional<std::is_same<T, double>::value && K == 2, MonoLds<K, T>, TileLds<K, T, 5>>::type;
    __shared__ EdgeRowsLds<K, T> er;
    __shared__ Img L;
    __shared__ WaveAcc<kResCols> W;
    fill_edge_rows<K, T>(er);
    __syncthreads();
    for_each_chunk(desc, chunks, cs,
                   [&](const StageArgs& a, int g0, int g1) { residual_run<K, T, true>(a, g0, g1, er, L, W); });
}

// ------------------------------------------------------------------------- pass 2: OE, limiter, alpha

// The full state (FP64) at the NP-point limiter node set of a cell with averages
// wa and modes w: the 3Q edge Gauss points, then two extra slots.  Optimal
// decomposition: the P1 vertices v1, v2 (eq. 1944) or the two P2 internal nodes
// (eq. 1139), at reference coordinates (n0x, n0e), (n1x, n1e); with the u* form
// (ustar, P2) both slots hold u*, the mean of the two internal nodes (equal node
// weights).  Classical decomposition (zxs): the slots repeat edge points 0 and 1
// (P1: no internal nodes) or hold u* (P2), which leaves every minimum unchanged.
template <int K, int NM>
__device__ __forceinline__ void node_values(const double (&wd)[4][NM], double n0x, double n0e, double n1x,
                                            double n1e, bool zxs, bool ustar, double (&pv)[3 * Rule<K>::NE + 2][4]) {
    constexpr int NE3 = 3 * Rule<K>::NE;
    const Tab<K, double>& TD = tab<K, double>();
#pragma unroll
    for (int t = 0; t < NE3; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) pv[t][v] = dot<NM>(wd[v], TD.ep[t]);   // edge i = t / NE, node nu = t % NE
    if (zxs) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if constexpr (K == 1) {
                pv[NE3][v] = pv[0][v];
                pv[NE3 + 1][v] = pv[1][v];
            } else {
                pv[NE3][v] = dot<NM>(wd[v], TD.zr);
                pv[NE3 + 1][v] = pv[NE3][v];
            }
        }
    } else {
        double p0[NM], p1[NM];
        psi<K>(n0x, n0e, p0);
        psi<K>(n1x, n1e, p1);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            pv[NE3][v] = dot<NM>(wd[v], p0);
            pv[NE3 + 1][v] = dot<NM>(wd[v], p1);
            if constexpr (K == 2) {
                if (ustar) pv[NE3][v] = pv[NE3 + 1][v] = 0.5 * (pv[NE3][v] + pv[NE3 + 1][v]);
            }
        }
    }
}

__device__ __forceinline__ double internal_energy(const double (&q)[4]) {
    return fma(-0.5 * frcp(q[0]), fma(q[1], q[1], q[2] * q[2]), q[3]);
}

// record of the filter pass: max wave speed, limited, bad and flattened counts,
// sum |K| m1bar, sum |K| m2bar, the boundary momentum flux A_1, A_2, B_1, B_2, and
// the minimum density and pressure over the limiter nodes of the output
constexpr int kFilCols = kFilterCols;
static_assert(kNumPartial + 1 + kFilCols <= kPartCols && kColBad < kPartCols && kResCols == kNumPartial + 2,
              "record columns");
__device__ constexpr int kFilOps[kFilCols] = {2, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1};

template <int K, typename T, bool kBatch>
__device__ __forceinline__ void filter_run(const StageArgs& a, int g0, int g1, MonoLds<K, T>& L,
                                           WaveAcc<kFilCols>& W) {
    using R = Rule<K>;
    using F = Fp<T>;
    constexpr int NM = R::NM;
    constexpr int NE = R::NE;
    constexpr int NP = 3 * NE + 2;   // limiter node set size
    constexpr bool kMixed = std::is_same<T, float>::value;
    const Glob* g = a.g;
    const int nc = a.m.n_cell;
    const double gamma = a.gamma;
    const T gammaT = (T)gamma;
    const bool oe = a.oe_enable && a.stage >= 0;
    const bool ri = a.oe_mode == 0;
    const T dt = (T)g->dt;
    // inverse L-infinity norms (0 in the zero branch of eq. OEScalar:Coef2)
    const T inv0 = (T)g->inv_nrm[0], inv3 = (T)g->inv_nrm[3];
    const T inv1 = (T)(ri ? g->inv_nrm_m : g->inv_nrm[1]), inv2 = (T)(ri ? g->inv_nrm_m : g->inv_nrm[2]);
    const SView<NM, T> wp = sview<NM, T>(a.w, a);
    const SView<NM, T> op = sview<NM, T>(a.uout, a);
    const MView mv = mview(a.m);
    int ops[kFilCols], cols[kFilCols];
#pragma unroll
    for (int k = 0; k < kFilCols; ++k) {
        ops[k] = kFilOps[k];
        cols[k] = kNumPartial + 1 + k;
    }

    auto tile_body = [&](int tile, int hc, int par) __attribute__((always_inline)) {
        const int c = tile * kTileCells + (int)threadIdx.x;
        const bool live = c < nc;
        const unsigned c8 = (unsigned)c * 8u, c4 = (unsigned)c * 4u, cT = (unsigned)c * (unsigned)sizeof(T);
        double wa[4];   // the averages: untouched by the OE (eq. OE:m0) and the limiter
        T w[4][NM];
        T geo[4];
        int lk[3];
        double area_d = 0.0;
        HaloCell<K, T> hcell;
        if (oe) halo_load<K, T>(hcell, hc, wp, mv);
        if (live) {
            load_cell<NM, T>(wp, c, wa, w);
            geo_of<T, 4>(mv, c8, geo);
            area_d = mv.A(c8);
#pragma unroll
            for (int i = 0; i < 3; ++i) lk[i] = bld<int>(mv.llink, c4, (unsigned)i * mv.n4);
            if (oe) mono_put<K, T>(L, threadIdx.x, wa, w, geo);
        }
        if (oe) {
            halo_put<K, T>(L, hcell, hc);
            __syncthreads();
        }
        double part[kFilCols];
#pragma unroll
        for (int k = 0; k < kFilCols; ++k) part[k] = acc_ident(kFilOps[k]);
        const T xx = geo[0], xy = geo[1], ex = geo[2], ey = geo[3];
        T od[4];   // the cell's edge vectors: its edges' lengths and normals
        if (live) edge_vectors(xx, xy, ex, ey, od);

        // OE damping rates: the degree-m modes of variable v decay at the rate
        // sum_{j <= m} sigma^j = inv_v * acc[v][m - 1], where acc sums over the cell's
        // edges beta/h A^{k,j} h^j sqrt(S_j / 2) for j <= m (eq. OEScalar:Coef2; eqs.
        // RIOESys:Coef1/Coef2) and inv_v, the reciprocal of the variable's norm, is the
        // same for every edge
        T acc[4][K];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int m = 0; m < K; ++m) acc[v][m] = (T)0.0;
        if (oe) {
            // Every edge inside the tile is worked once, by its owner (the other side
            // carries kLinkRecv): beta and the jump energies are the same from either
            // side (squares of jumps that change sign, a max over both sides), so the
            // owner forms both cells' rates, each with its own h, and hands the other
            // one its share through the tile's LDS once the image is no longer read.
            // A cell owns at most two in-tile edges (records kept in registers) and
            // every edge to a cell outside the tile.
            constexpr int NC = MonoLds<K, T>::NC;
            T rec[2][4][K];   // rates for the partners of this lane's in-tile edges
            int rto[2] = {-1, -1};   // their record index: local edge * kTileCells + slot
            if (live) {
                const bool own0 = lk[0] >= 0 && !link_recv(lk[0]);
                const bool own1 = lk[1] >= 0 && !link_recv(lk[1]);
                const bool own2 = lk[2] >= 0 && !link_recv(lk[2]);
                const int n_own = (int)own0 + (int)own1 + (int)own2;
                const T area = (T)area_d;
                const T i2a = F::rcp((T)2.0 * area);
                // sum over both ends of the squared jumps of order j: j = 0 value, 1
                // gradient; 2: the Hessian's jump, the same at both ends, weighted by
                // C_2 = (1, 2, 1), i.e. 2 (jxx^2 + 2 jxy^2 + jyy^2)
                auto energies = [&](const T (&jv)[2], const T (&jx)[2], const T (&jy)[2], const T (&dh)[3],
                                    T (&Sv)[K + 1]) __attribute__((always_inline)) {
                    Sv[0] = fma(jv[0], jv[0], jv[1] * jv[1]);
                    Sv[1] = fma(jx[0], jx[0], fma(jy[0], jy[0], fma(jx[1], jx[1], jy[1] * jy[1])));
                    if constexpr (K == 2) Sv[2] = (T)2.0 * fma(dh[0], dh[0], fma((T)2.0 * dh[1], dh[1], dh[2] * dh[2]));
                };
                // delta^j = A^{k,j} h^j / ||.|| sqrt(S_j / 2); a side with h and beta/h = bh
                // adds sum_{j <= m} bh delta^j to the rate of its degree-m modes (the
                // factor 1/||.||, the same for every edge, is applied to the sums)
                auto rates = [&](const T (&Sv)[K + 1], T bh, T h, T (&p)[K]) __attribute__((always_inline)) {
                    T s = bh * ((T)kA[K][0] * F::sqrt((T)0.5 * Sv[0]));
                    T hj = h;
#pragma unroll
                    for (int jj = 1; jj <= K; ++jj) {
                        s = fma(bh * hj, (T)kA[K][jj] * F::sqrt((T)0.5 * Sv[jj]), s);
                        p[jj - 1] = s;
                        hj *= h;
                    }
                };
                int nrec = 0;
#pragma unroll 1
                for (int r = 0; r < n_own; ++r) {
                    // this lane's r-th owned edge
                    const int i = r == 0 ? (own0 ? 0 : (own1 ? 1 : 2)) : ((r == 1 && own0 && own1) ? 1 : 2);
                    const int ll = i == 0 ? lk[0] : (i == 1 ? lk[1] : lk[2]);
                    const int j = ll & 3;
                    T nx, ny, len;
                    edge_normal(od, i, nx, ny, len);
                    const T il = F::rcp(len);
                    const T h = (T)2.0 * area * il, bh_len = len * i2a;   // h_K^(i) = 2|K| / l_i; 1/h = l_i / (2|K|)
                    // The edge's work, with the neighbour's coefficients from the image
                    // or (beyond the halo cap) converted from global memory: two copies of
                    // the code, so that the rare path costs the common one no registers.
                    // partner: the neighbour is a tile cell, whose rates are formed here too
                    auto edge = [&](auto&& nbc, const T (&dn)[4], bool partner) __attribute__((always_inline)) {
                        // the edge's two ends: own vertex i+1, then i+2, meets the
                        // neighbour's vertex j+2, then j+1
                        T Po[2][2], Pn[2][2];
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            vertex_point(od, (i + 1 + e) % 3, Po[e]);
                            vertex_point(dn, (j + 2 - e) % 3, Pn[e]);
                        }
                        // beta^(i): the max spectral radius over both ends of the edge and both
                        // sides, with K's normal, from the four variables' values there
                        T beta = (T)0.0;
                        {
                            T qo[2][4], qn[2][4];
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                T co[NC], cn[NC];
#pragma unroll
                                for (int k2 = 0; k2 < NC; ++k2) co[k2] = L.c[v][k2][threadIdx.x];
                                const T oa = kMixed ? (T)L.avg[kMixed ? v : 0][kMixed ? threadIdx.x : 0] : (T)0.0;
                                double na;
                                nbc(v, na, cn);
#pragma unroll
                                for (int e = 0; e < 2; ++e) {
                                    T vo, vn, g0, g1;
                                    mono_at<K, T>(co, Po[e], vo, g0, g1);
                                    mono_at<K, T>(cn, Pn[e], vn, g0, g1);
                                    qo[e][v] = kMixed ? oa + vo : vo;
                                    qn[e][v] = kMixed ? (T)na + vn : vn;
                                }
                                // one variable's coefficients in registers at a time
                                asm volatile("" ::: "memory");
                            }
#pragma unroll
                            for (int e = 0; e < 2; ++e)
                                beta = fmax(beta,
                                            fmax(spectral_radius(qo[e][0], qo[e][1], qo[e][2], qo[e][3], nx, ny, gammaT),
                                                 spectral_radius(qn[e][0], qn[e][1], qn[e][2], qn[e][3], nx, ny, gammaT)));
                        }
                        const T bh = beta * bh_len;
                        // the neighbour's side: h = 2|N| / l_i, 2|N| = d1 x d2 of its edge vectors
                        T hn = (T)0.0, bhn = (T)0.0;
                        if (partner) {
                            const T a2 = fma(dn[0], dn[3], -(dn[1] * dn[2]));
                            hn = a2 * il;
                            bhn = beta * len * F::rcp(a2);
                        }
                        // the coefficients are read again below rather than kept from above
                        asm volatile("" ::: "memory");
                        // Jumps (neighbour minus own) of variable v's value and physical
                        // gradient at the two ends, and of its (constant) Hessian.
                        auto jumps = [&](int v, T (&jv)[2], T (&jx)[2], T (&jy)[2], T (&dh)[3])
                                         __attribute__((always_inline)) {
                            T co[NC], cn[NC];
#pragma unroll
                            for (int k2 = 0; k2 < NC; ++k2) co[k2] = L.c[v][k2][threadIdx.x];
                            double na;
                            nbc(v, na, cn);
#pragma unroll
                            for (int e = 0; e < 2; ++e) {
                                T vo, gxo, gyo, vn, gxn, gyn;
                                mono_at<K, T>(co, Po[e], vo, gxo, gyo);
                                mono_at<K, T>(cn, Pn[e], vn, gxn, gyn);
                                // mixed: the FP64 difference of averages plus the float one of the rest
                                if constexpr (kMixed) jv[e] = (T)(na - L.avg[kMixed ? v : 0][kMixed ? threadIdx.x : 0]) + (vn - vo);
                                else jv[e] = vn - vo;
                                jx[e] = gxn - gxo;
                                jy[e] = gyn - gyo;
                            }
                            // the Hessian (2 cXX, cXY, 2 cYY)
                            if constexpr (K == 2) {
                                dh[0] = (T)2.0 * (cn[3] - co[3]);
                                dh[1] = cn[4] - co[4];
                                dh[2] = (T)2.0 * (cn[5] - co[5]);
                            }
                        };
                        T pn[4][K];   // the partner's rates from this edge
#pragma unroll
                        for (int v = 0; v < 4; ++v)
#pragma unroll
                            for (int m = 0; m < K; ++m) pn[v][m] = (T)0.0;
                        auto both = [&](int v, const T (&Sv)[K + 1]) __attribute__((always_inline)) {
                            T p[K];
                            rates(Sv, bh, h, p);
#pragma unroll
                            for (int m = 0; m < K; ++m) acc[v][m] += p[m];
                            if (partner) rates(Sv, bhn, hn, pn[v]);
                        };
                        {
                            T jv[2], jx[2], jy[2], dh[3], Sv[K + 1];
                            jumps(0, jv, jx, jy, dh);
                            energies(jv, jx, jy, dh, Sv);
                            both(0, Sv);
                            jumps(3, jv, jx, jy, dh);
                            energies(jv, jx, jy, dh, Sv);
                            both(3, Sv);
                        }
                        asm volatile("" ::: "memory");
                        {
                            // RIOE: the momentum enters as m_n = m.n and m_t = m.(-n_y, n_x), with
                            // K's normal on both sides, and delta(m) = max(delta(m_n), delta(m_t)),
                            // one root of the larger energy; component-wise: m_1, m_2 apart
                            T jv1[2], jx1[2], jy1[2], dh1[3], jv2[2], jx2[2], jy2[2], dh2[3];
                            jumps(1, jv1, jx1, jy1, dh1);
                            jumps(2, jv2, jx2, jy2, dh2);
                            const T ca = ri ? nx : (T)1.0, cb = ri ? ny : (T)0.0;
                            auto rot = [&](T& a1, T& a2) __attribute__((always_inline)) {
                                const T b1 = fma(ca, a1, cb * a2), b2 = fma(ca, a2, -(cb * a1));
                                a1 = b1;
                                a2 = b2;
                            };
#pragma unroll
                            for (int e = 0; e < 2; ++e) {
                                rot(jv1[e], jv2[e]);
                                rot(jx1[e], jx2[e]);
                                rot(jy1[e], jy2[e]);
                            }
                            if constexpr (K == 2) {
#pragma unroll
                                for (int k2 = 0; k2 < 3; ++k2) rot(dh1[k2], dh2[k2]);
                            }
                            T S1[K + 1], S2[K + 1];
                            energies(jv1, jx1, jy1, dh1, S1);
                            energies(jv2, jx2, jy2, dh2, S2);
                            if (ri) {
#pragma unroll
                                for (int jj = 0; jj <= K; ++jj) S1[jj] = fmax(S1[jj], S2[jj]);
                            }
                            both(1, S1);
                            if (!ri) both(2, S2);
                        }
                        if (partner) {
                            // kept for the partner (at most two per lane, by the edge orientation)
                            const bool r0 = nrec == 0;
#pragma unroll
                            for (int v = 0; v < 4; ++v)
#pragma unroll
                                for (int m = 0; m < K; ++m) {
                                    rec[0][v][m] = r0 ? pn[v][m] : rec[0][v][m];
                                    rec[1][v][m] = r0 ? rec[1][v][m] : pn[v][m];
                                }
                            const int to = j * kTileCells + ((ll >> 3) & kLinkSlotMask);
                            rto[0] = r0 ? to : rto[0];
                            rto[1] = r0 ? rto[1] : to;
                            ++nrec;
                        }
                    };
                    if (ll & kLinkGlobal) {
                        const int cell = (ll & ~kLinkGlobal) >> 3;
                        const unsigned n8 = (unsigned)cell * 8u, nT = (unsigned)cell * (unsigned)sizeof(T);
                        const T nxx = (T)mv.J(0, n8), nxy = (T)mv.J(1, n8), nex = (T)mv.J(2, n8), ney = (T)mv.J(3, n8);
                        T dn[4];
                        edge_vectors(nxx, nxy, nex, ney, dn);
                        edge(
                            [&](int v, double& na, T (&cn)[NC]) __attribute__((always_inline)) {
                                T u[NM];
                                na = wp.a(v, n8);
                                u[0] = (T)na;
#pragma unroll
                                for (int l = 1; l < NM; ++l) u[l] = wp.h(v, l, nT);
                                to_mono<K, T>(u, nxx, nxy, nex, ney, !kMixed, cn);
                            },
                            dn, false);
                    } else {
                        const int sl = (ll >> 3) & kLinkSlotMask;
                        T dn[4];
#pragma unroll
                        for (int k2 = 0; k2 < 4; ++k2) dn[k2] = L.d[k2][sl];
                        edge(
                            [&](int v, double& na, T (&cn)[NC]) __attribute__((always_inline)) {
                                na = kMixed ? L.avg[kMixed ? v : 0][kMixed ? sl : 0] : 0.0;
#pragma unroll
                                for (int k2 = 0; k2 < NC; ++k2) cn[k2] = L.c[v][k2][sl];
                            },
                            dn, sl < kTileCells);
                    }
                }
            }
            // the state again (from cache; not kept in registers through the edge work),
            // in flight while the partners' shares go through LDS.  The mixed P2 form
            // keeps it: its float modes fit beside the edge work without spilling.
            if (live && !(kMixed && K == 2)) load_cell<NM, T>(wp, c, wa, w);
            // the partners' shares: written over the image once every lane is done with it
            T (&R)[4][K][3][kTileCells] = oe_records<K, T>(L);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 2; ++q)
                if (rto[q] >= 0) {
                    const int e = rto[q] / kTileCells, s = rto[q] % kTileCells;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (ri && v == 2) continue;   // RIOE: m_2's rates are m_1's
#pragma unroll
                        for (int m = 0; m < K; ++m) R[v][m][e][s] = rec[q][v][m];
                    }
                }
            __syncthreads();
            if (live) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (link_recv(lk[i])) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            if (ri && v == 2) continue;
#pragma unroll
                            for (int m = 0; m < K; ++m) acc[v][m] += R[v][m][i][threadIdx.x];
                        }
                    }
                if (ri) {
#pragma unroll
                    for (int m = 0; m < K; ++m) acc[2][m] = acc[1][m];
                }
            }
            // the tile's last read of the image: from here a wave may go on to the next
            // tile (a batched tile keeps its barrier at the end, before its record flush)
            if constexpr (!kBatch) __syncthreads();
        }
        if (live) {
            if (oe) {
                // exact solution of the damping ODE: degree-m modes scaled by
                // exp(-dt sum_{j<=m} sigma^j); the cell average is untouched (eq. OE:m0)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const T inv = v == 0 ? inv0 : (v == 1 ? inv1 : (v == 2 ? inv2 : inv3));
#pragma unroll
                    for (int m = 1; m <= K; ++m) {
                        const T fct = F::exp(-dt * (inv * acc[v][m - 1]));
#pragma unroll
                        for (int l = m * (m + 1) / 2; l < (m + 1) * (m + 2) / 2; ++l) w[v][l] *= fct;
                    }
                }
            }
            // the full state in FP64 at the limiter's node set
            const double n0x = mv.N(0, c8), n0e = mv.N(1, c8);
            const double n1x = mv.N(2, c8), n1e = mv.N(3, c8);
            double wd[4][NM];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                wd[v][0] = wa[v];
#pragma unroll
                for (int l = 1; l < NM; ++l) wd[v][l] = (double)w[v][l];
            }
            double pv[NP][4];
            node_values<K, NM>(wd, n0x, n0e, n1x, n1e, a.zxs, a.ustar, pv);
            const double ub0 = wa[0], ub1 = wa[1], ub2 = wa[2], ub3 = wa[3];
            double th1 = 1.0, th2 = 1.0;
            if (a.bp_enable) {
                // step 1: density (Sec. 4.4, eq. 1944)
                double rmin = pv[0][0];
#pragma unroll
                for (int t = 1; t < NP; ++t) rmin = fmin(rmin, pv[t][0]);
                const double e1 = fmin(ub0, kEpsBP);
                th1 = rmin >= e1 ? 1.0 : fmin((ub0 - e1) / (ub0 - rmin), 1.0);
                // factor of the stored density modes: in the mixed form it aims above the
                // floor by the rounding bound; theta_2 below still comes from the density
                // pinned at eps_1 (rho e grows with rho at nodes below the average, so
                // that theta_2 is the smaller one), which keeps it at the FP64 value
                double th1s = th1;
                double as0 = 0.0, as1 = 0.0, as2 = 0.0, as3 = 0.0;   // mixed: sum_{l>=1} |c_l| per variable
                if constexpr (kMixed) {
                    as0 = abs_sum_hi<NM>(wd[0]);
                    as1 = abs_sum_hi<NM>(wd[1]);
                    as2 = abs_sum_hi<NM>(wd[2]);
                    as3 = abs_sum_hi<NM>(wd[3]);
                    const double t1 = fma(kMixMargin, as0, e1);
                    th1s = rmin >= t1 ? 1.0 : fmax(fmin((ub0 - t1) / (ub0 - rmin), 1.0), 0.0);
                }
                // step 2: internal energy E - |m|^2 / (2 rho) of the density-scaled state (eq. 1981)
                const double eb = ub3 - 0.5 * (ub1 * ub1 + ub2 * ub2) / ub0;
                const double e2 = fmin(eb, kEpsBP);
                double emin = INFINITY;
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    pv[t][0] = fma(th1, pv[t][0] - ub0, ub0);
                    emin = fmin(emin, internal_energy(pv[t]));
                }
                th2 = emin >= e2 ? 1.0 : fmin((eb - e2) / (eb - emin), 1.0);
                if constexpr (kMixed) {
                    // Rounding the scaled modes moves rho e at a node by at most, to first
                    // order, |dE| + |v| (|dm1| + |dm2|) + |v|^2/2 |drho|, with v the
                    // velocity of the limited state there and each |d.| <= margin * theta
                    // * sum_l |c_l|; theta_2 aims that far above the floor.
                    double vloc = 0.0;
#pragma unroll
                    for (int t = 0; t < NP; ++t) {
                        const double q0 = fma(th2, pv[t][0] - ub0, ub0);
                        const double q1 = fma(th2, pv[t][1] - ub1, ub1), q2 = fma(th2, pv[t][2] - ub2, ub2);
                        vloc = fmax(vloc, fma(q1, q1, q2 * q2) * frcp(q0 * q0));
                    }
                    const double vm = fsqrt(vloc);
                    const double t2 = e2 + kMixMargin * th2 * (as3 + vm * (as1 + as2) + 0.5 * vm * vm * th1 * as0);
                    th2 = emin >= t2 ? 1.0 : fmax(fmin((eb - t2) / (eb - emin), 1.0), 0.0);
                    th1 = th1s;
                    if (th1 * th2 < 1.0 || th2 < 1.0) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const double fct = v == 0 ? th1 * th2 : th2;
#pragma unroll
                            for (int l = 1; l < NM; ++l) w[v][l] = (T)((double)w[v][l] * fct);
                        }
                    }
                } else {
#pragma unroll
                    for (int l = 1; l < NM; ++l) {
                        w[0][l] *= th1;
#pragma unroll
                        for (int v = 0; v < 4; ++v) w[v][l] *= th2;
                    }
                }
                part[1] = (th1 < 1.0 || th2 < 1.0) ? 1.0 : 0.0;
                part[2] = (ub0 > 0.0 && eb > 0.0) ? 0.0 : 1.0;
                if constexpr (kMixed) {
                    if (th1 < 1.0 || th2 < 1.0) {
                        // check the coefficients as stored (rounded to float)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
#pragma unroll
                            for (int l = 1; l < NM; ++l) wd[v][l] = (double)w[v][l];
                        node_values<K, NM>(wd, n0x, n0e, n1x, n1e, a.zxs, a.ustar, pv);
                        bool ok = true;
#pragma unroll
                        for (int t = 0; t < NP; ++t)
                            ok = ok && pv[t][0] >= 0.5 * e1 && internal_energy(pv[t]) >= 0.5 * e2;
                        if (!ok) {
                            // keep the average only: admissible whenever the average is
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
#pragma unroll
                                for (int l = 1; l < NM; ++l) w[v][l] = (T)0.0;
#pragma unroll
                                for (int t = 0; t < NP; ++t) pv[t][v] = wa[v];
                            }
                            part[3] = 1.0;
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
            const bool any_bnd = lk[0] < 0 || lk[1] < 0 || lk[2] < 0;
            double amax = 0.0;
            // the output's density and pressure at every limiter node, for the diagnostics;
            // at the edge points the same 1/rho and p serve the wave speed and the flux
            double rmin_o = INFINITY, pmin_o = INFINITY;
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                const double q0 = fma(ta, pv[t][0] - ub0, ub0), q1 = fma(ta, pv[t][1] - ub1, ub1);
                const double q2 = fma(ta, pv[t][2] - ub2, ub2), q3 = fma(ta, pv[t][3] - ub3, ub3);
                const double ir = frcp(q0), mm = fma(q1, q1, q2 * q2);
                const double p = (gamma - 1.0) * fma(-0.5 * ir, mm, q3);
                rmin_o = fmin(rmin_o, q0);
                pmin_o = fmin(pmin_o, p);
                if (t >= 3 * NE) continue;   // the two inner nodes
                const int i = t / NE, nu = t % NE;
                T nxT, nyT, lenT;
                edge_normal(od, i, nxT, nyT, lenT);
                const double nx = (double)nxT, ny = (double)nyT;
                const double mn = fma(q1, nx, q2 * ny);
                // |v.n| + c, guarded below the floor as spectral_radius is
                const bool ok = q0 >= kEpsBP;
                const double irs = ok ? ir : 1.0 / kEpsBP;
                const double ps = ok ? p : (gamma - 1.0) * fma(-0.5 * irs, mm, q3);
                const double rr = fma(fabs(mn), irs, fsqrt(gamma * fmax(ps, 0.0) * irs));
                amax = (rr > amax || rr != rr) ? rr : amax;
                if (any_bnd && lk[i] < 0) {
                    const double lw = (double)lenT * R::ws[nu];
                    if (lk[i] == kLinkWall) {
                        const double ca = lw * fma(mn * mn, ir, p), cb = lw * mn;
                        part[6] = fma(ca, nx, part[6]);
                        part[7] = fma(ca, ny, part[7]);
                        part[8] = fma(cb, nx, part[8]);
                        part[9] = fma(cb, ny, part[9]);
                    } else {
                        part[6] = fma(lw, fma(q1 * mn, ir, p * nx), part[6]);
                        part[7] = fma(lw, fma(q2 * mn, ir, p * ny), part[7]);
                    }
                }
            }
            part[0] = amax;
            part[4] = area_d * wa[1];
            part[5] = area_d * wa[2];
            part[10] = rmin_o;
            part[11] = pmin_o;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                op.put_a(v, c8, wa[v]);
#pragma unroll
                for (int l = 1; l < NM; ++l) op.put_h(v, l, cT, w[v][l]);
            }
        }
        wave_acc_add<kFilCols>(W, ops, part, par);
        // a batched tile's record is flushed next, and the image rewritten by the next tile
        if constexpr (kBatch) __syncthreads();
    };
    walk_tiles<kBatch>(
        a, g0, g1, tile_body, [&](int par) { wave_acc_reset<kFilCols>(W, ops, par); },
        [&](int gi, int par) {
            if (gi < 0) wave_acc_flush<kFilCols>(W, ops, cols, a.part + blockIdx.x, kMaxBlocks, par, true);
            else wave_acc_flush<kFilCols>(W, ops, cols, a.part + a.gbase + gi, a.gstride, par, false);
        });
}
template <int K, typename T>
__global__ __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(K == 1 ? 3 : OEDG_FIL_WAVES))) void k_filter(
    StageArgs a) {
    if (!a.g->active || a.g->skip) return;
    __shared__ MonoLds<K, T> L;
    __shared__ WaveAcc<kFilCols> W;
    filter_run<K, T, false>(a, 0, 0, L, W);
}
template <int K, typename T>
__global__ __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(K == 1 ? 3 : OEDG_FIL_WAVES))) void k_filter_batch(
    const StageArgs* desc, const Chunk* chunks, ChunkSplit cs) {
    __shared__ MonoLds<K, T> L;
    __shared__ WaveAcc<kFilCols> W;
    for_each_chunk(desc, chunks, cs,
                   [&](const StageArgs& a, int g0, int g1) { filter_run<K, T, true>(a, g0, g1, L, W); });
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
        acc = op == 0 ? wave_sum(acc) : (op == 1 ? wave_min(acc) : wave_max(acc));
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

// The finalize kernels read the scalars they need before the reduction, so that
// their loads overlap it instead of following one another in thread 0 after it;
// an inactive or skipped instance's records are reduced and dropped.

// domain averages and L-infinity norms (eq. normOmg): ||u - ubar|| = max(max u - ubar, ubar - min u)
// and ||| m - mbar |||_inf (eqs. normOmg, RIOESys:Coef1) with its zero branch.
// An inadmissible average ends this attempt of the step: `skip` turns the rest
// of it into no-ops (u^n is untouched) until the third stage's finalize.
__device__ __forceinline__ void fin_residual(const double* base, size_t cstride, int G, Glob* g) {
    const int active = g->active, skip = g->skip;
    const double area_sum = g->area_sum;
    // 4 sums, 4 mins, 4 maxima, the max of |m - mbar|^2, then the bad-average count
    double tot[kNumPartial + 2];
    reduce_columns<kNumPartial + 2>(base, cstride, G, 0, 0x2AA5500u, tot, kColBad);
    // skipped (an earlier stage of this attempt failed): the pass wrote no records,
    // and the domain values of the last state it did run stay in place
    if (threadIdx.x != 0 || !active || skip) return;
    if (tot[kNumPartial + 1] > 0.0) g->skip = 1;
    double ub[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        ub[v] = tot[v] / area_sum;
        const double n = fmax(tot[8 + v] - ub[v], ub[v] - tot[4 + v]);
        g->ubar[v] = ub[v];
        g->nrm[v] = n;
        g->inv_nrm[v] = n <= kEpsOE * fmax(1.0, fabs(ub[v])) ? 0.0 : 1.0 / n;
    }
    const double n = sqrt(tot[kNumPartial]);
    const double mb = sqrt(ub[1] * ub[1] + ub[2] * ub[2]);
    g->nrm_m = n;
    g->inv_nrm_m = n <= kEpsOE * fmax(1.0, mb) ? 0.0 : 1.0 / n;
}

// alpha of the stage output; after the third stage (or the initial limiter pass)
// t, the step count and Delta t = C_SSP/alpha min_K C^DCW_{K,k}|K|, clamped to t_end.
// After the third stage of a skipped attempt: the step is retried from u^n with
// half the time step, or the run stops once max_restarts retries are used.
__device__ __forceinline__ void fin_filter(const double* base, size_t cstride, int G, Glob* g, int stage) {
    const int active = g->active, skip = g->skip;
    double t = 0.0, dt = 0.0, t_end = 0.0, minck = 0.0, c_ssp = 0.0, alpha_step = 0.0;
    long long step = 0, n_lim = 0, n_bad = 0, n_flat = 0, n_cfl = 0, n_restarts = 0;
    int err = 0, restarts = 0, max_restarts = 0;
    if (threadIdx.x == 0) {
        t = g->t;
        dt = g->dt;
        t_end = g->t_end;
        minck = g->minck;
        c_ssp = g->c_ssp;
        alpha_step = g->alpha_step;
        step = g->step;
        n_lim = g->n_limited;
        n_bad = g->n_bad;
        n_flat = g->n_flat;
        n_cfl = g->n_cfl_exc;
        n_restarts = g->n_restarts;
        err = g->err;
        restarts = g->restarts;
        max_restarts = g->max_restarts;
    }
    double r[kFilterCols];
    // max, sums, then two minima; its barrier also orders every thread's read of
    // `skip` before thread 0 may clear it
    reduce_columns<kFilterCols>(base, cstride, G, kNumPartial + 1, 2u | (1u << 20) | (1u << 22), r);
    if (threadIdx.x != 0 || !active) return;
    if (skip) {
        if (stage == 2) {
            g->skip = 0;
            if (restarts + 1 > max_restarts) {
                g->restarts = restarts + 1;
                g->err = 1;
                g->active = 0;
            } else {
                g->restarts = restarts + 1;
                g->dt = 0.5 * dt;
                g->alpha = alpha_step;   // the retry's first stage starts from u^n again
                g->n_restarts = n_restarts + 1;
            }
        }
        return;
    }
    const double alpha = r[0], lim = r[1], bad = r[2];
    g->min_rho_node = r[10];
    g->min_p_node = r[11];
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
    g->n_limited = n_lim + (long long)lim;
    g->n_bad = n_bad + (long long)bad;
    g->n_flat = n_flat + (long long)r[3];
    if (bad > 0) err = 1;
    g->err = err;
    if (stage < 2) {
        g->alpha = alpha;
        if (stage < 0) g->alpha_step = alpha;
        else if (alpha > alpha_step * (1.0 + 1e-12)) g->n_cfl_exc = n_cfl + 1;
    } else {
        t += dt;
        g->t = t;
        g->step = step + 1;
        g->alpha = alpha;
        g->alpha_step = alpha;
        g->restarts = 0;
    }
    int act = 1;
    if (stage < 0 || stage == 2) {
        double ndt = c_ssp * minck / alpha;
        const double rem = t_end - t;
        if (rem < ndt) ndt = rem;
        g->dt = ndt;
        if (!(isinf(t_end) || rem > 1e-12 * fmax(1.0, fabs(t_end)))) act = 0;
    }
    if (err) act = 0;
    if (!act) g->active = 0;
}

// One instance: the partials of the G workgroups of its passes.
__global__ __launch_bounds__(kFinThreads) void k_fin_residual(const double* part, int G, Glob* g) {
    fin_residual(part, kMaxBlocks, G, g);
}
__global__ __launch_bounds__(kFinThreads) void k_fin_filter(const double* part, int G, Glob* g, int stage) {
    fin_filter(part, kMaxBlocks, G, g, stage);
}

// A batch: workgroup i reduces the group records of instance desc[i].
__global__ __launch_bounds__(kFinThreads) void k_fin_residual_batch(const StageArgs* desc) {
    const StageArgs& a = desc[blockIdx.x];
    fin_residual(a.part + a.gbase, a.gstride, n_groups(a.m.n_cell), a.g);
}
__global__ __launch_bounds__(kFinThreads) void k_fin_filter_batch(const StageArgs* desc) {
    const StageArgs& a = desc[blockIdx.x];
    fin_filter(a.part + a.gbase, a.gstride, n_groups(a.m.n_cell), a.g, a.stage);
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
    const SView<NM, T> op = sview<NM, T>(a.uout, a);
    const unsigned c8 = (unsigned)c * 8u, cT = (unsigned)c * (unsigned)sizeof(T);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        op.put_a(v, c8, acc[v][0]);
#pragma unroll
        for (int l = 1; l < NM; ++l) op.put_h(v, l, cT, (T)acc[v][l]);
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

// host handles of the batched pass instantiations of one (degree, precision)
struct BatchSet {
    const void* pass[kNumPasses];   // residual, filter
};
template <int K, typename T>
BatchSet batch_set() {
    return {{reinterpret_cast<const void*>(&k_residual_batch<K, T>),
             reinterpret_cast<const void*>(&k_filter_batch<K, T>)}};
}
const BatchSet& batch_kernels(int kmask, int mixed) {
    static const BatchSet sets[2][2] = {{batch_set<1, double>(), batch_set<1, float>()},
                                        {batch_set<2, double>(), batch_set<2, float>()}};
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
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kPassThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1, cus = cus > 0 ? cus : 256;
    const int g = std::min(kMaxBlocks, std::max(8, (cus * per_cu) / 8 * 8));
    cache[kernel] = g;
    return g;
}

int launch_pass(int which, int k, const StageArgs& a, void* stream) {
    StageArgs args = a;
    void* argv[] = {&args};
    const int grid = grid_for_pass(which, k, a.mixed, a.m.n_cell);
    return (int)hipLaunchKernel(kernels_for(k, a.mixed).pass[which], dim3(grid), dim3(kPassThreads), argv, 0,
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
    const int tiles = n_tiles_of(n_cell);
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
    if (kmask < 1 || kmask > 2 || grid < 8 || (grid & 7) != 0) return (int)hipErrorInvalidValue;
    ChunkSplit split = cs;
    void* argv[] = {&desc, &chunks, &split};
    return (int)hipLaunchKernel(batch_kernels(kmask, mixed).pass[which], dim3(grid), dim3(kPassThreads), argv, 0,
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
