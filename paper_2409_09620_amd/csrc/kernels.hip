// gfx950 kernels of one BP RI-OEDG stage (2D Euler, P1/P2 modal DG on triangles).
//
// Three passes per stage, one thread per cell, state in structure-of-arrays
// [var][mode][cell] so every own-cell load and store is coalesced:
//   k_residual  volume + edge quadrature of eq. DGSystem:Dis with the LF flux
//               (eq. fluxLF), the diagonal mass, the SSP-RK3 combination (eq.
//               RKTime); writes the pre-filter state and per-block partials of
//               sum |K| ubar_K and of min/max at the volume points (eq. normOmg).
//   k_mnorm     ||| m - mbar |||_inf at the volume points (needs mbar first).
//   k_filter    RIOE damping (eq. oe:sys, coefficients of eqs. OEScalar:beta,
//               OEScalar:Coef2, oe:sysdelta2, RIOESys:CoefM), the BP limiter at
//               the decomposition nodes (Sec. 4.4), and the max wave speed of the
//               result (eq. 1250) that sets the next stage's LF viscosity and,
//               after the third stage, Delta t (Sec. 5 with eq. 1692 / eq. 1713).
// Each pass publishes per-workgroup partials; the last workgroup to finish (an
// atomic ticket) reduces them in a fixed order, so results do not depend on
// scheduling.  Neighbour data is gathered through the edge table (link).
#include <hip/hip_runtime.h>

#include <cmath>

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
    static constexpr double s[2] = {0.2113248654051871, 0.7886751345948129};
    static constexpr double ws[2] = {0.5, 0.5};
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

template <int K>
__device__ __forceinline__ void dpsi(double x, double e, double* dx, double* de) {
    dx[0] = 0.0;
    de[0] = 0.0;
    dx[1] = 4.0;
    de[1] = 2.0;
    dx[2] = 0.0;
    de[2] = 3.0;
    if constexpr (K == 2) {
        dx[3] = 48.0 * x + 24.0 * e - 24.0;
        de[3] = 24.0 * x + 8.0 * e - 8.0;
        dx[4] = 20.0 * e - 4.0;
        de[4] = 20.0 * x + 20.0 * e - 12.0;
        dx[5] = 0.0;
        de[5] = 20.0 * e - 8.0;
    }
}

// reference point of local edge i at parameter s (edge i runs from vertex i+1 to i+2)
__device__ __forceinline__ void edge_point(int i, double s, double& x, double& e) {
    x = i == 0 ? 1.0 - s : (i == 1 ? 0.0 : s);
    e = i == 0 ? s : (i == 1 ? 1.0 - s : 0.0);
}
__device__ __forceinline__ void vertex_point(int v, double& x, double& e) {
    x = v == 1 ? 1.0 : 0.0;
    e = v == 2 ? 1.0 : 0.0;
}

template <int NM>
__device__ __forceinline__ void eval4(const double (&u)[4][NM], const double* p, double* q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double s = u[v][0] * p[0];
#pragma unroll
        for (int l = 1; l < NM; ++l) s = fma(u[v][l], p[l], s);
        q[v] = s;
    }
}

// ------------------------------------------------------------------------- Euler

// normal flux F(q).n for a (possibly scaled) normal (nx, ny)
__device__ __forceinline__ void normal_flux(const double* q, double nx, double ny, double gm1, double* f) {
    const double ir = 1.0 / q[0];
    const double mn = q[1] * nx + q[2] * ny;
    const double p = gm1 * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) * ir);
    const double vn = mn * ir;
    f[0] = mn;
    f[1] = q[1] * vn + p * nx;
    f[2] = q[2] * vn + p * ny;
    f[3] = (q[3] + p) * vn;
}

// spectral radius |v.n| + c of F'(u).n (Example ex:euler); guarded so that a
// pre-limiter state with rho <= 0 or p < 0 still gives a finite value
__device__ __forceinline__ double spectral_radius(const double* q, double nx, double ny, double gamma) {
    const double rs = fmax(q[0], kEpsBP);
    const double ir = 1.0 / rs;
    const double p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) * ir);
    return fabs(q[1] * nx + q[2] * ny) * ir + sqrt(gamma * fmax(p, 0.0) * ir);
}

__device__ __forceinline__ double internal_energy(const double* q) {
    return q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0];
}

// ------------------------------------------------------------------------- reductions

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
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// op: 0 sum, 1 min, 2 max.  Result valid in thread 0.  Fixed reduction order.
template <int N>
__device__ __forceinline__ void block_reduce(double* vals, const int* ops, double (*lds)[N]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double v = vals[k];
        v = ops[k] == 0 ? wave_sum(v) : (ops[k] == 1 ? wave_min(v) : wave_max(v));
        if (lane == 0) lds[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double v = lds[0][k];
            for (int w = 1; w < kBlock / 64; ++w)
                v = ops[k] == 0 ? v + lds[w][k] : (ops[k] == 1 ? fmin(v, lds[w][k]) : fmax(v, lds[w][k]));
            vals[k] = v;
        }
    }
    __syncthreads();
}

// Publishes this block's partials (thread 0 wrote them) and tells whether this
// block is the last one of the grid to arrive.
__device__ __forceinline__ bool arrive_last(unsigned int* ticket) {
    __shared__ int last;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Reduces part[b * stride + k] over all blocks b in a fixed order.
template <int N>
__device__ __forceinline__ void reduce_partials(const double* part, int stride, int nblk, const int* ops,
                                                double* out, double (*lds)[N]) {
    double acc[N];
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] = ops[k] == 0 ? 0.0 : (ops[k] == 1 ? INFINITY : -INFINITY);
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double v = __hip_atomic_load(part + (size_t)b * stride + k, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
            acc[k] = ops[k] == 0 ? acc[k] + v : (ops[k] == 1 ? fmin(acc[k], v) : fmax(acc[k], v));
        }
    }
    block_reduce<N>(acc, ops, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < N; ++k) out[k] = acc[k];
}

// ------------------------------------------------------------------------- pass 1: residual

template <int K>
__global__ __launch_bounds__(kBlock) void k_residual(StageArgs a) {
    using R = Rule<K>;
    constexpr int NM = R::NM;
    Glob* g = a.g;
    if (!g->active) return;
    const int nc = a.m.n_cell;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    const size_t snc = (size_t)nc;

    double red[kNumPartial];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        red[v] = 0.0;
        red[4 + v] = INFINITY;
        red[8 + v] = -INFINITY;
    }

    if (c < nc) {
        const double alpha = g->alpha, dt = g->dt, gm1 = a.gamma - 1.0;
        double u[4][NM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) u[v][l] = a.uin[(v * NM + l) * snc + c];
        const double xx = a.m.jinv[c], xy = a.m.jinv[snc + c];
        const double ex = a.m.jinv[2 * snc + c], ey = a.m.jinv[3 * snc + c];
        const double area = a.m.area[c];

        double r[4][NM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) r[v][l] = 0.0;

        // volume term: |K| sum_mu w_mu F(u) . grad Psi_l, with grad Psi = J^{-T} grad_ref Psi
        // written as dPsi/dxi (F . grad xi) + dPsi/deta (F . grad eta)
#pragma unroll
        for (int m = 0; m < R::NQ; ++m) {
            double p[NM], dx[NM], de[NM], q[4], g1[4], g2[4];
            psi<K>(R::xi[m], R::eta[m], p);
            dpsi<K>(R::xi[m], R::eta[m], dx, de);
            eval4<NM>(u, p, q);
            normal_flux(q, xx, xy, gm1, g1);
            normal_flux(q, ex, ey, gm1, g2);
            const double wa = R::w[m] * area;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double a1 = wa * g1[v], a2 = wa * g2[v];
#pragma unroll
                for (int l = 1; l < NM; ++l) r[v][l] = fma(dx[l], a1, fma(de[l], a2, r[v][l]));
            }
        }

        // surface term: - sum_i l_i sum_nu w_nu Fhat(u_int, u_ext, n_i) Psi_l; the scaled
        // normal l_i n_i equals -2|K| grad(lambda_i) of the barycentric coordinate
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double gx = i == 0 ? -(xx + ex) : (i == 1 ? xx : ex);
            const double gy = i == 0 ? -(xy + ey) : (i == 1 ? xy : ey);
            const double lnx = -2.0 * area * gx, lny = -2.0 * area * gy;
            const double li = a.m.len[i * snc + c];
            const int link = a.m.link[i * snc + c];
            const bool has = link >= 0;
            const int nb = has ? (link >> 2) : c;
            const int j = link & 3;
            double un[4][NM];
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int l = 0; l < NM; ++l) un[v][l] = a.uin[(v * NM + l) * snc + nb];
#pragma unroll
            for (int nu = 0; nu < R::NE; ++nu) {
                double x, e, p[NM], qi[4], qe[4], fi[4], fe[4];
                edge_point(i, R::s[nu], x, e);
                psi<K>(x, e, p);
                eval4<NM>(u, p, qi);
                if (has) {
                    // the neighbour runs the shared edge the other way: parameter 1 - s
                    double xn, en, pn[NM];
                    edge_point(j, 1.0 - R::s[nu], xn, en);
                    psi<K>(xn, en, pn);
                    eval4<NM>(un, pn, qe);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) qe[v] = qi[v];
                }
                normal_flux(qi, lnx, lny, gm1, fi);
                normal_flux(qe, lnx, lny, gm1, fe);
                const double al = alpha * li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double fh = R::ws[nu] * 0.5 * (fi[v] + fe[v] - al * (qe[v] - qi[v]));
#pragma unroll
                    for (int l = 0; l < NM; ++l) r[v][l] = fma(-fh, p[l], r[v][l]);
                }
            }
        }

        // diagonal mass a_K^(l) = |K| (a_l/|K|), then the SSP-RK3 combination
        const double ia = 1.0 / area;
        const double sa = a.stage == 0 ? 0.0 : (a.stage == 1 ? 0.75 : 1.0 / 3.0);
        const double sb = a.stage == 0 ? 1.0 : (a.stage == 1 ? 0.25 : 2.0 / 3.0);
        double w[4][NM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) {
                const double du = r[v][l] * ia * kInvMass[l];
                const double adv = u[v][l] + dt * du;
                double val;
                if (a.stage == 0) {
                    val = adv;
                } else {
                    val = sa * a.u0[(v * NM + l) * snc + c] + sb * adv;
                }
                w[v][l] = val;
                a.w[(v * NM + l) * snc + c] = val;
            }
#pragma unroll
        for (int v = 0; v < 4; ++v) red[v] = area * w[v][0];
#pragma unroll
        for (int m = 0; m < R::NQ; ++m) {
            double p[NM], q[4];
            psi<K>(R::xi[m], R::eta[m], p);
            eval4<NM>(w, p, q);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                red[4 + v] = fmin(red[4 + v], q[v]);
                red[8 + v] = fmax(red[8 + v], q[v]);
            }
        }
    }

    __shared__ double lds[kBlock / 64][kNumPartial];
    const int ops[kNumPartial] = {0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2};
    block_reduce<kNumPartial>(red, ops, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < kNumPartial; ++k) a.part[(size_t)blockIdx.x * 16 + k] = red[k];
    if (!arrive_last(&g->ticket[0])) return;

    double tot[kNumPartial];
    reduce_partials<kNumPartial>(a.part, 16, gridDim.x, ops, tot, lds);
    if (threadIdx.x == 0) {
        // eq. normOmg: ||u - ubar||_inf = max(max u - ubar, ubar - min u) over the volume points
        for (int v = 0; v < 4; ++v) {
            const double ub = tot[v] / g->area_sum;
            const double n = fmax(tot[8 + v] - ub, ub - tot[4 + v]);
            g->ubar[v] = ub;
            g->nrm[v] = n;
            g->inv_nrm[v] = n <= kEpsOE * fmax(1.0, fabs(ub)) ? 0.0 : 1.0 / n;
        }
        g->ticket[0] = 0;
    }
}

// ------------------------------------------------------------------------- pass 2: momentum norm

template <int K>
__global__ __launch_bounds__(kBlock) void k_mnorm(StageArgs a) {
    using R = Rule<K>;
    constexpr int NM = R::NM;
    Glob* g = a.g;
    if (!g->active) return;
    const int nc = a.m.n_cell;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    const size_t snc = (size_t)nc;
    double best[1] = {0.0};
    if (c < nc) {
        const double mb1 = g->ubar[1], mb2 = g->ubar[2];
        double m1[NM], m2[NM];
#pragma unroll
        for (int l = 0; l < NM; ++l) {
            m1[l] = a.w[(1 * NM + l) * snc + c];
            m2[l] = a.w[(2 * NM + l) * snc + c];
        }
#pragma unroll
        for (int m = 0; m < R::NQ; ++m) {
            double p[NM];
            psi<K>(R::xi[m], R::eta[m], p);
            double s1 = m1[0] * p[0], s2 = m2[0] * p[0];
#pragma unroll
            for (int l = 1; l < NM; ++l) {
                s1 = fma(m1[l], p[l], s1);
                s2 = fma(m2[l], p[l], s2);
            }
            const double d1 = s1 - mb1, d2 = s2 - mb2;
            best[0] = fmax(best[0], d1 * d1 + d2 * d2);
        }
    }
    __shared__ double lds[kBlock / 64][1];
    const int ops[1] = {2};
    block_reduce<1>(best, ops, lds);
    double* part = a.part + (size_t)gridDim.x * 16;
    if (threadIdx.x == 0) part[blockIdx.x] = best[0];
    if (!arrive_last(&g->ticket[1])) return;
    double tot[1];
    reduce_partials<1>(part, 1, gridDim.x, ops, tot, lds);
    if (threadIdx.x == 0) {
        const double n = sqrt(tot[0]);
        const double mb = sqrt(g->ubar[1] * g->ubar[1] + g->ubar[2] * g->ubar[2]);
        g->nrm_m = n;
        g->inv_nrm_m = n <= kEpsOE * fmax(1.0, mb) ? 0.0 : 1.0 / n;
        g->ticket[1] = 0;
    }
}

// ------------------------------------------------------------------------- pass 3: OE, limiter, alpha

// value and physical gradient of all variables at reference point (x, e)
template <int K, int NM>
__device__ __forceinline__ void eval_grad(const double (&u)[4][NM], double x, double e, double xx, double xy,
                                          double ex, double ey, double* q, double* qx, double* qy) {
    double p[NM], dx[NM], de[NM];
    psi<K>(x, e, p);
    dpsi<K>(x, e, dx, de);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double s = 0.0, sx = 0.0, se = 0.0;
#pragma unroll
        for (int l = 0; l < NM; ++l) {
            s = fma(u[v][l], p[l], s);
            sx = fma(u[v][l], dx[l], sx);
            se = fma(u[v][l], de[l], se);
        }
        q[v] = s;
        qx[v] = sx * xx + se * ex;
        qy[v] = sx * xy + se * ey;
    }
}

// constant physical Hessian (xx, xy, yy) of a P2 field with modes u[0..5]
__device__ __forceinline__ void hessian(const double* u, double xx, double xy, double ex, double ey, double* h) {
    const double hxx = 48.0 * u[3];
    const double hxe = 24.0 * u[3] + 20.0 * u[4];
    const double hee = 8.0 * u[3] + 20.0 * u[4] + 20.0 * u[5];
    h[0] = hxx * xx * xx + 2.0 * hxe * xx * ex + hee * ex * ex;
    h[1] = hxx * xx * xy + hxe * (xx * ey + xy * ex) + hee * ex * ey;
    h[2] = hxx * xy * xy + 2.0 * hxe * xy * ey + hee * ey * ey;
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_filter(StageArgs a) {
    using R = Rule<K>;
    constexpr int NM = R::NM;
    Glob* g = a.g;
    if (!g->active) return;
    const int nc = a.m.n_cell;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    const size_t snc = (size_t)nc;
    const double gamma = a.gamma;
    double amax = 0.0;
    int n_lim = 0, n_bad = 0;

    if (c < nc) {
        double w[4][NM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) w[v][l] = a.w[(v * NM + l) * snc + c];
        const double xx = a.m.jinv[c], xy = a.m.jinv[snc + c];
        const double ex = a.m.jinv[2 * snc + c], ey = a.m.jinv[3 * snc + c];
        const double area = a.m.area[c];

        if (a.oe_enable && a.stage >= 0) {
            const double dt = g->dt;
            const double inv_r = g->inv_nrm[0], inv_e = g->inv_nrm[3];
            const double inv_m = g->inv_nrm_m, inv_1 = g->inv_nrm[1], inv_2 = g->inv_nrm[2];
            const bool ri = a.oe_mode == 0;
            double ho[4][3];
            if constexpr (K == 2) {
#pragma unroll
                for (int v = 0; v < 4; ++v) hessian(w[v], xx, xy, ex, ey, ho[v]);
            }
            double sig[4][K + 1];
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int j = 0; j <= K; ++j) sig[v][j] = 0.0;

#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int link = a.m.link[i * snc + c];
                if (link < 0) continue;   // transmissive boundary: zero jump
                const int nb = link >> 2, j = link & 3;
                double wn[4][NM];
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int l = 0; l < NM; ++l) wn[v][l] = a.w[(v * NM + l) * snc + nb];
                const double nxx = a.m.jinv[nb], nxy = a.m.jinv[snc + nb];
                const double nex = a.m.jinv[2 * snc + nb], ney = a.m.jinv[3 * snc + nb];
                const double li = a.m.len[i * snc + c];
                const double gx = i == 0 ? -(xx + ex) : (i == 1 ? xx : ex);
                const double gy = i == 0 ? -(xy + ey) : (i == 1 ? xy : ey);
                const double il = 1.0 / li;
                const double nx = -2.0 * area * gx * il, ny = -2.0 * area * gy * il;
                const double h = 2.0 * area * il;

                // S[q][j]: sum over the two endpoints of squared jumps of order j for
                // q = rho, m_n (or m1), m_t (or m2), E
                double S[4][K + 1];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int jj = 0; jj <= K; ++jj) S[q][jj] = 0.0;
                double beta = 0.0;
#pragma unroll
                for (int end = 0; end < 2; ++end) {
                    // own vertex i+1 (then i+2) meets the neighbour's vertex j+2 (then j+1)
                    const int ov = (i + 1 + end) % 3;
                    const int nv = (j + 2 - end) % 3;
                    double ox, oe, px, pe;
                    vertex_point(ov, ox, oe);
                    vertex_point(nv, px, pe);
                    double q[4], qx[4], qy[4], r[4], rx[4], ry[4];
                    eval_grad<K, NM>(w, ox, oe, xx, xy, ex, ey, q, qx, qy);
                    eval_grad<K, NM>(wn, px, pe, nxx, nxy, nex, ney, r, rx, ry);
                    beta = fmax(beta, fmax(spectral_radius(q, nx, ny, gamma), spectral_radius(r, nx, ny, gamma)));
                    double jv[4], jx[4], jy[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        jv[v] = r[v] - q[v];
                        jx[v] = rx[v] - qx[v];
                        jy[v] = ry[v] - qy[v];
                    }
                    if (ri) {   // m_n = m . n, m_t = m . (-n_y, n_x)
                        const double a0 = jv[1] * nx + jv[2] * ny, b0 = -jv[1] * ny + jv[2] * nx;
                        const double a1 = jx[1] * nx + jx[2] * ny, b1 = -jx[1] * ny + jx[2] * nx;
                        const double a2 = jy[1] * nx + jy[2] * ny, b2 = -jy[1] * ny + jy[2] * nx;
                        jv[1] = a0; jv[2] = b0; jx[1] = a1; jx[2] = b1; jy[1] = a2; jy[2] = b2;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        S[v][0] = fma(jv[v], jv[v], S[v][0]);
                        S[v][1] = fma(jx[v], jx[v], fma(jy[v], jy[v], S[v][1]));
                    }
                }
                if constexpr (K == 2) {
                    // second derivatives are constant per cell, so both endpoints carry
                    // the same jump: 2 (jxx^2 + 2 jxy^2 + jyy^2)
                    double hn[4][3];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        hessian(wn[v], nxx, nxy, nex, ney, hn[v]);
#pragma unroll
                        for (int d = 0; d < 3; ++d) hn[v][d] -= ho[v][d];
                    }
                    if (ri) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double a0 = hn[1][d] * nx + hn[2][d] * ny, b0 = -hn[1][d] * ny + hn[2][d] * nx;
                            hn[1][d] = a0;
                            hn[2][d] = b0;
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        S[v][2] = 2.0 * (hn[v][0] * hn[v][0] + 2.0 * hn[v][1] * hn[v][1] + hn[v][2] * hn[v][2]);
                }
                const double bh = beta / h;
                double hj = 1.0;
#pragma unroll
                for (int jj = 0; jj <= K; ++jj) {
                    const double f = kA[K][jj] * hj;
                    const double dr = f * inv_r * sqrt(0.5 * S[0][jj]);
                    const double de = f * inv_e * sqrt(0.5 * S[3][jj]);
                    double d1, d2;
                    if (ri) {
                        d1 = d2 = f * inv_m * fmax(sqrt(0.5 * S[1][jj]), sqrt(0.5 * S[2][jj]));
                    } else {
                        d1 = f * inv_1 * sqrt(0.5 * S[1][jj]);
                        d2 = f * inv_2 * sqrt(0.5 * S[2][jj]);
                    }
                    sig[0][jj] = fma(bh, dr, sig[0][jj]);
                    sig[1][jj] = fma(bh, d1, sig[1][jj]);
                    sig[2][jj] = fma(bh, d2, sig[2][jj]);
                    sig[3][jj] = fma(bh, de, sig[3][jj]);
                    hj *= h;
                }
            }
            // exact solution of the damping ODE: degree-m modes scaled by
            // exp(-dt sum_{j<=m} sigma^j); the cell average is untouched (eq. OE:m0)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double acc = sig[v][0];
#pragma unroll
                for (int m = 1; m <= K; ++m) {
                    acc += sig[v][m];
                    const double f = exp(-dt * acc);
#pragma unroll
                    for (int l = m * (m + 1) / 2; l < (m + 1) * (m + 2) / 2; ++l) w[v][l] *= f;
                }
            }
        }

        if (a.bp_enable) {
            // node set: 3 x NE edge Gauss points and two extra points (P1 vertices v1,
            // v2 of eq. 1944; P2 internal nodes of eq. 1139)
            const double n0x = a.m.node_ref[c], n0e = a.m.node_ref[snc + c];
            const double n1x = a.m.node_ref[2 * snc + c], n1e = a.m.node_ref[3 * snc + c];
            // step 1: density
            const double rb = w[0][0];
            double rmin = INFINITY;
#pragma unroll
            for (int t = 0; t < 3 * R::NE + 2; ++t) {
                double x, e, p[NM];
                if (t < 3 * R::NE) edge_point(t / R::NE, R::s[t % R::NE], x, e);
                else if (t == 3 * R::NE) { x = n0x; e = n0e; }
                else { x = n1x; e = n1e; }
                psi<K>(x, e, p);
                double s = w[0][0];
#pragma unroll
                for (int l = 1; l < NM; ++l) s = fma(w[0][l], p[l], s);
                rmin = fmin(rmin, s);
            }
            const double e1 = fmin(rb, kEpsBP);
            const double th1 = rmin >= e1 ? 1.0 : fmin((rb - e1) / (rb - rmin), 1.0);
#pragma unroll
            for (int l = 1; l < NM; ++l) w[0][l] *= th1;
            // step 2: internal energy E - |m|^2 / (2 rho)
            const double ub[4] = {w[0][0], w[1][0], w[2][0], w[3][0]};
            const double eb = internal_energy(ub);
            const double e2 = fmin(eb, kEpsBP);
            double emin = INFINITY;
#pragma unroll
            for (int t = 0; t < 3 * R::NE + 2; ++t) {
                double x, e, p[NM], q[4];
                if (t < 3 * R::NE) edge_point(t / R::NE, R::s[t % R::NE], x, e);
                else if (t == 3 * R::NE) { x = n0x; e = n0e; }
                else { x = n1x; e = n1e; }
                psi<K>(x, e, p);
                eval4<NM>(w, p, q);
                emin = fmin(emin, internal_energy(q));
            }
            const double th2 = emin >= e2 ? 1.0 : fmin((eb - e2) / (eb - emin), 1.0);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int l = 1; l < NM; ++l) w[v][l] *= th2;
            n_lim = (th1 < 1.0 || th2 < 1.0) ? 1 : 0;
            n_bad = (rb > 0.0 && eb > 0.0) ? 0 : 1;
        }

        // max wave speed over the edge Gauss points of the limited state (eq. 1250)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double gx = i == 0 ? -(xx + ex) : (i == 1 ? xx : ex);
            const double gy = i == 0 ? -(xy + ey) : (i == 1 ? xy : ey);
            const double il = 1.0 / a.m.len[i * snc + c];
            const double nx = -2.0 * area * gx * il, ny = -2.0 * area * gy * il;
#pragma unroll
            for (int nu = 0; nu < R::NE; ++nu) {
                double x, e, p[NM], q[4];
                edge_point(i, R::s[nu], x, e);
                psi<K>(x, e, p);
                eval4<NM>(w, p, q);
                const double rr = spectral_radius(q, nx, ny, gamma);
                amax = (rr > amax || rr != rr) ? rr : amax;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NM; ++l) a.uout[(v * NM + l) * snc + c] = w[v][l];
    }

    __shared__ double lds[kBlock / 64][3];
    double red[3] = {amax, (double)n_lim, (double)n_bad};
    const int ops[3] = {2, 0, 0};
    block_reduce<3>(red, ops, lds);
    double* part = a.part + (size_t)gridDim.x * 17;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = red[0];
        if (red[1] > 0) atomicAdd((unsigned long long*)&g->n_limited, (unsigned long long)red[1]);
        if (red[2] > 0) atomicAdd((unsigned long long*)&g->n_bad, (unsigned long long)red[2]);
    }
    if (!arrive_last(&g->ticket[2])) return;
    const int opm[1] = {2};
    double tot[1];
    __shared__ double lds1[kBlock / 64][1];
    reduce_partials<1>(part, 1, gridDim.x, opm, tot, lds1);
    if (threadIdx.x == 0) {
        const double alpha = tot[0];
        g->ticket[2] = 0;
        if (__hip_atomic_load(&g->n_bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) {
            g->err = 1;
            g->active = 0;
        }
        if (a.stage < 2) {
            g->alpha = alpha;
            if (a.stage < 0) g->alpha_step = alpha;
            else if (alpha > g->alpha_step * (1.0 + 1e-12)) g->n_cfl_exc += 1;
        } else {
            g->t += g->dt;
            g->step += 1;
            g->alpha = alpha;
            g->alpha_step = alpha;
        }
        if (a.stage < 0 || a.stage == 2) {
            double dt = g->c_ssp * g->minck / alpha;
            const double rem = g->t_end - g->t;
            if (rem < dt) dt = rem;
            g->dt = dt;
            if (!(isinf(g->t_end) || rem > 1e-12 * fmax(1.0, fabs(g->t_end)))) g->active = 0;
            if (g->err) g->active = 0;
        }
    }
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

// L2 projection (mass diagonal): u^(l) = sum_mu w_mu q(x_mu) Psi_l(x_mu) / (a_l/|K|).
// vx holds the oriented vertex coordinates [6][cell]; for the blast, vx[6][cell]
// flags the cells that own the origin vertex and P.p[4] is their total area.
template <int K>
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
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < NM; ++l) a.uout[(v * NM + l) * snc + c] = acc[v][l];
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

}  // namespace

int launch_residual(int k, const StageArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (k == 1) hipLaunchKernelGGL(k_residual<1>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_residual<2>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a);
    return (int)hipGetLastError();
}

int launch_mnorm(int k, const StageArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (k == 1) hipLaunchKernelGGL(k_mnorm<1>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_mnorm<2>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a);
    return (int)hipGetLastError();
}

int launch_filter(int k, const StageArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (k == 1) hipLaunchKernelGGL(k_filter<1>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_filter<2>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a);
    return (int)hipGetLastError();
}

int launch_project(int k, const StageArgs& a, int kind, const double* dparams, int n_params, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    ProblemParams P{};
    for (int i = 0; i < n_params && i < 20; ++i) P.p[i] = dparams[i];
    const double* vx = a.w;   // the pre-filter buffer carries the coordinates during set-up
    if (k == 1) hipLaunchKernelGGL(k_project<1>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a, kind, P, vx);
    else hipLaunchKernelGGL(k_project<2>, dim3(grid_for(a.m.n_cell)), dim3(kBlock), 0, s, a, kind, P, vx);
    return (int)hipGetLastError();
}

int launch_set_end(Glob* g, double t_end, void* stream) {
    hipLaunchKernelGGL(k_set_end, dim3(1), dim3(64), 0, (hipStream_t)stream, g, t_end);
    return (int)hipGetLastError();
}

}  // namespace oedg
