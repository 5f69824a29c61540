// Kernels of the hyperboloidal outer layer (Section 2.3, item 2).
//
// A context with a layered instance steps with these two-pass kernels: one
// thread per point, Eq. (3) into the half-step array, then Eq. (4).  The
// coefficients are the plain ones of the first-order system (the radial and
// angular tables the other kernels read) turned into the layer's by the
// per-position factors rho', H, rho'' of the map.  Changing to
// (tau, rho) with tau = t - h(r*), h' = H, and Pi~ = Pi / w, w = 1 - H b,
// v = 1 + H b, the system u_tau + D~ u_rho = S~ has
//   D~  = [[bo, 0], [d~, -bi]],  bo = b rho' / w,  bi = b rho' / v,
//   d~  = d rho' / (w^2 v),
//   S~  = (Pi~, ct~ Pi~ + fw [cthth (Phi_thth + cot Phi_th) + c0 Phi + F]),
//   ct~ = (ct w + d H + b^2 rho' rho'' - b H b') / (w v),  fw = 1 / (w v).
// Outside the layer (H = 0) these are the plain coefficients, bit for bit.
// At null infinity rho' -> 0 and the ingoing speed bi vanishes: no
// characteristic enters, and the last node takes the linear extrapolation
// 2 u_{N-2} - u_{N-3} of the new values.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_layer_launch.h"

namespace tk {

namespace {

struct LCoef {
    double bo, bi, cthth, cth, fw;
    cd ct, c0, d;
};

__device__ __forceinline__ LCoef lcoef_at(const Radial &R, const Angular &A, const LayerTab *tab, int q)
{
    const Coef<double> c = coef_at(R, A);
    LCoef o;
    o.bo = o.bi = c.b;
    o.cthth = c.cthth;
    o.cth = c.cth;
    o.fw = 1.0;
    o.ct = c.ct;
    o.c0 = c.c0;
    o.d = c.d;
    if (tab == nullptr) return o;
    const LayerTab L = load_entry(gload_ptr(tab) + q);
    if (L.H == 0.0) return o;
    const double Sh2 = R.rho2 - R.a2D * A.sn2;
    const double Sh = sqrt(Sh2);
    const double W = 1.0 / Sh2;
    const double bp = R.K * A.sn2 * W * sqrt(W);  // b' = d b / d r*
    // w = rho' b + (1 - b), with 1 - b = -a^2 Delta sin^2 / (Sh (Sh + rho)):
    // near null infinity 1 - b is far below the rounding of b
    const double omb = -(R.a2D * A.sn2) / (Sh * (Sh + R.rho));
    const double w = L.rhop * c.b + omb;
    const double v = 1.0 + L.H * c.b;
    const double fw = 1.0 / (w * v);  // the one division: 1/w = v fw, 1/v = w fw
    const double brp = c.b * L.rhop;
    o.bo = brp * (v * fw);
    o.bi = brp * (w * fw);
    const double dd = L.rhop * (v * fw) * fw;
    o.d = mk(c.d.re * dd, c.d.im * dd);
    const double g = c.b * c.b * L.rhop * L.rhopp - c.b * L.H * bp;
    o.ct = mk((c.ct.re * w + c.d.re * L.H + g) * fw, (c.ct.im * w + c.d.im * L.H) * fw);
    o.fw = fw;
    o.cthth = c.cthth * fw;
    o.cth = c.cth * fw;
    o.c0 = mk(c.c0.re * fw, c.c0.im * fw);
    return o;
}

// out = base - fac [ D~ du / h - S~ ] at one point (Eq. (3) with the
// averaged fields as base and fac = dt/2, Eq. (4) with u^n and fac = dt).
__device__ __forceinline__ P4 lw_layer(const LCoef &c, const P4 &base, cd phm, cd ph0, cd php, cd pi0, const P4 &du,
                                       double fac, const DevInst &I, cd F)
{
    const cd d2 = I.inv_dth2 * (php - 2.0 * ph0 + phm);
    const cd d1 = I.inv_2dth * (php - phm);
    const cd spi = cmul(c.ct, pi0) + c.cthth * d2 + c.cth * d1 + cmul(c.c0, ph0) + c.fw * F;
    const cd adv_phi = I.inv_h * (c.bo * du.phi);
    const cd adv_pi = I.inv_h * (cmul(c.d, du.phi) - c.bi * du.pi);
    const cd bphi = adv_phi - pi0, bpi = adv_pi - spi;
    return P4{base.phi - fac * bphi, base.pi - fac * bpi};
}

__device__ __forceinline__ cd source_at(const DevInst &I, const Radial &R, const Angular &A, double t)
{
    return R.srcg * A.srcg != 0.0 ? source_value(R.srcg, A.srcg, source_phase(I, t)) : mk(0, 0);
}

// Eq. (3) at half node i+1/2, row j (1 <= j <= n_theta - 2)
__device__ P4 half_at(const DevInst &I, const LayerTab *tab, const double4 *u, int i, int j, double t)
{
    const int p = I.pitch;
    const P4 a0 = ld_p4(u + (size_t)j * p + i), a1 = ld_p4(u + (size_t)j * p + i + 1);
    const P4 am0 = ld_p4(u + (size_t)(j - 1) * p + i), am1 = ld_p4(u + (size_t)(j - 1) * p + i + 1);
    const P4 ap0 = ld_p4(u + (size_t)(j + 1) * p + i), ap1 = ld_p4(u + (size_t)(j + 1) * p + i + 1);
    const P4 bar = half_sum(a1, a0);
    const cd phm = half_sum(am1, am0).phi, php = half_sum(ap1, ap0).phi;
    const Radial R = load_entry(gload_ptr(I.rad) + (2 * i + 1));
    const Angular A = load_entry(gload_ptr(I.ang) + j);
    const LCoef c = lcoef_at(R, A, tab, 2 * i + 1);
    return lw_layer(c, bar, phm, bar.phi, php, bar.pi, a1 - a0, 0.5 * I.dt, I, source_at(I, R, A, t));
}

// Eq. (4) at node i, row j (1 <= i <= n_r - 2, 1 <= j <= n_theta - 2)
__device__ P4 full_at(const DevInst &I, const LayerTab *tab, const double4 *u, const double4 *hf, int i, int j,
                      double t)
{
    const int p = I.pitch;
    const P4 h0 = ld_p4(hf + (size_t)j * p + i - 1), h1 = ld_p4(hf + (size_t)j * p + i);
    const P4 hm0 = ld_p4(hf + (size_t)(j - 1) * p + i - 1), hm1 = ld_p4(hf + (size_t)(j - 1) * p + i);
    const P4 hp0 = ld_p4(hf + (size_t)(j + 1) * p + i - 1), hp1 = ld_p4(hf + (size_t)(j + 1) * p + i);
    const P4 til = half_sum(h1, h0);
    const cd phm = half_sum(hm1, hm0).phi, php = half_sum(hp1, hp0).phi;
    const Radial R = load_entry(gload_ptr(I.rad) + (2 * i));
    const Angular A = load_entry(gload_ptr(I.ang) + j);
    const LCoef c = lcoef_at(R, A, tab, 2 * i);
    const P4 un = ld_p4(u + (size_t)j * p + i);
    return lw_layer(c, un, phm, til.phi, php, til.pi, h1 - h0, I.dt, I, source_at(I, R, A, t));
}

// u^{n+1} at the last node of a layered instance, row j (1 <= j <= n_theta - 2)
__device__ P4 scri_at(const DevInst &I, const LayerTab *tab, const double4 *u, const double4 *hf, int j, double t)
{
    const int n = I.n_r;
    const P4 a = full_at(I, tab, u, hf, n - 2, j, t), b = full_at(I, tab, u, hf, n - 3, j, t);
    return P4{mk(2.0 * a.phi.re - b.phi.re, 2.0 * a.phi.im - b.phi.im),
              mk(2.0 * a.pi.re - b.pi.re, 2.0 * a.pi.im - b.pi.im)};
}

__global__ void __launch_bounds__(256) k_layer_half(const DevInst *__restrict__ insts,
                                                    const LayerInst *__restrict__ lays,
                                                    const int2 *__restrict__ blocks, const DevCtl *__restrict__ ctl,
                                                    int kstep, int kflip)
{
    const int2 bl = blocks[blockIdx.x];
    const DevInst &I = insts[bl.x];
    const LayerTab *tab = lays[bl.x].on ? lays[bl.x].tab : nullptr;
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    const double4 *u = (const double4 *)I.u[b];
    double4 *hf = (double4 *)I.half;
    const int L = bl.y * 256 + (int)threadIdx.x;
    const int j = L / I.n_r, i = L - j * I.n_r;
    if (j >= I.n_theta || i >= I.n_r - 1) return;
    const double t = (double)n * I.dt;
    const int nt = I.n_theta;
    P4 out;
    if (j >= 1 && j <= nt - 2) {
        out = half_at(I, tab, u, i, j, t);
    } else if (!I.m_even) {
        out = zero4();
    } else {
        const int j1 = j == 0 ? 1 : nt - 2, j2 = j == 0 ? 2 : nt - 3;
        out = pole_bc(half_at(I, tab, u, i, j1, t), half_at(I, tab, u, i, j2, t));
    }
    st_p4(hf + (size_t)j * I.pitch + i, out);
}

__global__ void __launch_bounds__(256) k_layer_full(const DevInst *__restrict__ insts,
                                                    const LayerInst *__restrict__ lays,
                                                    const int2 *__restrict__ blocks, const DevCtl *__restrict__ ctl,
                                                    int kstep, int kflip)
{
    const int2 bl = blocks[blockIdx.x];
    const DevInst &I = insts[bl.x];
    const LayerTab *tab = lays[bl.x].on ? lays[bl.x].tab : nullptr;
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    const double4 *u = (const double4 *)I.u[b];
    double4 *un = (double4 *)I.u[b ^ 1];
    const double4 *hf = (const double4 *)I.half;
    const int L = bl.y * 256 + (int)threadIdx.x;
    const int j = L / I.n_r, i = L - j * I.n_r;
    if (j >= I.n_theta) return;
    const double t = (double)n * I.dt + 0.5 * I.dt;
    const int nt = I.n_theta;
    const bool scri = i == I.n_r - 1 && tab != nullptr;
    P4 out;
    if (i == 0 || (i == I.n_r - 1 && !scri)) {
        out = zero4();
    } else if (j >= 1 && j <= nt - 2) {
        out = scri ? scri_at(I, tab, u, hf, j, t) : full_at(I, tab, u, hf, i, j, t);
    } else if (!I.m_even) {
        out = zero4();
    } else {
        const int j1 = j == 0 ? 1 : nt - 2, j2 = j == 0 ? 2 : nt - 3;
        out = scri ? pole_bc(scri_at(I, tab, u, hf, j1, t), scri_at(I, tab, u, hf, j2, t))
                   : pole_bc(full_at(I, tab, u, hf, i, j1, t), full_at(I, tab, u, hf, i, j2, t));
    }
    st_p4(un + (size_t)j * I.pitch + i, out);
    if (i == I.i_obs && I.extract_every > 0 && (n + 1) % I.extract_every == 0) {
        const long long k = (n + 1) / I.extract_every - 1;
        TK_GLOBAL double *w = gstore_ptr(I.wave) + ((size_t)(k % I.wave_cap) * nt + j) * 2;
        w[0] = out.phi.re;
        w[1] = out.phi.im;
    }
}

}  // namespace

hipError_t launch_layer(const DevInst *d_inst, const LayerInst *d_lay, const int2 *d_blocks, int n_blocks,
                        const DevCtl *ctl, int kstep, int kflip, hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_layer_half, dim3(n_blocks), dim3(256), 0, s, d_inst, d_lay, d_blocks, ctl, kstep, kflip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_layer_full, dim3(n_blocks), dim3(256), 0, s, d_inst, d_lay, d_blocks, ctl, kstep, kflip);
    return hipGetLastError();
}

}  // namespace tk
