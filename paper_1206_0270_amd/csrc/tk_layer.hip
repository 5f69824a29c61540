// Kernels of the hyperboloidal outer layer (Section 2.3, item 2).
//
// A layered context steps with the marching kernels' layered form
// (tk_kernels.hip); these kernels are the alternative FP64 form, one step
// in two passes over whole instances: k_layer_half (Eq. (3) into the
// half-step array) and k_layer_full (Eq. (4)), then k_layer_scri for the
// null-infinity column.  They march chunks of theta rows with their radial
// factors in registers.
// Their coefficients are the plain ones of the first-order system (the
// radial and angular tables the other kernels read) turned into the layer's
// by the per-position factors rho', H, rho'' of the map.  Changing to
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

// Coefficients of the layer system at one point from the radial record R
// (held in registers for a whole march), the row's angular record A and the
// position's map factors L, read from the table in global memory where they
// are used (nullptr outside a layered instance).  The pointer goes to the
// table itself, not to a local copy: a pointer selected between a local
// record and null keeps the record in scratch memory, and a copy held in
// registers for the whole march costs the kernel its second wave.  1/sqrt is
// the hardware estimate refined by Newton steps, as in the fused kernels.
__device__ __forceinline__ LCoef lcoef_of(const Radial &R, const Angular &A, const TK_GLOBAL LayerTab *L)
{
    const double Sh2 = R.rho2 - R.a2D * A.sn2;
    const double sig = inv_sqrt(Sh2);  // 1 / Sigma-hat
    const double W = sig * sig;
    const double b = R.rho * sig;
    LCoef o;
    o.cthth = R.Dl * W;
    o.cth = o.cthth * A.cot;
    o.ct = mk(W * R.ct_re, W * (R.ct_im0 + R.ct_imc * A.cs));
    o.c0 = mk(W * (R.c0_re - R.Dl * A.V), W * R.c0_im);
    const double bp = R.K * A.sn2 * W * sig;  // b' = d b / d r*
    // d = -(c1 - b b' - b ct)
    o.d = mk(b * bp + b * o.ct.re - W * R.c1_re, b * o.ct.im - W * R.c1_im);
    o.bo = o.bi = b;
    o.fw = 1.0;
    if (L == nullptr || L->H == 0.0) return o;
    // w = rho' b + (1 - b), with 1 - b = -a^2 Delta sin^2 / (Sh (Sh + rho)):
    // near null infinity 1 - b is far below the rounding of b
    const double Sh = Sh2 * sig;
    const double omb = -(R.a2D * A.sn2) / (Sh * (Sh + R.rho));
    const double w = L->rhop * b + omb;
    const double v = 1.0 + L->H * b;
    const double fw = 1.0 / (w * v);  // 1/w = v fw, 1/v = w fw
    const double brp = b * L->rhop;
    o.bo = brp * (v * fw);
    o.bi = brp * (w * fw);
    const double dd = L->rhop * (v * fw) * fw;
    const double g = b * b * L->rhop * L->rhopp - b * L->H * bp;
    o.ct = mk((o.ct.re * w + o.d.re * L->H + g) * fw, (o.ct.im * w + o.d.im * L->H) * fw);
    o.d = mk(o.d.re * dd, o.d.im * dd);
    o.fw = fw;
    o.cthth *= fw;
    o.cth *= fw;
    o.c0 = mk(o.c0.re * fw, o.c0.im * fw);
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

__device__ __forceinline__ Angular angular_row(const DevInst &I, int j) { return load_entry(cload_ptr(I.ang) + j); }

__device__ __forceinline__ cd source_of(const DevInst &I, double gq, const Angular &A, cd e)
{
    return gq * A.srcg != 0.0 ? source_value(gq, A.srcg, e) : mk(0, 0);
}

__device__ __forceinline__ const double4 *row_ptr(const void *base, const DevInst &I, int j)
{
    return (const double4 *)base + (size_t)j * I.pitch;
}

// Eq. (3): one wave per work item, lane = half node i + 1/2 (i = i0 + lane),
// marching the item's rows with u^n rows j-1, j, j+1 of columns i, i+1 in
// registers.  A chunk that holds a pole row forms it after its rows 1, 2 (or
// n_theta - 3, n_theta - 2) from those values; the work list keeps such
// chunks at least three rows long.
__global__ void __launch_bounds__(256) k_layer_half(const DevInst *__restrict__ insts,
                                                    const LayerInst *__restrict__ lays,
                                                    const WorkItem *__restrict__ work, int n_work,
                                                    const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    const int w = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= n_work) return;
    const WorkItem it = work[w];
    const DevInst &I = insts[it.inst];
    const int i = it.i0 + (int)(threadIdx.x & 63);
    if (i >= I.n_r - 1) return;
    const LayerTab *tab = lays[it.inst].on ? lays[it.inst].tab : nullptr;
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    const double t = (double)n * I.dt;
    const cd e = source_phase(I, t);
    const int nt = I.n_theta;
    const int q = 2 * i + 1;
    const Radial R = load_entry(gload_ptr(I.rad) + q);
    const TK_GLOBAL LayerTab *L = tab ? gload_ptr(tab) + q : nullptr;
    double4 *hf = (double4 *)I.half;
    const int jb = it.j0 > 1 ? it.j0 : 1, je = it.j1 < nt - 1 ? it.j1 : nt - 1;
    P4 m0 = ld_p4(row_ptr(I.u[b], I, jb - 1) + i), m1 = ld_p4(row_ptr(I.u[b], I, jb - 1) + i + 1);
    P4 c0 = ld_p4(row_ptr(I.u[b], I, jb) + i), c1 = ld_p4(row_ptr(I.u[b], I, jb) + i + 1);
    P4 h1 = zero4(), h2 = zero4(), last = zero4(), before = zero4();
    for (int j = jb; j < je; ++j) {
        const P4 p0 = ld_p4(row_ptr(I.u[b], I, j + 1) + i), p1 = ld_p4(row_ptr(I.u[b], I, j + 1) + i + 1);
        const Angular A = angular_row(I, j);
        const LCoef c = lcoef_of(R, A, L);
        const P4 bar = half_sum(c1, c0);
        const P4 out = lw_layer(c, bar, half_sum(m1, m0).phi, bar.phi, half_sum(p1, p0).phi, bar.pi, c1 - c0,
                                0.5 * I.dt, I, source_of(I, R.srcg, A, e));
        st_p4(hf + (size_t)j * I.pitch + i, out);
        if (j == 1) h1 = out;
        if (j == 2) h2 = out;
        before = last;
        last = out;
        m0 = c0;
        m1 = c1;
        c0 = p0;
        c1 = p1;
    }
    if (it.j0 == 0) st_p4(hf + i, I.m_even ? pole_bc(h1, h2) : zero4());
    if (it.j1 == nt) st_p4(hf + (size_t)(nt - 1) * I.pitch + i, I.m_even ? pole_bc(last, before) : zero4());
}

// Eq. (4): lane = node i, marching the item's rows with the half-step rows
// j-1, j, j+1 of half nodes i - 1/2, i + 1/2 in registers; pole rows as in
// k_layer_half; Dirichlet at i = 0 and at the last node of a plain
// instance.  The last node of a layered instance is left to k_layer_scri.
__global__ void __launch_bounds__(256) k_layer_full(const DevInst *__restrict__ insts,
                                                    const LayerInst *__restrict__ lays,
                                                    const WorkItem *__restrict__ work, int n_work,
                                                    const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    const int w = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= n_work) return;
    const WorkItem it = work[w];
    const DevInst &I = insts[it.inst];
    const int i = it.i0 + (int)(threadIdx.x & 63);
    if (i >= I.n_r) return;
    const LayerTab *tab = lays[it.inst].on ? lays[it.inst].tab : nullptr;
    if (i == I.n_r - 1 && tab) return;
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    double4 *un = (double4 *)I.u[b ^ 1];
    const int nt = I.n_theta;
    const bool sampling = i == I.i_obs && I.extract_every > 0 && (n + 1) % I.extract_every == 0;
    TK_GLOBAL double *wv = nullptr;
    if (sampling) wv = gstore_ptr(I.wave) + (size_t)(((n + 1) / I.extract_every - 1) % I.wave_cap) * nt * 2;
    if (i == 0 || i == I.n_r - 1) {
        for (int j = it.j0; j < it.j1; ++j) {
            st_p4(un + (size_t)j * I.pitch + i, zero4());
            if (sampling) wv[2 * j] = wv[2 * j + 1] = 0.0;
        }
        return;
    }
    const double t = (double)n * I.dt + 0.5 * I.dt;
    const cd e = source_phase(I, t);
    const int q = 2 * i;
    const Radial R = load_entry(gload_ptr(I.rad) + q);
    const TK_GLOBAL LayerTab *L = tab ? gload_ptr(tab) + q : nullptr;
    const int jb = it.j0 > 1 ? it.j0 : 1, je = it.j1 < nt - 1 ? it.j1 : nt - 1;
    P4 m0 = ld_p4(row_ptr(I.half, I, jb - 1) + i - 1), m1 = ld_p4(row_ptr(I.half, I, jb - 1) + i);
    P4 c0 = ld_p4(row_ptr(I.half, I, jb) + i - 1), c1 = ld_p4(row_ptr(I.half, I, jb) + i);
    P4 h1 = zero4(), h2 = zero4(), last = zero4(), before = zero4();
    for (int j = jb; j < je; ++j) {
        const P4 p0 = ld_p4(row_ptr(I.half, I, j + 1) + i - 1), p1 = ld_p4(row_ptr(I.half, I, j + 1) + i);
        const P4 uo = ld_p4(row_ptr(I.u[b], I, j) + i);
        const Angular A = angular_row(I, j);
        const LCoef c = lcoef_of(R, A, L);
        const P4 til = half_sum(c1, c0);
        const P4 out = lw_layer(c, uo, half_sum(m1, m0).phi, til.phi, half_sum(p1, p0).phi, til.pi, c1 - c0, I.dt, I,
                                source_of(I, R.srcg, A, e));
        st_p4(un + (size_t)j * I.pitch + i, out);
        if (sampling) {
            wv[2 * j] = out.phi.re;
            wv[2 * j + 1] = out.phi.im;
        }
        if (j == 1) h1 = out;
        if (j == 2) h2 = out;
        before = last;
        last = out;
        m0 = c0;
        m1 = c1;
        c0 = p0;
        c1 = p1;
    }
    if (it.j0 == 0) {
        const P4 o = I.m_even ? pole_bc(h1, h2) : zero4();
        st_p4(un + i, o);
        if (sampling) {
            wv[0] = o.phi.re;
            wv[1] = o.phi.im;
        }
    }
    if (it.j1 == nt) {
        const P4 o = I.m_even ? pole_bc(last, before) : zero4();
        st_p4(un + (size_t)(nt - 1) * I.pitch + i, o);
        if (sampling) {
            wv[2 * (nt - 1)] = o.phi.re;
            wv[2 * (nt - 1) + 1] = o.phi.im;
        }
    }
}

// The last node of each layered instance (future null infinity): the linear
// extrapolation 2 u_{N-2} - u_{N-3} of the new values on rows 1 .. n_theta-2,
// then the pole rows from its rows 1, 2 (n_theta-2, n_theta-3).  One block
// per instance, threads striding over rows.
__global__ void __launch_bounds__(256) k_layer_scri(const DevInst *__restrict__ insts,
                                                    const LayerInst *__restrict__ lays, const DevCtl *__restrict__ ctl,
                                                    int kstep, int kflip)
{
    const int k = blockIdx.x;
    if (!lays[k].on) return;
    const DevInst &I = insts[k];
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    double4 *un = (double4 *)I.u[b ^ 1];
    const int nt = I.n_theta, N = I.n_r;
    const bool sampling = I.i_obs == N - 1 && I.extract_every > 0 && (n + 1) % I.extract_every == 0;
    TK_GLOBAL double *wv = nullptr;
    if (sampling) wv = gstore_ptr(I.wave) + (size_t)(((n + 1) / I.extract_every - 1) % I.wave_cap) * nt * 2;
    auto ext = [&](int j) {
        const P4 a = ld_p4(un + (size_t)j * I.pitch + N - 2);
        const P4 c = ld_p4(un + (size_t)j * I.pitch + N - 3);
        return P4{mk(2.0 * a.phi.re - c.phi.re, 2.0 * a.phi.im - c.phi.im),
                  mk(2.0 * a.pi.re - c.pi.re, 2.0 * a.pi.im - c.pi.im)};
    };
    for (int j = (int)threadIdx.x; j < nt; j += (int)blockDim.x) {
        P4 o;
        if (j >= 1 && j <= nt - 2)
            o = ext(j);
        else if (!I.m_even)
            o = zero4();
        else
            o = j == 0 ? pole_bc(ext(1), ext(2)) : pole_bc(ext(nt - 2), ext(nt - 3));
        st_p4(un + (size_t)j * I.pitch + N - 1, o);
        if (sampling) {
            wv[2 * j] = o.phi.re;
            wv[2 * j + 1] = o.phi.im;
        }
    }
}

}  // namespace

hipError_t launch_layer(const DevInst *d_inst, const LayerInst *d_lay, int n_inst, const WorkItem *d_work, int n_work,
                        const DevCtl *ctl, int kstep, int kflip, hipStream_t s)
{
    if (n_work <= 0) return hipSuccess;
    const int blocks = (n_work + 3) / 4;
    hipLaunchKernelGGL(k_layer_half, dim3(blocks), dim3(256), 0, s, d_inst, d_lay, d_work, n_work, ctl, kstep, kflip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_layer_full, dim3(blocks), dim3(256), 0, s, d_inst, d_lay, d_work, n_work, ctl, kstep, kflip);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_layer_scri, dim3(n_inst), dim3(256), 0, s, d_inst, d_lay, ctl, kstep, kflip);
    return hipGetLastError();
}

}  // namespace tk
