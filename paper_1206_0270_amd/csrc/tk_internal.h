// Internal layout shared by the host setup (tk_setup.cpp, tk_api.cpp) and the
// HIP kernels (tk_kernels.hip).  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/tk.h"

namespace tk {

// Radial factors of the first-order system at one radial position q
// (q = 2i: node i, q = 2i+1: half node i+1/2).  With
//   Sh2 = rho2 - a2D sin^2,  W = 1/Sh2,  sig = sqrt(W)
// the coefficients of u_t + D u_{r*} = S (D = [[b, 0], [d, -b]],
// S = (Pi, ct Pi + cthth (Phi_thth + cot Phi_th) + c0 Phi + F)) are
//   b     = rho sig
//   cthth = Dl W
//   ct    = W (ct_re + i (ct_im0 + ct_imc cos))
//   c1    = W (c1_re + i c1_im)
//   c0    = W (c0_re - Dl V(theta) + i c0_im)
//   b'    = K sin^2 W sig
//   d     = -(c1 - b b' - b ct)
// These are the terms of Eq. (1) after the m-mode decomposition of Eq. (2)
// in the Kerr azimuth, divided by the Psi_tt coefficient.
struct alignas(16) Radial {
    double rho2, a2D, rho, Dl;
    double ct_re, ct_im0, ct_imc, K;
    double c1_re, c1_im, c0_re, c0_im;
    double rstar;
    double srcg;  // amplitude * g_r(r* - r*_p) of the particle source (0 off its window)
    double pad1, pad2;
};
static_assert(sizeof(Radial) == 128, "Radial must stay 128 bytes");

// Angular factors at row j (rows 1 .. n_theta-2; pole rows unused).
struct alignas(16) Angular {
    double sn2, cs, cot, V;  // sin^2, cos, cot, (m + s cos)^2/sin^2 - s
    double theta;
    double srcg;   // g_theta(theta - pi/2) of the particle source (0 off its window)
    // The same, scaled for the fused kernels' radial factor D2h = Delta /
    // (2 dtheta^2): a^2 Delta sin^2 = D2h sa, kct Delta cos = D2h kcs,
    // Delta V = D2h V2; and cot dtheta / 2.
    double cot_h, sa, kcs, V2;
    double pad1, pad2;
};
static_assert(sizeof(Angular) == 96, "Angular must stay 96 bytes");

// The fused kernels' angular factors in float (FP32 form).
struct alignas(16) AngularF {
    float sa, sn2, kcs, V2, cot_h, pad1, pad2, pad3;
};

// One instance as the kernels see it (device memory, read-only in kernels).
struct alignas(16) DevInst {
    // grid
    int n_r, n_theta, pitch, m_even;  // m_even: m + s even (Neumann poles), else zero poles
    int m, i_obs, extract_every, wave_cap;
    double h, dth, dt, inv_h;
    double inv_dth2, inv_2dth, rstar_min, pad0;
    // state: two buffers of n_theta rows x pitch points.  FP64 mode: double4
    // (Phi.re, Phi.im, Pi.re, Pi.im).  FP32 mode: float4 values + ushort4
    // bf16 compensation terms.
    void *u[2];
    void *c[2];
    void *half;  // two-pass kernel's half-step array (FP64, n_theta x pitch)
    const Radial *rad;     // [2 n_r - 1]
    const Angular *ang;    // [n_theta]
    const AngularF *angf;  // [n_theta]
    double *wave;          // [wave_cap][n_theta][2]
    // source
    int src_kind;
    int lay_c0;  // first column whose half node lies beyond rho = R (n_r without a layer)
    int pad2, pad3;
    double src_amp, src_phase0, src_Omega, src_rstar_p;
    double src_sig_r, src_sig_th, src_win, src_t0;
    double a2, kct;        // a^2 and -2 s a (to rebuild a^2 Delta and Im ct's cos part)
    double src_ramp_inv, pad6;  // 1 / T_on of the source's switch-on (0: none)
    // hyperboloidal layer: the instance's LayerTab table [2 n_r - 1] (the
    // map factors rho', H, rho'' per radial position), or null without one
    // (its first column: lay_c0 above)
    const void *lay;
    long long lay_on;
};

// Fused-kernel work item: a block of columns [i0, i0 + width) x rows [j0, j1)
struct alignas(16) WorkItem {
    int inst, i0, j0, j1;
};

// Device-resident control block of a context.
struct alignas(16) DevCtl {
    long long step;  // step counter n (time of instance k = n dt_k)
    long long cur;   // state buffer (0 or 1) holding u^n; every launch flips it
    long long pad[6];
};

// Host-side description after validation (one per instance).
struct HostInst {
    tk_instance_desc desc;
    tk_source_desc src;
    double h, dth, rp, rm;
    double src_Omega, src_rstar_p;
    int i_obs, pitch, wave_cap;
    size_t off_u[2], off_c[2], off_half, off_rad, off_ang, off_angf, off_wave;  // workspace offsets
    long long wave_drained;  // samples already handed out
};

// Time-independent factors of the smeared particle source: with
// g(xi) = exp(-xi^2/(2 sig^2)) / (sig sqrt(2 pi)) cut at |xi| > win sig,
// F(t, r*_q, theta_j) = [A g_r(q)] g_theta(j) exp(-i m (Omega t + phase0)).
void fill_source(const HostInst &hi, Radial *rad, Angular *ang);

// Host-side setup (tk_setup.cpp)
double tortoise_of_x(double M, double a, double x);
double x_of_tortoise(double M, double a, double rstar);
void fill_radial(const HostInst &hi, Radial *rad);
void fill_angular(const HostInst &hi, Angular *ang);
double stable_dt_bound(const tk_instance_desc &d);
double orbit_frequency(double M, double a, double r0);

}  // namespace tk
