// Hyperboloidal outer layer (Section 2.3, item 2): its tables and host
// setup (no HIP types here; the launcher is in tk_layer_launch.h).
//
// On rho in [R, S] (R = layer_start > 0, S = rstar_max) the grid coordinate
// rho is compactified, r* = rho / Omega(rho) with
// Omega = 1 - ((rho - R) / (S - R))^4, so that the last node rho = S is
// future null infinity; the time there is tau = t - h(r*) with
// h' = H = 1 - rho', rho' = d rho / d r*.  Outgoing rays keep unit speed in
// rho, ingoing ones stop at S, and the evolved pair is (Phi, Pi~) with
// Pi~ = Pi / (1 - H b).  Below R everything is as without the layer
// (rho = r*, tau = t, Pi~ = Pi).
#pragma once

#include "tk_internal.h"

namespace tk {

// Layer factors at one radial position q (node or half node), from the map
// alone: rho', H = 1 - rho', rho'' = d rho' / d rho.  (1, 0, 0) below R.
struct alignas(16) LayerTab {
    double rhop, H, rhopp, pad;
};
static_assert(sizeof(LayerTab) == 32, "LayerTab must stay 32 bytes");

// Per-instance layer descriptor on the device: tab[2 n_r - 1] for an
// instance with a layer (its last node is then null infinity), nullptr for
// one without (Dirichlet at the last node, as in the other kernels).
struct alignas(16) LayerInst {
    const LayerTab *tab;
    long long on;
};

// The map at grid position rho: r*, rho', H, rho''.  rho <= R gives (rho, 1, 0, 0).
void layer_map(double R, double S, double rho, double *rstar, double *rhop, double *H, double *rhopp);

// Layer factors for the 2 n_r - 1 radial positions of a layered instance.
void fill_layer(const HostInst &hi, LayerTab *tab);

}  // namespace tk
