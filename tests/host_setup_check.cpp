// Test driver: prints the library's host-side setup values (inverse tortoise
// coordinate, radial and angular tables, source tables) so that tests/test_host_setup.py can
// compare them with closed forms and with the oracle.  Built with g++ by the
// test; links the library's own tk_setup.cpp.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tk_internal.h"

int main(int argc, char **argv)
{
    if (argc < 9) return 2;
    tk_instance_desc d{};
    d.M = atof(argv[1]);
    d.a = atof(argv[2]);
    d.s = atoi(argv[3]);
    d.m = atoi(argv[4]);
    d.n_r = atoi(argv[5]);
    d.n_theta = atoi(argv[6]);
    d.rstar_min = atof(argv[7]);
    d.rstar_max = atof(argv[8]);
    d.dt = 0.01;
    tk::HostInst h{};
    h.desc = d;
    h.h = (d.rstar_max - d.rstar_min) / (d.n_r - 1);
    h.dth = M_PI / (d.n_theta - 1);
    double q = __builtin_sqrt((d.M - d.a) * (d.M + d.a));
    h.rp = d.M + q;
    h.rm = d.M - q;
    std::vector<tk::Radial> rad(2 * d.n_r - 1);
    std::vector<tk::Angular> ang(d.n_theta);
    tk::fill_radial(h, rad.data());
    tk::fill_angular(h, ang.data());
    for (size_t k = 0; k < rad.size(); ++k) {
        const tk::Radial &R = rad[k];
        printf("R %zu %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", k, R.rstar,
               R.rho2, R.a2D, R.rho, R.Dl, R.ct_re, R.ct_im0, R.ct_imc, R.K, R.c1_re, R.c1_im, R.c0_re, R.c0_im);
    }
    for (int j = 0; j < d.n_theta; ++j)
        printf("A %d %.17g %.17g %.17g %.17g %.17g\n", j, ang[j].theta, ang[j].sn2, ang[j].cs, ang[j].cot, ang[j].V);
    printf("B %.17g\n", tk::stable_dt_bound(d));
    if (argc >= 11) {  // source tables: kind, r0 (amplitude 1, widths 2 cells, window 6 sigma)
        h.src.kind = atoi(argv[9]);
        h.src.r0 = atof(argv[10]);
        h.src.amplitude = 1.0;
        h.src.sigma_r_cells = h.src.sigma_th_cells = 2.0;
        h.src.window_sigmas = 6.0;
        h.src_rstar_p = tk::tortoise_of_x(d.M, d.a, h.src.r0 - h.rp);
        tk::fill_source(h, rad.data(), ang.data());
        printf("P %.17g\n", h.src_rstar_p);
        for (size_t k = 0; k < rad.size(); ++k) printf("S %zu %.17g %.17g\n", k, rad[k].rstar, rad[k].srcg);
        for (int j = 0; j < d.n_theta; ++j) printf("T %d %.17g %.17g\n", j, ang[j].theta, ang[j].srcg);
    }
    return 0;
}
