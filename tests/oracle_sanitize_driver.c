/* Test driver: the oracle compiled together with this file under AddressSanitizer
 * and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  It runs small
 * grids with every source kind, with and without the switch-on, both pole
 * rules, with and without a hyperboloidal layer, and reads back the state and
 * the waveform. */
#include "../oracle/teuk_oracle.c"

#include <stdio.h>

static int run_case(double a, int s, int m, int n_r, int n_theta, int kind, double ramp, double layer_R)
{
    or_desc d;
    memset(&d, 0, sizeof d);
    d.M = 1.0;
    d.a = a;
    d.s = s;
    d.m = m;
    d.n_r = n_r;
    d.n_theta = n_theta;
    d.rstar_min = -20.0;
    d.rstar_max = 30.0;
    d.dt = 0.02;
    d.i_obs = n_r - 5;
    d.extract_every = 3;
    d.src_kind = kind;
    d.src_r0 = 7.5;
    d.src_amp = 1.0;
    d.src_phase0 = 0.4;
    d.src_sigma_r_cells = 2.0;
    d.src_sigma_th_cells = 2.0;
    d.src_window_sigmas = 6.0;
    d.src_t0 = 3.0;
    d.src_ramp = ramp;
    d.layer_R = layer_R;
    if (layer_R != 0) d.i_obs = n_r - 1;  /* read the waveform at null infinity */
    void *g = or_grid_new(&d);
    if (!g) return 1;
    size_t npt = (size_t)n_r * n_theta;
    double *phi = calloc(2 * npt, sizeof(double)), *pi = calloc(2 * npt, sizeof(double));
    for (size_t p = 0; p < 2 * npt; ++p) phi[p] = 1e-3 * (double)((p * 2654435761u) % 1000) / 1000.0;
    or_set_state(g, phi, pi, 0);
    long samples = or_run(g, 60);  /* samples in the waveform ring */
    or_get_state(g, phi, pi);
    double wave[64 * 2 * 64];
    long n = or_get_wave(g, wave, 64);
    double out[2];
    or_source_value(g, 1.0, 7.0, 1.5, out);
    int bad = samples != 20 || n != 20;
    if (bad) fprintf(stderr, "case a=%g m=%d kind=%d: %ld / %ld samples\n", a, m, kind, samples, n);
    for (size_t p = 0; p < 2 * npt; ++p) bad |= !isfinite(phi[p]) || !isfinite(pi[p]);
    or_grid_free(g);
    free(phi);
    free(pi);
    return bad;
}

int main(void)
{
    int bad = 0;
    for (int kind = 0; kind <= 3; ++kind) {
        bad |= run_case(0.9, -2, 2, 41, 9, kind, 0.0, 0.0);
        bad |= run_case(0.6, -2, 3, 37, 10, kind, 0.5, 0.0);
        bad |= run_case(0.0, 1, -2, 30, 7, kind, 0.0, 0.0);
        bad |= run_case(0.7, -2, 2, 43, 9, kind, 0.3, 20.0);  /* hyperboloidal layer on [20, 30] */
    }
    printf("%s\n", bad ? "FAILED" : "ok");
    return bad;
}
