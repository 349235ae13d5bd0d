/* C ABI of the warm start's field operations.
 *
 * The warm start (casclb_unet.h) builds an estimate of a steady periodic
 * flow + scalar state from steady solves of the same problem on the L/2 and
 * L/4 lattices and a network's correction, and initialises the L x L lattice
 * from it.  These calls are the steps between the solver and the network,
 * all on device memory: restriction of the force and source to a coarser
 * lattice, prolongation of coarse steady fields, the extrapolated combination
 * of two levels, removal of the modes a start from rest never has, packing of
 * the network's input, unpacking of its output, and the initial moments.  The
 * paper prescribes none of this; the solver it prepares is the cascaded
 * scheme with the split force and source steps (Sec. 3-5).
 *
 * Layout: a field array holds `planes` consecutive L x L planes of float64,
 * node x + L y within a plane (x fastest), the node order of casclb.h, so the
 * moments of a stacked 2D context (u as [2][nz][L][L]) are valid inputs.
 * Network tensors are float32 NHWC, [batch][L][L][channels].
 *
 * Conventions: every pointer except the lb_warm_channel array (host) is
 * device memory owned by the caller, on the current HIP device; work is
 * enqueued on `stream` (a hipStream_t of that device, NULL = the null stream)
 * and nothing synchronises.  Returns 0, LB_EINVAL (bad sizes or NULL
 * pointers; nothing enqueued) or LB_EHIP.  No call allocates memory.
 */
#ifndef CASCLB_WARM_H
#define CASCLB_WARM_H

#include <stddef.h>
#include <stdint.h>

#include "casclb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LB_WARM_MAX_L 2048
#define LB_WARM_MAX_CHANNELS 16
#define LB_WARM_MAX_K2 8

/* dst plane p ((L/2) x (L/2)) = scale * the means of the 2 x 2 blocks of src
 * plane p: coarse node X sits at fine position 2X + 1/2.  L even, 2..2048.
 * Under diffusive scaling (dx x2, dt x4) a force restricts with scale 8 and a
 * source with scale 4. */
int lb_warm_restrict(const double* src, int32_t planes, int32_t L, double scale, double* dst, void* stream);

/* dst plane p ((2 Lc) x (2 Lc)) = scale * the periodic Catmull-Rom
 * interpolation of src plane p (Lc x Lc, 2 <= Lc <= 1024) at the fine nodes: fine
 * node 2X + 1 lies 1/4 of a coarse spacing past coarse node X, fine node 2X
 * lies 3/4 past X - 1; separable, 4 x 4 taps.  Preserves the plane mean. */
int lb_warm_prolong(const double* src, int32_t planes, int32_t Lc, double scale, double* dst, void* stream);

/* out[i] = a x[i] + b y[i], i < n (out may alias x or y). */
int lb_warm_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, void* stream);

/* In place, per L x L plane: removes the mean, the two Nyquist lines (the
 * Fourier modes with k_x = pi or k_y = pi) and, with k2max > 0, the low modes
 * 0 < kx^2 + ky^2 <= k2max (integer wave numbers of the period L; k2max <=
 * LB_WARM_MAX_K2, and those modes must lie below L/2).  The lattice iteration
 * leaves the Nyquist modes unchanged, a start from rest under smooth forcing
 * has none, and any in an estimate would stay in the converged state; the low
 * modes are removed from a correction that should not touch the largest
 * scales.  L even, 2..2048.  One workgroup per plane reads it twice; sums in a
 * fixed order (deterministic). */
int lb_warm_project(double* data, int32_t planes, int32_t L, int32_t k2max, void* stream);

/* One channel of a pack / unpack: `src` is a [batch][n] slice (image b at
 * src + b n); NULL in lb_warm_pack means a constant channel.  `dst` is used
 * by lb_warm_unpack only. */
typedef struct lb_warm_channel {
    const double* src;
    double* dst;
    double scale;
    double offset;
} lb_warm_channel;

/* out[(b n + i) C + c] = (float)(scale_c src_c[b n + i] + offset_c), the NHWC
 * network input; C = nchannels (1..16), channels a host array. */
int lb_warm_pack(const lb_warm_channel* channels, int32_t nchannels, int32_t batch, int64_t n, float* out,
                 void* stream);

/* dst_c[b n + i] = src_c[b n + i] + scale_c y[(b n + i) C + c] (offset ignored;
 * a NULL src reads as zero): the estimate from a guess and the network's
 * correction y, or the correction alone. */
int lb_warm_unpack(const float* y, const lb_warm_channel* channels, int32_t nchannels, int32_t batch, int64_t n,
                   void* stream);

/* The moments that lb_init_equilibrium_device takes for an estimate of the
 * half-forced state (density deviation drho, half-forced u [2][batch][n],
 * half-sourced phi) of `batch` problems with force F [2][batch][n] and source
 * S [batch][n] (S and phi may be NULL for a flow-only lattice):
 *   rho = rho0 + drho;
 *   if zero_momentum: u -= sum(rho u) / sum(rho) per problem (a start from rest
 *     keeps the total half-forced momentum at zero under zero-mean forcing);
 *   u_out = u - F / (2 rho), phi_out = phi - S / 2 (eq. 25 and 43 read
 *     backwards: the initial state's own half-forced moments are the estimate).
 * One workgroup per problem; sums in a fixed order (deterministic). */
int lb_warm_initial_state(const double* drho, const double* u, const double* phi, const double* F, const double* S,
                          int32_t batch, int64_t n, double rho0, int32_t zero_momentum, double* rho_out,
                          double* u_out, double* phi_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CASCLB_WARM_H */
