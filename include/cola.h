/*
 * libcola -- COLA particle-mesh N-body step and 2LPT initial conditions on AMD MI355X (gfx950).
 *
 * Method: Izard, Crocce & Fosalba, "ICE-COLA: Towards fast and accurate synthetic galaxy
 * catalogues optimizing a quasi N-body method" (arXiv:1509.04685).
 *
 *   Sec. 1, Eq. 1-2  the displacement splits into the 2LPT trajectory and a residual; only the
 *                    residual's time derivative is discretised, the 2LPT acceleration is analytic.
 *   Sec. 2.2         2LPT Gaussian initial conditions; a particle-mesh force on a mesh PM_grid
 *                    times finer per side than the particle grid; four FFTs per force (one forward
 *                    of the density, three inverse, one per force component).
 *   Sec. 4.2, Eq. 3  n time nodes spaced uniformly in f(a), Delta f = (f(1) - f(a_i)) / (n - 1);
 *                    the optimum is f(a) = a (linear), 40 nodes, z_i = 19, PM_grid = 3 (Sec. 4.5).
 *   Sec. 2.5         matter power spectrum: CIC onto a grid, FFT, band average of |delta_k|^2,
 *                    CIC window divided out.
 *
 * Conventions (every entry point):
 *   - Units: lengths in h^-1 Mpc, wavenumbers in h/Mpc, time through the scale factor a, H0 = 1;
 *     momenta p = a^2 dx/dt in units of H0 h^-1 Mpc.
 *   - Arrays are C order [x][y][z], z fastest.  Particle arrays are structure-of-arrays in
 *     Lagrangian index order, idx = (i * N_p + j) * N_p + l.
 *   - A batch holds n_real realizations of one problem; every particle array then holds
 *     n_real * N_p^3 floats, realization r at offset r * N_p^3.
 *   - Every pointer in cola_particles, the P(k) outputs and the workspace is DEVICE memory
 *     owned by the caller; the library never allocates, frees or keeps it.  Problem and
 *     cosmology structs and seed arrays are HOST memory, read during the call only.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL = default stream).
 *     Arguments are validated on the host before any launch, so error returns never leave
 *     work queued.  Returns COLA_OK (0) or a negative cola_status; cola_status_string gives
 *     the message.  After COLA_ERR_HIP the stream's contents are undefined.
 *   - The workspace is carved by the library; cola_workspace_bytes gives its size.  Between
 *     calls it caches the force mesh of the current node (see cola_particles.force_node).
 *   - Calls that overlap on one workspace race; use one workspace per stream.
 */
#ifndef COLA_H
#define COLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COLA_OK = 0,
    COLA_ERR_INVALID_ARG = -1,        /* NULL pointer, out-of-range parameter             */
    COLA_ERR_UNSUPPORTED_SIZE = -2,   /* a mesh size that is odd or has a prime factor > 3 */
    COLA_ERR_WORKSPACE_TOO_SMALL = -3,
    COLA_ERR_HIP = -4,                /* a HIP runtime call failed                         */
    COLA_ERR_STATE = -5,              /* particle state does not fit the call (node range)  */
    COLA_ERR_NONFINITE = -6           /* a floating-point argument is NaN or infinite (box,
                                         z_init, a_final, sampling power, cosmology, a_out,
                                         network scales and knots, masses, mass edges)       */
} cola_status;

/* Flat LCDM, Omega_L = 1 - Omega_m, no radiation (Sec. 2.1: Omega_m 0.25, Omega_b 0.044,
 * h 0.7, n_s 0.95, sigma_8 0.8).  The linear spectrum is the BBKS fit with the Sugiyama
 * shape parameter, normalised to sigma_8 in 8 h^-1 Mpc top-hat spheres at a = 1 (the paper
 * used CAMB, Sec. 2.1). */
typedef struct {
    double omega_m, omega_b, h, n_s, sigma_8;
} cola_cosmology;

/* One simulation as Table 1 parameterises it. */
typedef struct {
    double  box;        /* L, side of the periodic box [h^-1 Mpc]                             */
    int32_t n_part;     /* N_p particles per side (N_p^3 particles), >= 2                     */
    int32_t pm_factor;  /* PM_grid: the force mesh has N_g = pm_factor * N_p cells per side   */
    double  z_init;     /* a_0 = 1 / (1 + z_init)                                             */
    double  a_final;    /* last node, normally 1                                              */
    int32_t n_steps;    /* number of time nodes n of Eq. 3, both ends included (n >= 2);
                           one force evaluation per node, n - 1 drifts                        */
    int32_t sampling;   /* time sampling f(a) of Eq. 3, nodes equally spaced in f (Sec. 4.2):
                           0 = linear, f = a (the paper's choice); 1 = logarithmic, f = ln a;
                           2 = power, f = a^sampling_power                                    */
    int32_t n_real;     /* realizations in the batch, >= 1                                    */
    int32_t frame;      /* 0 = COLA: integrate the residual from the 2LPT path (Eq. 1-2);
                           1 = PM only: the plain kick-drift-kick leapfrog with the LPT frame
                           switched off (the comparison of Appendix B)                        */
    double  sampling_power;  /* p of f = a^p for sampling = 2 (finite, > 0); ignored otherwise */
} cola_problem;

/* Particle state of a batch.  Each pointer: n_real * N_p^3 floats on the device.
 *   x     displacement from the Lagrangian position q (not the absolute position), where
 *         q = idx_d * L / N_p + H / 2 per axis, H = L / N_g: the lattice sits at force-mesh
 *         cell centres (on a node the CIC weights have a kink).
 *   p     residual momentum p_res = p - a^2 (dD1/dt Psi1 + dD2/dt Psi2) (Eq. 1-2 frame);
 *         with frame = 1 (PM only) the full momentum p = a^2 dx/dt.
 *   psi1  first-order Lagrangian displacement at D1 = 1; psi2 second order (D2 < 0 convention).
 * node        index of the time node the state sits at (0 after cola_ic_2lpt).
 * force_node  node whose force mesh the workspace `force_ws` holds, or -1.  Set by the
 *             library; set it to -1 yourself after changing x, or the parameters or scales of
 *             the network of cola_step_lc.
 * force_ws    workspace that holds that force mesh.
 * The library also keeps, per workspace, which state (identified by its x[0] array), node and
 * network (its params array, or none) the force meshes belong to; every call that writes a
 * workspace drops that record.  A cached force is used only when both agree, so sharing a
 * workspace between states, or between cola_step and cola_step_lc, costs a force evaluation,
 * never a wrong force. */
typedef struct {
    float* x[3];
    float* p[3];
    float* psi1[3];
    float* psi2[3];
    int32_t node;
    int32_t force_node;
    const void* force_ws;
} cola_particles;

/* Bytes of device workspace needed by every call on `prob` with a P(k) mesh of n_pk per side
 * (n_pk = 0: no P(k) buffers).  Returns 0 for invalid arguments. */
size_t cola_workspace_bytes(const cola_problem* prob, int32_t n_pk);

/* 2LPT Gaussian initial conditions (Sec. 2.2; Crocce, Pueblas & Scoccimarro 2006).
 * White noise per Lagrangian cell from Philox4x64-10 keyed by the realization's seed
 * (Sec. 2.3: one seed, one field) with the cell index as counter; delta_k = FFT[w] *
 * sqrt(P(k) N_p^3 / L^3), k = 0 removed; Psi1 = IFFT[i k delta / k^2]; Psi2 =
 * IFFT[-i k S_k / k^2] with S = sum_{i>j}(phi_ii phi_jj - phi_ij^2), phi_ij = IFFT[k_i k_j delta/k^2];
 * a factor odd in k_d is zeroed on the Nyquist plane of axis d.  On return x = D1(a_0) Psi1 +
 * D2(a_0) Psi2, p = 0 (frame 0) or the 2LPT momentum a^2 (dD1/dt Psi1 + dD2/dt Psi2) at a_0
 * (frame 1), node = 0, force_node = -1.
 * seeds: host array of n_real seeds.  ws: cola_workspace_bytes(prob, 0) bytes at least. */
int cola_ic_2lpt(const cola_problem* prob, const cola_cosmology* cosmo, const uint64_t* seeds,
                 cola_particles* out, void* ws, size_t ws_bytes, void* stream);

/* Particle-mesh acceleration at the current positions (Sec. 2.2): CIC onto the N_g^3 mesh,
 * delta = rho / rho_bar - 1, forward FFT, g_k = i k delta_k / k^2 (k = 0 and each component's
 * own Nyquist plane set to 0), three inverse FFTs, CIC interpolation.  acc[d]: device arrays of
 * n_real * N_p^3 floats receiving g_d (the physical acceleration is (3/2) Omega_m g / a).
 * Leaves the force mesh in `ws` but does not change `in`. */
int cola_pm_force(const cola_problem* prob, const cola_particles* in, float* acc[3],
                  void* ws, size_t ws_bytes, void* stream);

/* COLA steps from node j_begin (= io->node) to node j_end (Eq. 1-2, Eq. 3 nodes, kick-drift-kick
 * in the 2LPT frame):
 *   kick  p += (3/2) Omega_m K [g - D1 Psi1 - (D2 - D1^2) Psi2],  K = int da / (a^2 E)
 *   drift x += p Dr + dD1 Psi1 + dD2 Psi2,                         Dr = int da / (a^3 E)
 * Half-nodes are arithmetic mid-points in a.  On return p is synchronised at node j_end,
 * io->node = j_end and the force of node j_end sits in ws (io->force_node = j_end), so the next
 * call does not evaluate it again: a run costs exactly n force evaluations. */
int cola_step(const cola_problem* prob, const cola_cosmology* cosmo, int32_t j_begin,
              int32_t j_end, cola_particles* io, void* ws, size_t ws_bytes, void* stream);

/* Matter power spectrum at a_out (Sec. 2.5).  Needs a_j <= a_out < a_{j+1} for j = io->node
 * (or a_out = a_j); between nodes the positions are drifted on a copy with the half-step
 * momentum (the main run is unchanged).  CIC onto n_pk^3 cells, FFT, |delta_k|^2 / W^2 with
 * W = prod_d sinc^2(pi m_d / n_pk); bin b >= 1 holds b^2 <= |m|^2 < (b+1)^2 (integer test,
 * k = 0 excluded); P_b = (L^3 / n_pk^6) sum w |delta|^2 / W^2 / sum w, w the full-k-space
 * multiplicity of each half-spectrum mode; sums in float64.  No shot-noise subtraction; the aliasing
 * correction is cola_power_spectrum_jing.  Outputs (device, n_real * n_bins each, bin 0 empty): k_mean [h/Mpc], pk
 * [(h^-1 Mpc)^3], n_modes.  n_pk: even, factors 2 and 3 only.  ws: cola_workspace_bytes(prob,
 * n_pk) bytes at least.  Between nodes it uses the force of node j that the workspace holds for
 * this state (from cola_step or cola_step_lc); with none cached it evaluates and caches the plain
 * mesh force of node j. */
int cola_power_spectrum(const cola_problem* prob, const cola_cosmology* cosmo,
                        cola_particles* in, double a_out, int32_t n_pk, int32_t n_bins,
                        double* k_mean, double* pk, double* n_modes,
                        void* ws, size_t ws_bytes, void* stream);

/* cola_power_spectrum with the aliasing correction of Jing (2005) that Sec. 2.5 applies.  For a
 * spectrum that is locally a power law P ~ k^n_eff, a mode's expected |delta_m|^2 is C(m) P(|m|),
 *   C(m) = sum_{|j_d| <= 2} W^2(u) (|u| / |m|)^n_eff,  u = |m| + j n_pk,  W(u) = prod_d sinc^2(pi u_d / n_pk)
 * (images about the absolute mode integers).  Starting from cola_power_spectrum's estimate, each of
 * `iterations` passes (1..16; 4 converge on noisy spectra) takes n_eff per bin as the
 * mode-weighted least-squares slope of ln P on ln k over the bins within a factor 1.35 in k
 * (clamped to [-4, 4]; 0 where that window holds one bin) and rebins |delta_m|^2 / C(m).  Shot
 * noise is corrected with the signal (a flat spectrum has n_eff = 0).  C is evaluated in float32
 * once per class of sorted absolute mode integers.  Outputs, workspace and state rules are those of
 * cola_power_spectrum (k_mean and n_modes are identical to it). */
int cola_power_spectrum_jing(const cola_problem* prob, const cola_cosmology* cosmo,
                             cola_particles* in, double a_out, int32_t n_pk, int32_t n_bins,
                             int32_t iterations, double* k_mean, double* pk, double* n_modes,
                             void* ws, size_t ws_bytes, void* stream);

/* Redshift-space multipoles (Sec. 6: Eq. 5 mapping, Eq. 6 multipoles).  Plane-parallel: the line
 * of sight is axis `los` (0, 1, 2).  With redshift_space != 0 each particle is moved along the line
 * of sight by v_los / (a H(a)) (Eq. 5), v = a dx/dt its peculiar velocity at the state's node (the
 * momentum is synced only at nodes, so a_out must equal the scale factor of in->node; otherwise
 * COLA_ERR_STATE); with redshift_space = 0 the real-space positions are used.  The density on the
 * n_pk^3 mesh, its transform, the CIC window and the shells are those of cola_power_spectrum, and
 * each mode is weighted by the Legendre polynomial of mu = k_los / |k|:
 *   P_ell(k_b) = (2 ell + 1) sum_modes w |delta_k|^2 / W^2 L_ell(mu) / sum_modes w,  ell = 0, 2, 4
 * (P_0 is cola_power_spectrum's P(k)).  Outputs: device [n_real][n_bins] float64 each, overwritten.
 * No Jing (2005) aliasing correction and no shot-noise subtraction (the paper states neither
 * method for matter).  ws: cola_workspace_bytes(prob, n_pk).  The state is not changed. */
int cola_power_multipoles(const cola_problem* prob, const cola_cosmology* cosmo, cola_particles* in,
                          double a_out, int32_t los, int32_t redshift_space, int32_t n_pk, int32_t n_bins,
                          double* k_mean, double* p0, double* p2, double* p4, double* n_modes, void* ws,
                          size_t ws_bytes, void* stream);

/* ---- learned coarse-mesh force correction ---------------------------------------------- */

/* Sec. 4.4 shows that a force mesh coarser than PM_grid = 3 biases haloes through the force
 * resolution, and Sec. 7 keeps PM_grid >= 3 for that reason.  This library adds (its own design,
 * not the paper's) a small periodic 3D convolutional network on the PM_grid = 1 mesh that maps the
 * mesh fields to a force correction dF, added to the mesh force before it is interpolated:
 *   X0 = (delta, g_x, g_y, g_z) * in_scale
 *   A1 = silu(conv3(W1, X0) + b1),  A2 = silu(conv3(W2, A1) + b2),  dF = (W3 A2 + b3) * out_scale
 * conv3 is the periodic 3x3x3 cross-correlation Z[o][v] = sum_i sum_d W[o][i][tap(d)] X[i][v + d],
 * d in {-1,0,1}^3, tap(d) = (dx+1) 9 + (dy+1) 3 + (dz+1); silu(z) = z / (1 + exp(-z)); W3 is 1x1x1.
 * The convolutions run on BF16 matrix cores with FP32 accumulation; activations are stored in
 * BF16, parameters and the optimizer state in FP32.  Mesh sizes: multiples of 16. */
typedef struct {
    int32_t channels;    /* C: 16 or 32                                                       */
    float in_scale[4];   /* input normalisation of delta, g_x, g_y, g_z                        */
    float out_scale;     /* output scale (at a = 1)                                            */
    float out_scale_slope; /* in the step the scale at a node is out_scale (1 + slope (1 - a)); the
                            other entry points use out_scale                                   */
    float out_band;      /* band-pass weight beta: the output becomes dF + beta (K dF - K K dF),
                            K the periodic [1, 2, 1] / 4 smoothing along each mesh axis (a mode
                            is multiplied by 1 + beta c (1 - c), c = prod_d cos^2(pi m_d / n));
                            0 = off.  Applied in every entry point, backward included          */
    int32_t n_knots;     /* 0, or 2..8: in the step the scale is further multiplied by the
                            piecewise-linear interpolation of (knot_a[i], knot_v[i]) at the
                            node's a (knot_a increasing; constant beyond the end knots).  Lets
                            a calibration set the correction's strength per epoch              */
    float knot_a[8];
    float knot_v[8];
    int32_t n_gknots;    /* 0, or 2..10: the corrected force of cola_step_lc and cola_pm_force_lc
                            computes its mesh force with the Green's function times a radial
                            transfer T(u, a), u = |k| / k_N (k_N = pi n / L, the mesh's Nyquist
                            wavenumber): in u the cubic Hermite interpolant of (gknot_u[j],
                            gknot_t[i][j]) with slope 0 at the first knot, centred-difference
                            slopes inside and the one-sided slope at the last knot (gknot_u
                            increasing; constant beyond the end knots); in a piecewise linear
                            over the schedule's knot_a (row i; row 0 alone when n_knots = 0).
                            The network's dF is added unfiltered.  0: T = 1                      */
    float gknot_u[10];
    float gknot_t[8][10];
    float* params;       /* device, cola_lc_param_count(C) floats, flat in the order
                            w1 (C,4,27) b1 (C) w2 (C,C,27) b2 (C) w3 (3,C) b3 (3), C order       */
    float* grads;        /* device, same size: cola_lc_backward adds into it, cola_lc_adam
                            clears it; NULL for inference                                      */
    float* adam_m;       /* device, same size: Adam moments; NULL for inference                */
    float* adam_v;
    void* packed;        /* device, cola_lc_packed_bytes(C): BF16 copies of the conv weights,
                            written by cola_lc_pack (and by cola_lc_adam after each update)    */
} cola_lc_net;

int64_t cola_lc_param_count(int32_t channels);  /* 0 for an unsupported C */
size_t cola_lc_packed_bytes(int32_t channels);
/* Device workspace of the network on an n_mesh^3 mesh for n_real realizations; training keeps the
 * activations the backward pass needs. */
size_t cola_lc_workspace_bytes(int32_t n_mesh, int32_t channels, int32_t n_real, int32_t training);

/* Rewrites net->packed from net->params.  Call after writing params. */
int cola_lc_pack(const cola_lc_net* net, void* stream);

/* dF of the network on one n_mesh^3 mesh.  delta, g[3]: device, dense n_mesh^3 floats each (the
 * fields of cola_pm_fields); df[3]: device, dense n_mesh^3, overwritten (accumulate = 0) or added
 * into (1).  training = 1 keeps the activations in ws for one cola_lc_backward; ws holds
 * cola_lc_workspace_bytes(n_mesh, C, 1, training) bytes. */
int cola_lc_forward(const cola_lc_net* net, int32_t n_mesh, const float* delta, const float* g[3],
                    float* df[3], int32_t accumulate, int32_t training, void* ws, size_t ws_bytes,
                    void* stream);

/* Adds to net->grads the gradient of a loss L with respect to the parameters, given
 * d_df = dL/d(dF) (device, dense [3][n_mesh^3]) for the last training forward pass in ws (same
 * net, same n_mesh, parameters unchanged since). */
int cola_lc_backward(const cola_lc_net* net, int32_t n_mesh, const float* d_df, void* ws,
                     size_t ws_bytes, void* stream);

/* Training loss on particles at absolute positions pos[3] (device, n floats each):
 *   L = sum_p |g1_p + G[dF]_p - g3_p|^2 / sum_p |g3_p - g1_p|^2
 * with G the CIC interpolation of dF (device, dense n_mesh^3 per component) in a box of side box,
 * g1 the coarse-mesh and g3 the target acceleration at the particles (device, n floats each).
 * stats (device, 2 doubles): L and the denominator, overwritten.  d_df (device, dense
 * [3][n_mesh^3]): dL/d(dF), overwritten. */
int cola_lc_loss(int32_t n_mesh, double box, const float* pos[3], int64_t n, const float* df[3],
                 const float* g1[3], const float* g3[3], double* stats, float* d_df, void* stream);

/* One Adam step (Kingma & Ba 2015) at step number t >= 1 on net->params with net->grads, then
 * clears net->grads and repacks the BF16 weights. */
int cola_lc_adam(const cola_lc_net* net, int32_t t, float lr, float beta1, float beta2, float eps,
                 void* stream);

/* ---- ensembles ------------------------------------------------------------------------- */

/* One shape class of an ensemble: n_real = prob.n_real realizations of one problem. */
typedef struct {
    cola_problem prob;
    const uint64_t* seeds;   /* host, n_real seeds                                          */
    cola_particles* parts;   /* device arrays of n_real * N_p^3 floats                       */
    void* ws;                /* device workspace of cola_workspace_bytes(&prob, n_pk) bytes  */
    size_t ws_bytes;
    int32_t n_out;           /* P(k) outputs at the scale factors a_out (host, ascending)    */
    const double* a_out;
    int32_t n_pk, n_bins;
    double* k_mean;          /* device, [n_out][n_real][n_bins] each                         */
    double* pk;
    double* n_modes;
    const cola_lc_net* net;  /* NULL: plain steps; else the class runs cola_step_lc with this
                                network (N_g a multiple of 16)                               */
    void* lc_ws;             /* device, cola_lc_workspace_bytes(N_g, C, n_real, 0) bytes when
                                net is set                                                   */
    size_t lc_ws_bytes;
} cola_ensemble_class;

/* Mock ensembles (Sec. 2.3: realizations that differ only in their seed; the paper's purpose is
 * ensembles of mocks, Sec. 1).  For every class: cola_ic_2lpt, then cola_step (cola_step_lc with
 * the class's network) up to each output node with cola_power_spectrum at each a_out, then to the
 * last node -- all realizations of a class advance together in batched launches.  A captured
 * graph reads the network's parameters from device memory at every replay, but keeps the scales
 * and schedule it was captured with.
 *   mode 0: launch eagerly on `stream`, classes one after the other.
 *   mode 1: capture the whole ensemble into one hipGraph, each class on its own stream forked
 *           from `stream` so the classes overlap, instantiate it, launch it on `stream` and keep
 *           the executable graph; a later call with identical arguments (same pointers, sizes,
 *           seeds, outputs, cosmology) relaunches it without host work.
 * On return every class's particles are at their last node.  cola_ensemble_release frees the
 * cached graphs and streams. */
int cola_ensemble_run(int32_t n_classes, cola_ensemble_class* classes, const cola_cosmology* cosmo,
                      int32_t mode, void* stream);
int cola_ensemble_release(void);

/* FFT autotuner.  Times every admissible kernel shape (values per thread, lines or columns per
 * block) of each FFT pass at the problem's force-mesh, lattice and P(k) sizes, on `stream`, and
 * keeps the fastest for every later call in this process (until then a fixed heuristic is
 * used).  Uses ws as scratch: its contents, including a cached force mesh, are destroyed --
 * call it before cola_ic_2lpt or set force_node = -1 afterwards.  Synchronises the stream.
 * report (host, may be NULL): one line per pass with the chosen shape and its time. */
int cola_autotune(const cola_problem* prob, int32_t n_pk, void* ws, size_t ws_bytes, void* stream,
                  char* report, size_t report_len);

/* Pins the kernel shape of one FFT pass kind at mesh side n for the rest of the process, as the
 * autotuner would: kind one of "z_r2c", "z_c2r", "rows_y", "cols_x", "x_green", "y_split",
 * "x_mult", "z_c2r3" (the step's z pass writing the three force components interleaved);
 * values_per_thread and width (lines per block for the z passes and the y rows, a power
 * of two dividing n for the z passes; columns per tile for the x passes) must form an admissible
 * shape; use_static: 0 the plan built at run time, 1 the compile-time plan of that shape, 2 (x-column
 * kinds) the compile-time plan whose LDS exchanges move the real and then the imaginary parts
 * through half the LDS (COLA_ERR_INVALID_ARG if the library has no such plan).  Host only: nothing
 * is launched. */
int cola_fft_set_shape(int32_t n, const char* kind, int32_t values_per_thread, int32_t width, int32_t use_static);

/* cola_step with the network's correction: at each force evaluation the density contrast and the
 * mesh force of every realization feed the network and dF is added to the force mesh before the
 * kick.  lc_ws: cola_lc_workspace_bytes(N_g, C, n_real, 0) bytes.  N_g a multiple of 16.  The
 * cached force is then the corrected one (recorded with net->params, so cola_step on the same
 * state evaluates its own plain force).  j_end = j_begin evaluates and caches the corrected force
 * of the current node without stepping.  cola_power_spectrum between nodes drifts with the cached
 * force of the state's node whatever network made it; with none cached it evaluates the plain
 * force, so a corrected run keeps its corrected force cached (as every cola_step_lc leaves it). */
int cola_step_lc(const cola_problem* prob, const cola_cosmology* cosmo, int32_t j_begin,
                 int32_t j_end, cola_particles* io, const cola_lc_net* net, void* lc_ws,
                 size_t lc_ws_bytes, void* ws, size_t ws_bytes, void* stream);

/* The corrected acceleration of cola_step_lc at the current positions, without stepping: the
 * mesh force of cola_pm_force plus the network's dF (output scale evaluated as in the step at
 * scale factor a, a > 0), interpolated to the particles.  acc[d]: device, n_real * N_p^3 floats.
 * lc_ws, ws: as for cola_step_lc.  The state is not changed; ws's force cache is dropped. */
int cola_pm_force_lc(const cola_problem* prob, const cola_particles* in, const cola_lc_net* net, double a,
                     void* lc_ws, size_t lc_ws_bytes, float* acc[3], void* ws, size_t ws_bytes, void* stream);

/* cola_pm_force for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same passes and the same result, with
 * the workspace taken from a fixed 96 MiB device array that the library holds on each GPU until
 * the process ends, instead of a caller buffer.  The caller still passes the state and acc.
 * Problems whose cola_workspace_bytes(prob, 0) exceeds 96 MiB (for example 128^3 particles on a
 * 128^3 mesh, 128 MiB; 64^3 particles on a 128^3 mesh need 65 MiB) return COLA_ERR_WORKSPACE_TOO_SMALL before
 * any launch.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race, and a state's cached force is never kept in it.  No hipMalloc, hipFree or other
 * allocating call is made. */
int cola_pm_force_noalloc(const cola_problem* prob, const cola_particles* in, float* acc[3], void* stream);

/* Mesh fields of arbitrary particles: CIC of the absolute positions pos[3] (device, n floats
 * each, any real, wrapped into the box) onto n_mesh^3 cells, delta = rho / rho_bar - 1, the force
 * g_k = i k delta_k / k^2 as in cola_pm_force, and its CIC interpolation to the particles.  Each
 * output may be NULL: delta (dense n_mesh^3), g[3] (dense n_mesh^3 each), acc[3] (n each), all
 * device.  ws: cola_pm_fields_workspace_bytes(n_mesh) bytes. */
size_t cola_pm_fields_workspace_bytes(int32_t n_mesh);
int cola_pm_fields(int32_t n_mesh, double box, const float* pos[3], int64_t n, float* delta, float* g[3],
                   float* acc[3], void* ws, size_t ws_bytes, void* stream);

/* Force meshes of a density-contrast mesh (Sec. 2.2: one forward FFT, the k-space force, three
 * inverse FFTs), the transform passes of the step without its deposit and gather:
 * g_d = IFFT[i k_d delta_k / k^2] (k = 0 and component d's own Nyquist plane set to 0).
 * delta: device, dense n_mesh^3 floats; g[d]: device, dense n_mesh^3 floats each, overwritten.
 * n_mesh: even, factors 2 and 3 only, <= 1536.  ws: cola_pm_fields_workspace_bytes(n_mesh). */
int cola_mesh_force(int32_t n_mesh, double box, const float* delta, float* g[3], void* ws, size_t ws_bytes,
                    void* stream);

/* Absolute positions q + x of a batch, wrapped into [0, box): pos[d] device arrays of
 * n_real * N_p^3 floats. */
int cola_positions(const cola_problem* prob, const cola_particles* in, float* pos[3], void* stream);

/* ---- friends-of-friends haloes (Sec. 2.1, Sec. 2.5) ---------------------------------------
 *
 * Haloes are friends-of-friends groups (Davis et al. 1985) at a linking length b, 0.2 of the mean
 * inter-particle separation in the paper (Sec. 2.1; b = 0.2 * box / N_p).  Two particles are
 * friends when their periodic distance is below b; groups are the connected components of that
 * graph.  The test is taken in float32, each operation rounded on its own:
 *   d = x_j - x_i, then d -= box if d > box/2, d += box if d < -box/2 (each axis);
 *   d2 = (dx*dx + dy*dy) + dz*dz;  friends iff d2 < float32(b) * float32(b).
 * Groups of at least n_min particles (more than 100 in Sec. 2.5: n_min = 101) are haloes with the
 * Warren et al. mass
 * M = m_p N (1 - N^-0.6) (Sec. 2.5). */

/* Workspace for cola_fof and cola_fof_catalogue with n particles in a box of side box at linking
 * length link (0 for invalid arguments).  About 24 n bytes plus 12 bytes per cell of a grid of at
 * most n cells. */
size_t cola_fof_workspace_bytes(int64_t n, double box, double link);

/* Groups of n particles.  pos[d]: device arrays of n floats (absolute positions, any real; cells
 * are taken modulo the box), 1 <= n < 2^31, 0 < link < box / 2.  group: device n int32, out:
 * group[i] = the smallest particle index in i's group (so group[i] <= i, and group[i] == i marks
 * a group's label).  group_size: device n int32, out: at a label r the number of members of its
 * group, 0 at every other index.  The result is deterministic.  The time grows with the square
 * of the particles per cell (cells of side >= link, about one particle per cell on average), so
 * inputs that pile most particles into one small region are slow.  Errors: COLA_ERR_INVALID_ARG,
 * COLA_ERR_WORKSPACE_TOO_SMALL, COLA_ERR_HIP. */
int cola_fof(const float* pos[3], int64_t n, double box, double link, int32_t* group, int32_t* group_size,
             void* ws, size_t ws_bytes, void* stream);

/* Halo catalogue of the groups of cola_fof with at least n_min members, ordered by label:
 * halo_root[h] (label), halo_n[h] (members), halo_mass[h] (Warren mass with particle mass
 * particle_mass), halo_com[d][h] (centre of mass: the label particle's position plus the mean of
 * the members' float32 minimum-image offsets from it, accumulated in float64, wrapped into
 * [0, box)).  All outputs are device arrays of max_halos entries; max_halos must be at least
 * n / n_min (the most haloes there can be).  n_halos: device int64, out: the number of haloes.
 * ws: as for cola_fof (its contents from cola_fof are not used). */
int cola_fof_catalogue(const float* pos[3], int64_t n, double box, const int32_t* group,
                       const int32_t* group_size, int32_t n_min, double particle_mass, int64_t max_halos,
                       int32_t* halo_root, int32_t* halo_n, double* halo_mass, double* halo_com[3],
                       int64_t* n_halos, void* ws, size_t ws_bytes, void* stream);

/* Binned halo mass function: counts[b] (device, n_bins uint64, overwritten) = the number of
 * groups with N >= n_min members whose Warren mass lies in [10^e_b, 10^e_{b+1}), e = the host
 * array log10_mass_edges of n_bins + 1 strictly increasing values, 1 <= n_bins <= 64.  The mass
 * increases with N, so the host turns each edge into the smallest N whose float64 Warren mass
 * reaches it and the device bins the integer sizes.  dn/dlog10 M = counts / (box^3 * width). */
int cola_fof_mass_histogram(const int32_t* group_size, int64_t n, int32_t n_min, double particle_mass,
                            const double* log10_mass_edges, int32_t n_bins, uint64_t* counts, void* stream);

/* Particle mass m_p = Omega_m rho_crit (box / n_part)^3 in h^-1 M_sun, rho_crit = 2.775e11
 * h^2 M_sun Mpc^-3 (0 for invalid arguments). */
double cola_particle_mass(const cola_cosmology* cosmo, double box, int32_t n_part);

/* ---- component entry points (the stages above, exposed for parity checks) ------------- */

/* CIC density contrast of arbitrary positions (Sec. 2.2, Sec. 2.5: cloud-in-cell assignment) by
 * the step's own deposit: records binned by mesh tile, counting sort, per-tile accumulation in
 * 32.32 fixed point, every cell written once (deterministic; no atomics to device memory).
 * pos[d]: device arrays of n floats (absolute positions, any real, wrapped periodically),
 * 1 <= n < 2^31; delta: device, dense n_mesh^3 floats, overwritten; rho_bar = n / n_mesh^3;
 * 2 <= n_mesh <= 1536.  ws: device, cola_cic_workspace_bytes(n, n_mesh) bytes (0 for invalid
 * arguments or a mesh whose tile keys would not fit 32 bits). */
int cola_cic_density(const float* pos[3], int64_t n, int32_t n_mesh, double box, float* delta,
                     void* ws, size_t ws_bytes, void* stream);
size_t cola_cic_workspace_bytes(int64_t n, int32_t n_mesh);

/* 3D real-to-complex FFT, unnormalised forward (sign -1): in n^3 floats, out n*n*(n/2+1)
 * complex (float2, re/im interleaved), numpy rfftn layout.  3D complex-to-real inverse
 * (unnormalised, sign +1): the reverse.  n even with factors 2 and 3 only. */
size_t cola_fft_workspace_bytes(int32_t n);
int cola_fft_r2c(int32_t n, const float* in, float* out, void* ws, size_t ws_bytes, void* stream);
int cola_fft_c2r(int32_t n, const float* in, float* out, void* ws, size_t ws_bytes, void* stream);

/* ---- host-only helpers (no device work; usable without a GPU) --------------------------- */

/* The float64 schedule the step uses: for each node j, 6 doubles
 *   a_j, D1(a_j), D2(a_j), K(a_j, a_{j+1/2}), K(a_{j+1/2}, a_{j+1}), Dr(a_j, a_{j+1})
 * (the last three are 0 on the last node).  out: host array of 6 * n_steps doubles. */
int cola_schedule_table(const cola_problem* prob, const cola_cosmology* cosmo, double* out);

/* Linear power spectrum at a = 1 [(h^-1 Mpc)^3] at wavenumber k [h/Mpc]; -1 on bad input. */
double cola_linear_power(const cola_cosmology* cosmo, double k);

/* ---- diagnostics ----------------------------------------------------------------------- */

/* Per-kernel timing.  While enabled, each library kernel launch is bracketed by a pair of HIP
 * events recorded on its stream; cola_profiler_read waits for the recorded events and returns,
 * per kernel kind, the summed milliseconds and the launch count (arrays of n_kinds, host
 * memory), then forgets them.  cola_profiler_enable resets the record; not thread-safe across
 * concurrent streams' readings. */
int cola_profiler_enable(int on);
int cola_profiler_num_kinds(void);
const char* cola_profiler_kind_name(int kind);
int cola_profiler_read(int32_t n_kinds, double* total_ms, int64_t* launches);
/* The same records grouped by (kind, tag), where the tag is a size label (the mesh side for FFT
 * passes, else 0): up to cap groups written to the host arrays kinds, tags, total_ms, launches.
 * Returns the number of groups (>= 0) or a negative status; forgets the records like
 * cola_profiler_read. */
int cola_profiler_read_groups(int32_t cap, int32_t* kinds, int64_t* tags, double* total_ms, int64_t* launches);

/* Plain device-to-device copy of `bytes` bytes with the library's streaming kernel (16-byte
 * vectors): the yardstick against which hardware byte counters are scaled. */
int cola_copy(const void* src, void* dst, size_t bytes, void* stream);

/* One BF16 matrix-core product D = A B (A 16x32, B 32x16 BF16 bit patterns, D 16x16 FP32, all
 * row-major device arrays) through the operand layout the network's convolutions assume. */
int cola_mfma_selftest(const uint16_t* a, const uint16_t* b, float* d, void* stream);

/* Message for a cola_status value (static storage). */
const char* cola_status_string(int status);

/* Detail of the last COLA_ERR_HIP on this thread: the failing call and the HIP error text. */
const char* cola_last_error(void);

/* Library version string (static storage). */
const char* cola_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COLA_H */
