/*
 * galkin: batched forward-model log-likelihood (and its gradient) of the
 * bulge + disc(s) + halo disc-galaxy model of Rigamonti et al. 2022
 * (arXiv 2205.06819), on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for many parameter vectors theta at once, the
 * paper's model maps (Sec. 2.1-2.4), their Gaussian-PSF average (Sec. 3.1,
 * PSF convolution equation) and the four-term Gaussian log-likelihood
 * (Sec. 2.5.1, likelihood equation) against uploaded data maps.  Data are
 * uploaded once per grid, as the paper's Appendix A prescribes; each call
 * then evaluates a whole batch in one stream-ordered launch sequence.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Return value: GK_OK (0) on success, a negative GK_E* code otherwise;
 *    nothing is enqueued when an argument is rejected.  last_error() gives a
 *    message for the calling thread.  Functions never abort and never print.
 *  - Parameter vectors (theta) are float64, row-major [B][stride], stride >= P
 *    (P = n_params(grid)), in the sampling coordinates listed below; gradients
 *    are with respect to these coordinates.  Rows outside the physical domain
 *    (R <= 0, M/L <= 0, |k| > 1, i not in (0, 90) deg, c <= 0, non-finite
 *    entries) are not errors: they give logL = -inf and a zero gradient row.
 *  - "device" pointers are HIP device memory of the grid's device; the caller
 *    owns them.  The library keeps no caller pointer after a call returns.
 *  - hot-path calls (loglike_batch, loglike_grad_batch, eval_maps,
 *    loglike_joint, hmc_leapfrog) are
 *    asynchronous on the given hipStream_t (NULL = default stream): they do
 *    not allocate, synchronise or read device memory on the host, so they
 *    may be captured in a HIP graph.  Calls that share one grid handle must
 *    not run concurrently (they share its workspace).
 *
 * Parameter layout (theta columns), components as configured in the grid:
 *    frame              x0 [px], y0 [px], PA [deg], i [deg]
 *    bulge              log10 Mb [Msun], Rb [kpc], (M/L)b [Msun/Lsun]
 *                       (Hernquist, Sec. 2.2, or Jaffe, Appendix B)
 *    disc j (1..n)      log10 Mdj [Msun], Rdj [kpc], (M/L)dj, kj
 *    halo               log10 Mh [Msun], then c (NFW) or Rh [kpc] (Hernquist)
 * The galaxy centre is the grid centre ((nx-1)/2, (ny-1)/2) plus (x0, y0)
 * (scaled and offset by the descriptor's frame fields when the centre
 * parameters are shared by several pixelisations); the position angle is
 * counter-clockwise from +x (x = column index).
 */
#ifndef GALKIN_H
#define GALKIN_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GK_OK = 0,
    GK_EINVAL = -1,   /* invalid argument (null pointer, size, descriptor)   */
    GK_ENOMEM = -2,   /* device or host allocation failed                    */
    GK_EHIP = -3,     /* a HIP runtime call or kernel launch failed          */
    GK_ESTATE = -4    /* call out of order (e.g. loglike before set_data)    */
};

enum { GK_BULGE_NONE = 0, GK_BULGE_HERNQUIST = 1, GK_BULGE_JAFFE = 2 /* Appendix B */ };
enum { GK_HALO_NONE = 0, GK_HALO_HERNQUIST = 1, GK_HALO_NFW = 2 };
enum { GK_PSF_MAPS = 0, GK_PSF_LUMINOSITY = 1 };

typedef struct gk_grid* gk_grid_t;   /* opaque; owns all device buffers */

/* Grid and model description.  Maps are [ny][nx], x = column (fastest). */
typedef struct {
    int    nx, ny;         /* pixels per row / column, 1..4096                  */
    double pixel_kpc;      /* kpc per pixel, > 0                                */
    int    supersample;    /* s: odd, 1..15; the model is sampled on a lattice  */
                           /* of spacing 1/s pixel (Appendix A sub-grid)        */
    double psf_sigma_px;   /* Gaussian PSF sigma in pixels, >= 0; the average   */
                           /* runs over lattice points within 3 sigma (Sec 3.1) */
    int    bulge;          /* GK_BULGE_*                                        */
    int    n_discs;        /* 0, 1 or 2 exponential discs (Sec. 2.3)            */
    int    halo;           /* GK_HALO_*                                         */
    double hubble_h;       /* NFW: M200 at 200 rho_crit(H0 = 100 h); e.g. 0.7   */
    int    psf_mode;       /* GK_PSF_MAPS: each model map averaged over the PSF */
                           /* (Sec. 3.1); GK_PSF_LUMINOSITY: the PSF averages   */
                           /* B, B v, B (sigma^2 + v^2) and the mass density,   */
                           /* and v, sigma, M/L follow from their ratios        */
    /* Observations of one galaxy on several pixelisations (one grid each,     */
    /* Sec. 3.2: the maps may come with different numbers of pixels) share the */
    /* centre parameters x0, y0 through a common frame:                        */
    double frame_px_kpc;   /* pixel size of the frame x0, y0 are measured in;  */
                           /* 0 (or this grid's pixel_kpc): its own pixels     */
    double frame_dx;       /* the frame's centre, in this grid's pixels, from  */
    double frame_dy;       /* this grid's centre (0, 0 when they coincide)     */
} gk_grid_desc;

/* Create a grid handle on the current HIP device: the pixel grid and its
 * model lattice (Sec. 2.1; Appendix A's sub-grid), the PSF stencil (Sec. 3.1)
 * and the component set (Sec. 2.2-2.3).  Uploads the stencil tables and
 * allocates every device buffer the hot-path calls need for batches of up to
 * max_batch vectors (>= 1), so those calls never allocate (Appendix A:
 * allocate once, transfer once).  The gradient's pixel-adjoint buffer is
 * capped at ~2 GiB (larger gradient batches run in chunks).  *out receives
 * the handle; GK_EINVAL for an invalid descriptor or a PSF wider than this
 * build supports (3 sigma s <= 25 lattice points, floor(2 pad / s) <= 10),
 * GK_ENOMEM / GK_EHIP when the device refuses. */
int create_grid(const gk_grid_desc* desc, int max_batch, gk_grid_t* out);

/* Release a grid handle and its device memory (synchronises the device);
 * cached many-grid plans that use it are dropped. */
int destroy_grid(gk_grid_t grid);

/* Number of model parameters P of the grid's component set (the layout at
 * the top of this file; 17 for bulge + two discs + halo, as in the paper's
 * Table 1), or GK_EINVAL for a NULL grid. */
int n_params(gk_grid_t grid);

/* Upload the observed maps (Sec. 2.5.1): value and err are float32
 * [4][ny][nx] for surface brightness [Lsun/pc^2], l.o.s. velocity [km/s],
 * l.o.s. dispersion [km/s] and M/L [Msun/Lsun]; err are 1-sigma errors.
 * A pixel is masked in a map when its err is <= 0 or not finite, or its
 * value is not finite.  on_device != 0 means both pointers are device
 * memory.  The data are copied (the caller keeps ownership); this call is
 * synchronous with respect to the given stream and may be repeated.  A map
 * with no valid pixel is not convolved by the log-likelihood calls (a grid
 * that carries only some maps pays only for those); when that set changes,
 * the grid's cached many-grid plans are dropped (which synchronises). */
int set_data(gk_grid_t grid, const float* value, const float* err, int on_device,
             void* hip_stream);

/* The Gaussian log-likelihood of Sec. 2.5.1 (likelihood equation) for each
 * parameter vector:
 *   logL[b] = sum over the four maps and their valid pixels of
 *   -1/2 [ (F_m(p) - d_m(p))^2 / e_m(p)^2 + ln(2 pi e_m(p)^2) ],
 * with F the model of Sec. 2.1-2.4 (surface brightness, light-weighted
 * velocity and dispersion, <L/M>) averaged over the PSF (Sec. 3.1; the model
 * M/L map is 1 / <L/M>, eq:ML_ratio), for b in [0, B).  theta: device float64
 * [B][stride]; logL: device float64 [B] (-inf for rows outside the physical
 * domain).  B may be 0 (nothing is enqueued); B <= max_batch, else GK_EINVAL;
 * GK_ESTATE before set_data.  One launch per call. */
int loglike_batch(gk_grid_t grid, const double* theta, int B, int stride, double* logL,
                  void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * log-likelihoods as loglike_batch, with the launch's scratch (per-vector band
 * tickets and FP64 band partials) taken from a fixed array of 16 MiB that
 * each device holds from library load until the process ends, instead of the
 * grid's workspace.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and clears the tickets with a kernel.  It needs
 * B x (4 + 8 nbands) bytes of scratch, nbands being the bands of the launch
 * shape for B (get_launch_shape); larger requests return GK_EINVAL.  All such
 * calls on one device share the array: calls that overlap in time on one
 * device (different streams or threads) race and must be serialised by the
 * caller.  The grid must live on the current device. */
int loglike_batch_noalloc(gk_grid_t grid, const double* theta, int B, int stride, double* logL,
                          void* hip_stream);

/* As loglike_batch, and also grad[b][k] = d logL[b] / d theta[b][k] for
 * k < P (columns P..stride-1 of grad are set to 0; zero rows outside the
 * domain).  grad: device float64 [B][stride].  Not a method of the paper
 * (which samples without gradients): the derivative of the same model
 * (Sec. 2.1-2.4, 3.1, 2.5.1), by a hand-written adjoint — the forward
 * launch also writes d logL / d F per pixel, a second launch applies the
 * transposed PSF stencil and the reverse point model — exact for the FP32
 * model up to FP32 rounding, accumulated in FP64.  Two launches per chunk of
 * at most ~2 GiB / (16 bytes x pixels) vectors.  The log-likelihoods equal
 * loglike_batch's bit for bit. */
int loglike_grad_batch(gk_grid_t grid, const double* theta, int B, int stride, double* logL,
                       double* grad, void* hip_stream);

/* The model maps themselves (Sec. 2.4 total brightness, velocity and
 * dispersion equations; eq:ML_ratio) averaged over the PSF (Sec. 3.1) at
 * every pixel, float32 device [B][4][ny][nx]: surface brightness [Lsun/pc^2],
 * l.o.s. velocity and dispersion [km/s] and M/L (= 1 / PSF-averaged <L/M>).
 * Requires no data.  Rows outside the physical domain give NaN maps. */
int eval_maps(gk_grid_t grid, const double* theta, int B, int stride, float* maps,
              void* hip_stream);

/* Hamiltonian Monte Carlo trajectory of n_steps leapfrog steps for every
 * row (the gradient-driven sampler pattern the adjoint enables; not a method
 * of the paper, which uses nested sampling, Sec. 2.5).  With H = -logL(theta)
 * + p^T M^-1 p / 2: half kick p += (eps/2) grad, then n_steps times a drift
 * theta += eps M^-1 p followed by a full kick (half kick after the last
 * drift).  theta, momentum: device float64 [B][stride], updated in place;
 * inv_mass: device float64 [P] (diagonal M^-1); logL, grad: device outputs
 * (log-likelihood and gradient at the final position).  Rows with a
 * non-finite log-likelihood are frozen.  Enqueues n_steps + 1 gradient
 * evaluations and updates on the stream; allocates nothing, so a call can be
 * captured once in a HIP graph and replayed. */
int hmc_leapfrog(gk_grid_t grid, double* theta, double* momentum, const double* inv_mass, double eps,
                 int n_steps, int B, int stride, double* logL, double* grad, void* hip_stream);

/* Joint log-likelihood of ONE galaxy observed on several pixelisations
 * (Sec. 3.2: the observables may be mapped with different numbers of pixels;
 * the Gaussian terms of Sec. 2.5.1 add over the grids).  grids: host array of
 * n_grids >= 1 distinct handles with data, on the current device, all with
 * the same component set (the same parameter vector; their descriptors' frame
 * fields place the shared centre).  A grid contributes the maps it carries:
 * give zero errors in set_data for the maps it does not.  theta: device
 * float64 [B][stride]; logL[b] = sum over grids of each grid's logL; grad
 * (may be NULL) likewise summed.  Grid 0's launch stores, the others add, in
 * grid order on the stream, so repeated calls give identical results.  Uses
 * the grids' workspaces; allocates nothing. */
int loglike_joint(const gk_grid_t* grids, int n_grids, const double* theta, int B, int stride,
                  double* logL, double* grad, void* hip_stream);

/* Log-likelihoods of many galaxies in ONE persistent launch (the batched
 * form of the paper's per-galaxy likelihood, Sec. 2.5.1, over a catalogue).
 * grids: host array of n_gal distinct handles (all with data, all on the
 * current device).  theta_offset: host int array [n_gal + 1], theta_offset[0]
 * = 0, non-decreasing; rows theta_offset[g] .. theta_offset[g+1]-1 of theta
 * (device float64 [rows][stride], stride >= every grid's P) belong to galaxy g
 * and number at most that grid's max_batch; logL: device float64 [rows].
 * Each workgroup evaluates one (galaxy, row, pixel band) item; items are
 * dispatched in decreasing cost order (the items of luminosity-weighted
 * grids, GK_PSF_LUMINOSITY, in a second launch of their own).  The first call with a given (grids, theta_offset,
 * launch shapes) builds and uploads that work plan (allocating and
 * synchronising); repeated calls with the same arguments only enqueue the
 * launch and may then be captured in a HIP graph.  A destroyed grid's plans
 * are dropped.  grad (device float64 [rows][stride]) may be NULL; if given, the
 * gradient is computed as well, by one forward + adjoint launch pair per
 * galaxy.  The grids' workspaces are used: no other call on these grids may
 * run concurrently. */
int loglike_multi(const gk_grid_t* grids, int n_gal, const double* theta, const int* theta_offset,
                  int stride, double* logL, double* grad, void* hip_stream);

/* Data preparation (run once per galaxy, before set_data).
 *
 * Colour-M/L relation (Sec. 2.5.1, eq:ML-color; errors as in Appendix C):
 *   ml[i]  = 10^(a + b (m_beta[i] - m_gamma[i]))
 *   err[i] = ml[i] ln(10) sqrt(b^2 (dm_beta[i]^2 + dm_gamma[i]^2) + sigma_a^2)
 * with sigma_a the relation's scatter in dex.  All arrays are float32 device
 * memory of n pixels (any layout, e.g. [ny][nx]); pixels with a non-finite
 * magnitude or error get ml = NaN and err = 0, which set_data treats as
 * masked.  Asynchronous on the stream. */
int ml_from_colour(const float* m_beta, const float* m_gamma, const float* dm_beta, const float* dm_gamma,
                   int n, double a, double b, double sigma_a, float* ml, float* err, void* hip_stream);

/* Surface-brightness error model (Sec. 3, data): a relative error plus a
 * constant systematic floor set by the faintest pixel, added in quadrature:
 *   err[i] = sqrt((rel B[i])^2 + (floor_frac min B)^2)
 * where min B is over pixels with finite B > 0; other pixels get err = 0
 * (masked).  float32 device arrays of n pixels; one workgroup;
 * asynchronous on the stream. */
int brightness_errors(const float* B, int n, double rel, double floor_frac, float* err, void* hip_stream);

/* Launch shape used for batches of size >= batch_min: a band of band_h x
 * band_w pixels per workgroup (band_h, band_w >= 1) and steps pixel rows per
 * model phase (1..4; 0 = chosen from the lattice factor).  The autotuner sets
 * these.  GK_EINVAL if the shape does not fit the kernel's limits (band_w <=
 * 128, at most 1024 bands, LDS).  Also used by loglike_multi (band_w capped at
 * 64 there). */
int set_launch_shape(gk_grid_t grid, int batch_min, int band_h, int band_w, int steps);

/* The launch shape calls with B parameter vectors use: band_h, band_w
 * (pixels, clipped to the grid) and steps (pixel rows per model phase, 0 =
 * automatic), written to host ints — the library default unless
 * set_launch_shape installed a rule for that batch size.  For autotuners,
 * which time this shape alongside their own candidates. */
int get_launch_shape(gk_grid_t grid, int B, int* band_h, int* band_w, int* steps);

/* Launch shape of the gradient's second pass (the adjoint kernel): one
 * workgroup per vector and band of band_h x band_w pixels (band_w <= 128, at
 * most 1024 bands), which evaluates the block of the supersampled lattice
 * that its band owns (the lattice points between its pixels' centres, the
 * outer bands also the margins) and reads the pixel adjoints of every pixel
 * reaching that block; `rows` lattice rows per phase (1..16; 0 = chosen
 * from the band width).  The shape changes only the FP32 summation order of
 * the gradient.  GK_EINVAL if the shape does not fit the kernel's limits
 * (80 KiB of LDS).  Not a hot-path call: it may allocate the per-band
 * gradient partials and then synchronises the device.  For autotuners. */
int set_adjoint_shape(gk_grid_t grid, int band_h, int band_w, int rows);

/* The adjoint's current launch shape (band_h, band_w, rows), written to host
 * ints; GK_EINVAL if the grid fits no adjoint shape of this build (then only
 * the forward calls work on it). */
int get_adjoint_shape(gk_grid_t grid, int* band_h, int* band_w, int* rows);

/* Message describing the last error returned on the calling thread. */
const char* last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GALKIN_H */
