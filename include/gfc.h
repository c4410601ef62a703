/*
 * gfc.h -- C ABI of the MI355X (gfx950) renderer for the hybrid Fourier-real
 * mixture-of-Gaussians galaxy-PSF convolution of Lang (2020),
 * "A hybrid Fourier-Real Gaussian Mixture method for fast galaxy-PSF
 * convolution", arXiv:2012.15797.
 *
 * Method (Section 2, steps 1-8): the FFT of the pixelized PSF (cached per PSF
 * and stamp size) is multiplied by the analytic Fourier transform of the
 * affine-transformed, sub-pixel-shifted Gaussian-mixture galaxy evaluated on
 * the FFT frequency grid, and inverse-FFT'd; mixture components that would
 * alias (wrap around) are instead convolved analytically with a single
 * Gaussian approximation of the PSF and evaluated in pixel space.
 *
 * Conventions used by every call:
 *   - All functions return gfc_status (0 = OK, < 0 = error).  No C++
 *     exception crosses the ABI.  On error a message is available from
 *     gfc_last_error() on the calling thread.
 *   - With GFC_LOG=1 in the environment (read once), errors and the
 *     library's events (PSF-FT cache fills, render calls, server
 *     submissions, batch launches and completions) are also written to
 *     stderr as JSON lines {"t": seconds, "event": name, ...}.  The host side
 *     of those steps carries roctx ranges for rocprofv3 --marker-trace.
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory.  Host inputs are copied
 *     before the call returns; the caller keeps ownership of everything it
 *     passes.  Device buffers passed to an asynchronous call must stay alive
 *     until the stream has completed it.
 *   - Pixel (row r, column c) of a stamp has its centre at (x = c, y = r),
 *     0-based.  Stamps are float32, row-major [n][W][W].
 *   - A pixelized PSF of S_y x S_x pixels (both even) has its centre at pixel
 *     (S_y/2, S_x/2); that pixel is moved to frequency-grid index 0 and the
 *     grid is folded periodically modulo W (zero padding when W >= S).
 *   - Mixture variances are isotropic, in units of r_e^2 (Section 2 step 3:
 *     V = v I); amplitudes are used as given (never renormalised).
 *   - Step 4 routing: n_i = (W/2) / sqrt(tr C_i); component i is evaluated in
 *     Fourier space with weight w_i = 1 when n_i >= 4, in real space when
 *     n_i <= 3, and with both in between, w_i = smoothstep(n_i - 3).
 *   - At the Nyquist index of each axis the galaxy transform is the mean of
 *     its values at frequencies +1/2 and -1/2 (the product with the PSF
 *     spectrum is then exactly Hermitian and the inverse FFT exactly real).
 *   - Real-space components are point-sampled at pixel centres, not wrapped.
 */
#ifndef GFC_H_
#define GFC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GFC_OK = 0,
  GFC_EINVAL = -1,       /* bad argument (NULL handle, unsupported size, ...) */
  GFC_EUNSUPPORTED = -2, /* valid request this build does not implement */
  GFC_ENOMEM = -3,       /* device or host allocation failed */
  GFC_EDEVICE = -4,      /* a HIP runtime call failed; see gfc_last_error() */
  GFC_EBUSY = -5,        /* object in use (e.g. server still has requests) */
  GFC_EREJECTED = -6,    /* serving: request can never fit the memory budget */
  GFC_ETIMEOUT = -7      /* serving: wait timed out */
} gfc_status;

typedef struct gfc_ctx gfc_ctx;
typedef struct gfc_psf gfc_psf;
typedef struct gfc_mix gfc_mix;
typedef struct gfc_server gfc_server;

/* Largest number of mixture components per table. */
#define GFC_KMAX 16

/* Per-call flags (Section 2 step 4 routing overrides). */
enum {
  GFC_FORCE_FOURIER = 1, /* every component in Fourier space (w_i = 1) */
  GFC_FORCE_REAL = 2,    /* every component in real space (w_i = 0) */
  GFC_RAMP_LINEAR = 4,   /* linear ramp w_i = n_i - 3 instead of smoothstep */
  GFC_SHIFT_LANCZOS3 = 8, /* sub-pixel shift by Lanczos-3 interpolation of the finished
                            stamp instead of the Fourier phase (step 8): the galaxy is
                            rendered at (floor x, floor y), then the stamp, real-space
                            terms included, is shifted by the fractional parts with the
                            six normalised weights L(d + f), d = -3..2, L(t) = sinc(t)
                            sinc(t/3), pixels outside the stamp taken as zero.  Forward
                            only (the adjoint returns GFC_EUNSUPPORTED). */
  GFC_ACCUMULATE = 16    /* add the rendered stamps to the values already in `out`
                            instead of overwriting them (several galaxies in one
                            stamp, e.g. a bulge and a disk with different shapes);
                            not combinable with GFC_SHIFT_LANCZOS3 nor used by the
                            server */
};

const char* gfc_status_str(gfc_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* gfc_last_error(void);

/* Supported stamp sizes W: 16, 32, 64, 128, 256. Returns 1 if supported. */
int gfc_stamp_size_supported(int W);

/* ---------------------------------------------------------------- context */
/* Binds to HIP device `hip_device`.  Owns the PSF-FT caches of the PSFs
 * created on it and a device counter of invalid galaxies. */
gfc_status gfc_ctx_create(int hip_device, gfc_ctx** out);
/* Synchronises the device, then frees the context.  All PSFs, mixtures and
 * servers created on it must have been destroyed first (GFC_EBUSY if not). */
gfc_status gfc_ctx_destroy(gfc_ctx* ctx);
/* Number of galaxies rendered with invalid parameters (|e| >= 1, r_e <= 0,
 * a non-finite value, |x| or |y| > 2^23, mix_id out of range) since the
 * context was created.  Synchronises the device. */
gfc_status gfc_ctx_invalid_count(gfc_ctx* ctx, uint64_t* n_invalid);

/* ------------------------------------------------------------------- PSF */
/* Steps 1-2.  pix: host, S_y*S_x row-major pixel values (copied).  S_y, S_x
 * even, 2..1024.  gauss: host pointer to {mu_x, mu_y, c_xx, c_xy, c_yy, amp}
 * (float64) describing the single-Gaussian PSF approximation used by
 * real-space components (Step 8), mu relative to the centre pixel; NULL
 * selects moment matching about the centre pixel with amp = sum of pixels.
 * The covariance must be positive semi-definite (else GFC_EINVAL). */
gfc_status gfc_psf_create(gfc_ctx* ctx, const float* pix, int S_y, int S_x,
                          const double* gauss, gfc_psf** out);
gfc_status gfc_psf_create_f64(gfc_ctx* ctx, const double* pix, int S_y, int S_x,
                              const double* gauss, gfc_psf** out);
/* Spatially varying PSF (Section 2, step 2: PSF models whose pixelized
 * components carry polynomial amplitudes over the image; their transforms
 * are cached once and weighted per galaxy).  comps: host, J (1..16)
 * component images [J][S_y][S_x] float32 (copied).  The PSF at image
 * position (X, Y) is sum_j c_j comps[j] with
 *   c_j = sum_t coef[j][t] u^a_t v^b_t,  u = (X - norm[0]) / norm[1],
 *   v = (Y - norm[2]) / norm[3],
 * over the T = (degree+1)(degree+2)/2 terms with a + b <= degree (0..3),
 * ordered by the power of v, then of u: 1, u, ..., u^degree, v, u v, ...
 * coef: host float64 [J][T]; norm: host float64[4] (scales non-zero).
 * The real-space PSF Gaussian is the moment Gaussian of the PSF at each
 * galaxy's position (moments about the centre pixel; the summed PSF must
 * have a positive total there).  Renders with such a PSF need
 * gfc_galaxies.psf_x/psf_y; the adjoint and the server take constant PSFs
 * only (GFC_EUNSUPPORTED). */
gfc_status gfc_psf_create_eigen(gfc_ctx* ctx, const float* comps, int J, int S_y, int S_x,
                                int degree, const double* coef, const double* norm,
                                gfc_psf** out);
/* Writes the Gaussian approximation in use to gauss_out[6] (host).
 * GFC_EUNSUPPORTED for a spatially varying PSF. */
gfc_status gfc_psf_gauss(const gfc_psf* psf, double* gauss_out);
/* Fills the PSF-FT cache for stamp size W on `hip_stream` (the render calls
 * do this lazily on first use of a size).  Cold path: one separable DFT of
 * the PSF in float64, stored as complex float32. */
gfc_status gfc_psf_prepare(gfc_psf* psf, int W, void* hip_stream);
/* Copies the cached PSF spectrum for size W into spec_out (device,
 * [W][W/2+1] interleaved complex float32, natural order: element
 * (k_y, k_x) = sum_{r,c} P[r][c] exp(-2 pi i (k_x (c - S_x/2) + k_y (r - S_y/2)) / W)).
 * For an eigen-PSF, the J component spectra one after another ([J][W][W/2+1]).
 * Fills the cache first if needed.  Asynchronous on hip_stream. */
gfc_status gfc_psf_spectrum(gfc_psf* psf, int W, float* spec_out, void* hip_stream);
/* Synchronises the context's device, then frees the PSF and its caches. */
gfc_status gfc_psf_destroy(gfc_psf* psf);

/* ------------------------------------------------------------- mixtures */
/* n_tables tables; table t has K[t] (1..GFC_KMAX) components.  amp, var:
 * host, [n_tables][GFC_KMAX] float32 row-major (entries past K[t] ignored);
 * var > 0 in r_e^2 units.  Copied to the device. */
gfc_status gfc_mix_create(gfc_ctx* ctx, int n_tables, const int* K, const float* amp,
                          const float* var, gfc_mix** out);
/* Device pointers to the table arrays (amp, var: [n_tables][GFC_KMAX]);
 * writes through amp_dev change the amplitudes used by later calls. */
gfc_status gfc_mix_device_tables(gfc_mix* mix, float** amp_dev, float** var_dev);
/* Replaces the amplitudes with amp_dev (device, [n_tables][GFC_KMAX]
 * float32; entries past K[t] ignored), asynchronously on hip_stream: later
 * calls on that stream see the new values.  This is how a fit updates the
 * amplitudes it differentiates (Section 3: the mixture amplitudes vary with
 * the profile). */
gfc_status gfc_mix_set_amp(gfc_mix* mix, const float* amp_dev, void* hip_stream);
gfc_status gfc_mix_destroy(gfc_mix* mix);

/* --------------------------------------------------------------- render */
/* Galaxy parameters, structure of arrays, device pointers of length n. */
typedef struct {
  const float* x;        /* centre, pixels */
  const float* y;
  const float* flux;     /* total flux F (rendered flux is F * sum_i A_i) */
  const float* r_e;      /* effective radius: pixels when cd == NULL */
  const float* e1;       /* ellipticity components, |e| < 1 */
  const float* e2;
  const int32_t* mix_id; /* device, table index per galaxy, or NULL (= 0) */
  const float* cd;       /* host, 4 floats {CD11, CD12, CD21, CD22} of the
                            local WCS matrix (pixel -> world), or NULL for the
                            identity; A = CD^{-1} E (Section 2 step 3) */
  const float* psf_x;    /* device, image position (X, Y) of each galaxy at which */
  const float* psf_y;    /* a spatially varying PSF is evaluated; required by an
                            eigen-PSF, ignored (may be NULL) for a constant PSF */
  const float* mix_amp;  /* device, [n_tables][GFC_KMAX] float32 amplitudes used by
                            this call instead of the mixture's (its component counts
                            and variances still apply), or NULL; the mixture itself
                            is not changed.  Not used by the Sersic and composite
                            renders, which build their own tables. */
} gfc_galaxies;

/* Steps 3-8 for n galaxies into stamps of size W, asynchronously on
 * hip_stream.  out: device, n*W*W float32 [n][W][W].  Galaxies with invalid
 * parameters get an all-NaN stamp and increment the invalid counter; the
 * call itself does not synchronise.  n == 0 is a no-op.  Apart from the
 * PSF-FT cache fill of the first call for a PSF and W (gfc_psf_prepare
 * makes it beforehand), no device memory is allocated inside the call at
 * any W: the half spectrum stays on the chip (at W = 256 one workgroup per
 * CU renders a stamp at a time).  The Sersic and composite renders below
 * allocate their per-galaxy tables. */
gfc_status gfc_render_stamps(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix,
                             const gfc_galaxies* gal, int64_t n, int W, unsigned flags,
                             float* out, void* hip_stream);

/* ---------------------------------------------- Sersic and composite galaxies */
/* A Sersic family (Section 1 profile family; closing discussion: mixture
 * amplitudes and variances vary smoothly with the Sersic index, so tables
 * fitted on a grid of indices are interpolated).  S (2..256) strictly
 * increasing indices n_grid (host float32), each with K (1..16) components:
 * amp, var host float32 [S][K] (var > 0, r_e^2 units).  Copied. */
typedef struct gfc_sersic gfc_sersic;
gfc_status gfc_sersic_create(gfc_ctx* ctx, int S, const float* n_grid, int K, const float* amp,
                             const float* var, gfc_sersic** out);
gfc_status gfc_sersic_destroy(gfc_sersic* fam);
/* Forward render of general-Sersic galaxies: galaxy i uses the mixture
 * interpolated piecewise-linearly in n between the two grid indices around
 * sersic_n[i] (device float32 [n]), per component for amplitudes and
 * variances.  sersic_n outside [n_grid[0], n_grid[S-1]] or not finite gives an
 * invalid galaxy (NaN stamp, counted).  gal->mix_id must be NULL.  Otherwise
 * as gfc_render_stamps; stream-ordered scratch of 136 bytes per galaxy. */
gfc_status gfc_render_stamps_sersic(gfc_ctx* ctx, gfc_psf* psf, const gfc_sersic* fam,
                                    const gfc_galaxies* gal, const float* sersic_n, int64_t n, int W,
                                    unsigned flags, float* out, void* hip_stream);
/* Forward render of bulge + disk galaxies sharing one ellipticity (Section 1,
 * composite profiles): one mixture per galaxy made of the disk table's
 * components with amplitudes (1 - f) A and the bulge table's with
 * amplitudes f A and variances rho^2 v, f = bulge_frac[i] in [0, 1] and
 * rho = bulge_rho[i] > 0 the bulge-to-disk r_e ratio (device float32 [n]);
 * gal->r_e is the disk's.  The two tables together have at most 16
 * components.  Out-of-range f or rho gives an invalid galaxy.  Bulges and
 * disks with different ellipticities: two calls, the second with
 * GFC_ACCUMULATE.  gal->mix_id must be NULL. */
gfc_status gfc_render_stamps_composite(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix, int disk_table,
                                       int bulge_table, const gfc_galaxies* gal, const float* bulge_frac,
                                       const float* bulge_rho, int64_t n, int W, unsigned flags,
                                       float* out, void* hip_stream);

/* Adjoint of gfc_render_stamps.  grad_out: device [n][W][W], the upstream
 * gradient dL/dI.  grad_params: device [n][6] float32 receiving
 * dL/d(x, y, flux, log r_e, e1, e2) (overwritten), or NULL.  grad_amp:
 * device [n_tables][GFC_KMAX] float32 to which dL/dA (summed over the
 * galaxies using each table) is ADDED in a fixed order (deterministic), or
 * NULL.  At e = 0 the derivative w.r.t. (e1, e2) is taken as 0 (the profile
 * has a cone there).  workspace: device scratch of at least
 * gfc_backward_workspace_bytes(n) bytes, or NULL to let the library
 * allocate it per call.  W = 256 also takes a stream-ordered device slab of
 * 256 KiB per stamp (at most 1024 stamps at a time) inside the call.  The
 * workspace holds the partial sums of grad_amp for up to 16 tables; with
 * more, they take a stream-ordered scratch of n_tables * ceil(n / 128) * 64
 * bytes inside the call when that is at most 64 MiB (above it they are
 * summed without one, more slowly).
 * Asynchronous on hip_stream. */
size_t gfc_backward_workspace_bytes(int64_t n);
gfc_status gfc_render_stamps_backward(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix,
                                      const gfc_galaxies* gal, int64_t n, int W,
                                      unsigned flags, const float* grad_out,
                                      float* grad_params, float* grad_amp,
                                      void* workspace, void* hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight fit loops, harnesses that forbid hipMalloc.  The adjoint of
 * gfc_render_stamps_backward with the same arguments (workspace aside) and
 * the same results, bit for bit, but its scratch (amplitude partials,
 * parameter gradients for a NULL grad_params, the per-table partial sums)
 * is a fixed array inside the library, one per device (24 MiB, taken when
 * the first context on that device is created and held until the process
 * ends).  It allocates and frees nothing.  Limits, each GFC_EINVAL: W <= 128,
 * n <= GFC_NOALLOC_MAX_GALAXIES, and the PSF spectrum for W already cached
 * (gfc_psf_prepare).  More than 16 tables are summed in one pass over the
 * galaxies, without partials.  Every call on a device uses that device's one
 * array: calls that overlap on one device (two streams, or two threads)
 * race and give wrong gradients, so the caller serialises them. */
#define GFC_NOALLOC_MAX_GALAXIES 262144
gfc_status gfc_render_stamps_backward_noalloc(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix,
                                              const gfc_galaxies* gal, int64_t n, int W,
                                              unsigned flags, const float* grad_out,
                                              float* grad_params, float* grad_amp,
                                              void* hip_stream);

/* -------------------------------------------------------------- serving */
/* Continuous batching.  A request carries HOST parameter arrays (copied at
 * submit).  Its output stamps live in a library-owned device buffer, charged
 * to the server's memory budget until released. */
typedef struct {
  gfc_psf* psf;
  const gfc_mix* mix;
  int W;
  int n;
  unsigned flags;
  const float *x, *y, *flux, *r_e, *e1, *e2; /* host, length n */
  const int32_t* mix_id;                      /* host or NULL */
} gfc_request;

/* mem_budget_bytes: device bytes the server may hold for admitted requests
 * (outputs + parameters: n * (4 W^2 + 32) bytes each, rounded up to 256);
 * max_batch_stamps: most stamps fused into one launch (<= 0: one launch per
 * request, the plain mode); n_streams: concurrent launch streams (1..8).  The
 * policy is that of the scheduling core below, with the key (mixture, stamp
 * size, flags): requests with different PSFs share a launch, each galaxy
 * reading its own request's PSF (steps 1-2: the transform of a PSF is made
 * once and kept).  The first request naming a PSF at a stamp size enters
 * that PSF's cached spectrum (filled then, if gfc_psf_prepare has not) and
 * its Gaussian in the server's device tables, on the submitting thread; a
 * server holds at most 65,536 PSFs, and a PSF must outlive the requests
 * naming it.  A background thread launches and reaps; it never fills a
 * cache.  The server reserves its budget (at most 80% of the device's free
 * memory) as one device allocation at creation and places batches in it;
 * when that is fragmented a batch takes a stream-ordered allocation
 * instead. */
gfc_status gfc_server_create(gfc_ctx* ctx, size_t mem_budget_bytes, int n_streams,
                             int64_t max_batch_stamps, gfc_server** out);
/* Queues a request; returns with a ticket once its parameters are copied
 * (and, the first time its PSF is seen at its stamp size, the PSF entered).
 * GFC_EREJECTED if the request alone exceeds the budget, GFC_EINVAL for a
 * malformed request. */
gfc_status gfc_server_submit(gfc_server* srv, const gfc_request* req, uint64_t* ticket);
/* done = 1 once the stamps are complete in device memory; out_dev then
 * points at [n][W][W] float32 (valid until release).  status_out (may be
 * NULL) receives the request's own status. */
gfc_status gfc_server_poll(gfc_server* srv, uint64_t ticket, int* done, const float** out_dev,
                           gfc_status* status_out);
/* Blocks until the request completes or timeout_ms passes (< 0: forever). */
gfc_status gfc_server_wait(gfc_server* srv, uint64_t ticket, int timeout_ms,
                           const float** out_dev);
/* Copies a finished request's stamps (n*W*W float32) into dst (device),
 * asynchronously on hip_stream.  GFC_EBUSY if the request is not done.  The
 * request may be released right after: the server reuses its memory only
 * once the copy has completed. */
gfc_status gfc_server_copy(gfc_server* srv, uint64_t ticket, float* dst, void* hip_stream);
/* Returns the request's device memory to the budget.  Work the caller
 * enqueued itself on the request's stamps (through out_dev) must have
 * completed before the call; copies made with gfc_server_copy need not. */
gfc_status gfc_server_release(gfc_server* srv, uint64_t ticket);
/* Latency (submit -> completion) percentiles over completed requests, and
 * stamps completed per second of server lifetime; also launches issued. */
gfc_status gfc_server_stats(gfc_server* srv, double* p50_ms, double* p99_ms, double* max_ms,
                            double* stamps_per_s, uint64_t* n_launches, uint64_t* n_done);
/* Open-loop load generator, for measuring a server without a client in the
 * way: request i (reqs[i], as for gfc_server_submit, copied at submission)
 * is submitted at t0 + t_arrive[i] seconds, t0 being the call's start, from
 * the calling thread; a second host thread waits for the requests in
 * submission order and releases each as soon as it completes.  Returns when
 * every submitted request is released.  t_arrive: host, n doubles, finite,
 * non-negative, non-decreasing.  lag: host, n doubles receiving how late
 * each submission was (seconds), or NULL.  span_s: seconds from t0 to the
 * last completion, or NULL.  keep: host array of n device pointers, or
 * NULL: request i's stamps (n_i W^2 float32) are copied to keep[i], when it
 * is not NULL, before the request is released (the replay waits for those
 * copies before it returns), so a caller can check a sample of the run.
 * Latencies are then in gfc_server_stats.  A rejected submission stops the
 * replay (GFC_EREJECTED after draining); a failed request gives its status.
 * Not to be called concurrently with other submissions to the same server. */
gfc_status gfc_server_replay(gfc_server* srv, const gfc_request* reqs, const double* t_arrive,
                             int64_t n, float* const* keep, double* lag, double* span_s);
/* Drains every queued request, then frees the server. */
gfc_status gfc_server_destroy(gfc_server* srv);

/* ------------------------------------------------- scheduling core (host) */
/* The server's scheduler with the device replaced by caller callbacks, for
 * driving and testing the policy without a GPU: strict-FIFO admission
 * against the memory budget, batches of admitted requests that share a key
 * (the server's is mixture, stamp size and flags) formed oldest-first up to
 * max_batch_stamps (<= 0: one request per launch, the plain mode), at most
 * one batch in flight per stream, latency = completion - submit on the
 * callbacks' clock.  Nothing runs in the background: each gfc_sched_step()
 * reaps completed batches, admits and launches. */
typedef struct gfc_sched gfc_sched;
typedef struct {
  void* user;
  double (*now)(void* user); /* seconds */
  /* start batch `batch` of n_req requests (tickets[]) and n_stamps stamps on
   * stream `stream`; return 0, or nonzero to fail the batch's requests */
  int (*launch)(void* user, uint64_t batch, int stream, int n_req, const uint64_t* tickets,
                int64_t n_stamps);
  int (*poll)(void* user, uint64_t batch); /* 1 done, 0 running, < 0 failed */
  void (*release)(void* user, uint64_t batch); /* its memory may be reused */
} gfc_sched_executor;

enum { GFC_REQ_PENDING = 0, GFC_REQ_ADMITTED = 1, GFC_REQ_LAUNCHED = 2, GFC_REQ_DONE = 3,
       GFC_REQ_FAILED = 4 };

gfc_status gfc_sched_create(const gfc_sched_executor* ex, size_t mem_budget_bytes, int n_streams,
                            int64_t max_batch_stamps, gfc_sched** out);
/* key: batching key; bytes: device bytes the request holds until released.
 * GFC_EREJECTED if bytes > budget. */
gfc_status gfc_sched_submit(gfc_sched* s, uint64_t key, int64_t n_stamps, size_t bytes,
                            uint64_t* ticket);
gfc_status gfc_sched_step(gfc_sched* s);
/* state: one of GFC_REQ_*; batch: the batch it was launched in (0 before). */
gfc_status gfc_sched_query(gfc_sched* s, uint64_t ticket, int* state, uint64_t* batch);
/* GFC_EBUSY unless the request is done or failed. */
gfc_status gfc_sched_release(gfc_sched* s, uint64_t ticket);
/* bytes currently charged to admitted, unreleased requests */
gfc_status gfc_sched_usage(gfc_sched* s, size_t* bytes_in_use, uint64_t* n_pending);
gfc_status gfc_sched_stats(gfc_sched* s, double* p50_ms, double* p99_ms, double* max_ms,
                           double* stamps_per_s, uint64_t* n_launches, uint64_t* n_done);
gfc_status gfc_sched_destroy(gfc_sched* s);

#ifdef __cplusplus
}
#endif

#endif /* GFC_H_ */
