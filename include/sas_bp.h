/*
 * sas_bp.h - time-domain backprojection (TDBP) for synthetic aperture sonar
 * on AMD MI355X (gfx950). C ABI: plain pointers and sizes only.
 *
 * What is computed (Eq. 1 and the inversion it defines, Sec. II-A; beam test
 * per pixel after block culling, Sec. II-C; transmitter and receiver tested
 * separately, Sec. III-B). For every pixel centre p of a regular grid, every
 * ping i and every receiver element e:
 *
 *   d_T = |p - T_i|,  d_R = |p - R_ie|,  tau = (d_T + d_R) / c
 *   u   = (tau - t0) * f_s,  n = floor(u),  w = u - n
 *   L   = (1 - w) * echo[i][e][n] + w * echo[i][e][n+1]   (samples outside
 *         [0, n_sample) read as zero)
 *   g   = [|p_x - T_x| <= sin(a) d_T] * [|p_x - R_x| <= sin(a) d_R]  (a = gate
 *         half-angle about the broadside plane; g = 1 when a = 0)
 *   I(p) = sum_i sum_e g * L * exp(+j 2 pi f_c tau)
 *
 * Positions are fixed during a ping (stop-and-hop) unless a swath selects
 * continuous motion (desc.motion, the receiver location x_RX(t) of Eq. 1
 * with the transmitter stationary while it transmits): the receivers then move
 * during reception, at the ping's velocity, R_ie(t) = R_ie + v_i t, or along
 * the ping's up-sampled position table, R_ie(t) = R_ie + Delta_i(t), and tau
 * is the root of c tau = d_T + |p - R_ie(tau)| (the gate keeps the ping-time
 * positions). Echoes are range compressed and at complex baseband, so the
 * carrier phase is re-applied.
 * Axes are north-east-down (Sec. II-B): x along-track, y across, z down.
 * A pixel centre is origin + index * spacing on each axis.
 *
 * Arithmetic: per tile of pixels and per (ping, element) the reference range
 * and carrier phase are formed in FP64 on the GPU; per-pixel delay offsets,
 * interpolation and accumulation run in FP32. Results agree with an FP64
 * evaluation of the sum to about 1e-5 relative L2 for FP32 echoes.
 *
 * Ownership: the caller allocates and owns every array passed in (echoes,
 * navigation, sound speed, images, gradients); they must stay valid until the
 * work enqueued on the caller's stream has completed. A plan owns one device
 * workspace slab sized when the plan is made, plus a captured HIP graph.
 *
 * Concurrency: a plan accepts one call in flight at a time; use one plan per
 * concurrent stream. Calls are asynchronous on the given stream.
 *
 * Errors: every function returns a status code; nothing is thrown across the
 * ABI. Arguments are checked on the host before anything is enqueued; a
 * failed check leaves outputs untouched. sas_bp_last_error_detail() gives a
 * thread-local message for the last failure on the calling thread.
 * Navigation or a sound speed that is not finite, or c below the plan's c_min,
 * is detected on the device: affected swaths produce zero images and the
 * plan's sticky status becomes SAS_BP_ENAV (read with sas_bp_plan_status()).
 */
#ifndef SAS_BP_H
#define SAS_BP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SAS_BP_ABI_VERSION 6

typedef struct sas_bp_plan_s* sas_bp_plan_t;

enum sas_bp_status {
    SAS_BP_OK = 0,
    SAS_BP_EINVAL = 1,        /* bad argument (size, pointer, alignment, value)   */
    SAS_BP_EUNSUPPORTED = 2,  /* valid but not supported (dtype, tiling, size)    */
    SAS_BP_ENOMEM = 3,        /* device allocation failed or workspace limit hit  */
    SAS_BP_EDEVICE = 4,       /* HIP runtime error                                */
    SAS_BP_ENAV = 5,          /* device found non-finite navigation or bad c      */
    SAS_BP_ECONVERGE = 6      /* refraction: a leg's crossing point did not converge within
                                 the Newton step cap (the image is written; the terms of
                                 such legs may carry a larger delay error)            */
};

/* Echo storage. Samples are complex, real part first.
 *   C64    : float  [P][E][N_s][2]
 *   F16X2  : half   [P][E][N_s][2], value = stored * echo_scale[i]
 *   BF16X2 : bfloat16 [P][E][N_s][2], value = stored * echo_scale[i]
 * Interpolation and accumulation are FP32 for every storage type. */
enum sas_bp_echo_dtype {
    SAS_BP_ECHO_C64 = 0,
    SAS_BP_ECHO_F16X2 = 1,
    SAS_BP_ECHO_BF16X2 = 2
};

/* Interpolation of the echo at the sample position u (Sec. II-A's sum reads
 * the echo between samples; the paper does not name the interpolator):
 *   LINEAR : (1 - w) E[n] + w E[n+1], n = floor(u), w = u - n (the default)
 *   SINC8  : sum over m = n - 3 .. n + 4 of E[m] h(u - m), the Hann-windowed
 *            sinc h(t) = sinc(t) (1 + cos(pi t / 4)) / 2; about 4x the work,
 *            image only (sas_bp_adjoint and sas_bp_reproject refuse it). */
enum sas_bp_interp {
    SAS_BP_INTERP_LINEAR = 0,
    SAS_BP_INTERP_SINC8 = 1
};

/* Receiver motion during reception (sas_bp_swath_desc.motion; the receiver
 * location x_RX(t) of Eq. 1, the transmitter stationary while it transmits):
 *   STOP_AND_HOP : receivers fixed at rx_pos for the whole ping (the default)
 *   VELOCITY     : R(t) = rx_pos + v t with v = io.rx_vel of the ping
 *   TABLE        : R(t) = rx_pos + Delta(t), Delta linear between the ping's
 *                  up-sampled track samples io.rx_track[j] at t = j track_dt
 *                  (and along the first and last segments beyond the ends),
 *                  the paper's interpolated position table (Sec. II-C).
 * t is time after transmit; tau solves c tau = |p - T| + |p - R(tau)|. The
 * beam gate keeps the ping-time positions. Linear interpolation only; image
 * only (the adjoint and reprojection refuse motion). For TABLE the kernel
 * takes, per tile and ping, the straight line of the table segment that holds
 * the tile centre's delay and certifies, per (tile, ping, element), that the
 * table departs from that line by at most 2e-6 m over the tile's delays
 * (from the largest velocity change between segments); a record that fails
 * that bound is reported like bad navigation (SAS_BP_ENAV). */
enum sas_bp_motion {
    SAS_BP_MOTION_STOP_AND_HOP = 0,
    SAS_BP_MOTION_VELOCITY = 1,
    SAS_BP_MOTION_TABLE = 2
};

/* One swath: acquisition constants and image grid. */
typedef struct {
    int32_t n_ping;         /* P >= 1                                          */
    int32_t n_elem;         /* E, 1..256 receiver elements per ping            */
    int32_t n_sample;       /* N_s, 2..2^31-1 samples per (ping, element)      */
    int32_t echo_dtype;     /* enum sas_bp_echo_dtype                          */
    int64_t n[3];           /* nx, ny, nz >= 1 (nz == 1: a 2D image)           */
    double origin[3];       /* centre of pixel (0,0,0), metres                 */
    double spacing[3];      /* > 0, metres; spacing[2] unused when nz == 1     */
    double f_c;             /* carrier frequency re-applied as exp(+j2 pi f_c tau), Hz, >= 0 */
    double f_s;             /* complex sample rate, Hz, > 0                    */
    double t0;              /* time of sample 0 after transmit, s             */
    double gate_half_angle; /* radians in [0, pi/2); 0 disables the beam gate */
    double c_min;           /* smallest sound speed the plan must accept, m/s; 0 selects 1400 */
    int32_t interp;         /* enum sas_bp_interp; all swaths of a plan share it */
    int32_t motion;         /* enum sas_bp_motion. All swaths of a plan share it. A
                               velocity (or table segment) that is not finite, of speed
                               >= c/2, or one that moves a delay by more than one sample
                               across a tile, is reported like bad navigation
                               (SAS_BP_ENAV). */
    int32_t refract;        /* 1: sediment-water interface refraction in the propagation
                               time (Sec. III-B): the flat seafloor z = z_interface
                               separates water (sound speed c, above; the array must be
                               in the water) from sediment (c_sediment, below); a leg to
                               a pixel below it crosses at the point of least travel time
                               (Snell's law), legs to pixels at or above it are straight;
                               the gate keeps straight lines. Linear interpolation, no
                               motion, image only; each leg's time is an FP32 offset
                               from an FP64 reference leg to its tile's centre column
                               (its crossing solved in FP64), the pixel's crossing
                               taken from the reference's second-order expansion when
                               a convexity bound certifies it, else from bracketed FP32
                               Newton steps (SAS_BP_ECONVERGE if those do not stop). */
    int32_t track_n;        /* samples per ping of io.rx_track, 2..2^24 (motion = TABLE) */
    double c_sediment;      /* m/s, > 0 (refract = 1)                             */
    double z_interface;     /* m, the interface depth (refract = 1)               */
    double track_dt;        /* s between samples of io.rx_track, > 0 (motion = TABLE) */
} sas_bp_swath_desc;

/* Where the plan's tiling comes from (sas_bp_options.tune_mode).
 *   DEFAULT : the explicit tile fields, else the automatic choice; sas_bp_autotune
 *             returns a stored choice for the shape class when there is one
 *             (process cache, then the tune_cache file) and times otherwise.
 *   CACHED  : sas_bp_plan takes the tiling stored for the plan's shape class
 *             (process cache, then the tune_cache file) in place of the tile
 *             and chunk fields, or the automatic choice when none is stored;
 *             sas_bp_autotune as for DEFAULT.
 *   SEARCH  : sas_bp_autotune always times the candidates and replaces the
 *             stored choice; sas_bp_plan as for CACHED.
 * A shape class is the GPU architecture, echo dtype, interpolator, motion
 * and propagation models, 2D/3D, gate on/off, and the largest element count,
 * window length and total pixels in power-of-two buckets. */
enum sas_bp_tune_mode {
    SAS_BP_TUNE_DEFAULT = 0,
    SAS_BP_TUNE_CACHED = 1,
    SAS_BP_TUNE_SEARCH = 2
};

/* Plan options; a NULL options pointer selects every default. */
typedef struct {
    int32_t device;          /* HIP device ordinal                             */
    int32_t tile_x, tile_y, tile_z; /* pixel tile shape; 0 = automatic         */
    int32_t pings_per_chunk; /* pings staged in LDS per pass (the adjoint's, and the
                                image's unless elems_per_chunk is set); 0 = automatic */
    int32_t threads;         /* threads per workgroup (256 or 512); 0 = automatic */
    int32_t use_graph;       /* 1 = replay a captured HIP graph (default), 0 = direct launches */
    int32_t elems_per_chunk; /* image: (ping, element) records staged per pass when
                                below n_elem (part of a ping; overrides pings_per_chunk
                                for the image, not the adjoint); 0 = automatic */
    size_t workspace_limit;  /* bytes; 0 = unlimited                           */
    int32_t tune_mode;       /* enum sas_bp_tune_mode                          */
    int32_t no_cull;         /* 1: no block culling (Sec. II-C): every ping of every tile
                                is visited and every (ping, element) is gated pixel row by
                                pixel row, as in a per-pixel field-of-view test. The image
                                is the same as with the cull (bitwise); this exists to show
                                that, and costs the time the cull saves. 0 = cull. */
    const char* tune_cache;  /* path of the tuning cache (JSON) that sas_bp_autotune
                                writes and CACHED / SEARCH plans read; NULL = the
                                process cache only. The file is rewritten whole (through
                                a temporary file and a rename) when a search stores a
                                choice; a file that cannot be read counts as empty. */
} sas_bp_options;

/* Device pointers for one swath. All must be device memory. */
typedef struct {
    const void* echo;        /* [P][E][N_s] complex, layout per echo_dtype; 16-byte aligned */
    const float* echo_scale; /* f32[P] for F16X2/BF16X2; ignored (may be NULL) for C64      */
    const double* tx_pos;    /* f64[P][3]   transmitter position of each ping               */
    const double* rx_pos;    /* f64[P][E][3] receiver positions                             */
    const double* c;         /* f64[1] sound speed, read on the device at every call        */
    void* image;             /* complex64 [nz][ny][nx] output (x fastest), overwritten      */
    const double* rx_vel;    /* f64[P][3] receiver velocity during reception of each ping,
                                m/s; required when desc.motion = VELOCITY, else ignored     */
    const double* rx_track;  /* f64[P][track_n][3] displacement of each ping's receivers
                                from rx_pos at t = j track_dt after transmit, m (normally 0
                                at j = 0); required when desc.motion = TABLE, else ignored  */
} sas_bp_swath_io;

/* Make a plan for n_swaths swaths (1..4096). Validates every descriptor,
 * chooses the tiling and allocates the workspace. On success *out holds a new
 * plan that the caller releases with sas_bp_destroy(). */
int sas_bp_plan(const sas_bp_swath_desc* desc, int n_swaths,
                const sas_bp_options* options, sas_bp_plan_t* out);

/* Workspace bytes sas_bp_plan() would allocate for these swaths (host only). */
int sas_bp_workspace_size(const sas_bp_swath_desc* desc, int n_swaths,
                          const sas_bp_options* options, size_t* bytes);

/* Form the image of every swath (the sum above), one image per io entry.
 * io has n_swaths entries matching the plan's descriptors. All swaths run in a
 * single persistent launch. stream is a hipStream_t (NULL = default). */
int sas_bp_image(sas_bp_plan_t plan, const sas_bp_swath_io* io, int n_swaths, void* stream);

/* Vector-Jacobian product of the image with respect to the geometry.
 * Given a cotangent Gbar per swath (complex64, image layout; Gbar =
 * dJ/dRe I + j dJ/dIm I), writes
 *   grad_tx[s] : f64[P][3]    dJ/dT_i
 *   grad_rx[s] : f64[P][E][3] dJ/dR_ie
 *   grad_c[s]  : f64[1]       dJ/dc
 * using dI/dtau = [f_s (E[n+1] - E[n]) + j 2 pi f_c L] exp(j 2 pi f_c tau),
 * dtau/dT = (T - p)/(c d_T), dtau/dR = (R - p)/(c d_R), dtau/dc = -tau/c
 * (gate held fixed). Outputs are overwritten. Reduction order is fixed, so
 * results are bitwise reproducible for a given plan. The adjoint stages whole
 * pings; with a tiling whose window of one ping's elements exceeds the LDS,
 * it returns SAS_BP_EUNSUPPORTED (the plan's image still works). */
int sas_bp_adjoint(sas_bp_plan_t plan, const sas_bp_swath_io* io,
                   const void* const* grad_image, double* const* grad_tx,
                   double* const* grad_rx, double* const* grad_c,
                   int n_swaths, void* stream);

/* Reprojection: the linear adjoint of the image with respect to the echo
 * (the transpose of the backprojection sum; the echo-to-image map of Eq. 1
 * inverted, Sec. II-A, is complex-linear, I = A E). For an image-shaped
 * complex64 Y per swath (image_in[s], layout of sas_bp_swath_io.image) it
 * writes echo_out[s] = A^H Y, complex64 [P][E][N_s] in the echo layout,
 * overwritten: every term with g = 1 adds
 *   (1 - w) exp(-j 2 pi f_c tau) Y(p)   to sample n = floor(u)
 *   w       exp(-j 2 pi f_c tau) Y(p)   to sample n + 1
 * of row (ping, element), for samples inside the record. With Y = Gbar
 * (dJ/dRe I + j dJ/dIm I) this is dJ/dRe E + j dJ/dIm E. Navigation, c and
 * the plan's tiling are those of sas_bp_image (io as for sas_bp_image; its
 * echo and image are not read or written). The output is the same for
 * 16-bit echo plans (the gradient with respect to the dequantised echo).
 * Within a tile of pixels, contributions are summed in fixed point (int32,
 * resolution about 1e-6 of the tile's largest |Re Y|, |Im Y|); across tiles
 * with float atomics, so results agree with the definition to FP32 rounding
 * but are not bitwise reproducible. A tile whose Y holds a non-finite value
 * contributes nothing. Buffers must be 8-byte aligned device memory.
 * Asynchronous on `stream`. */
int sas_bp_reproject(sas_bp_plan_t plan, const sas_bp_swath_io* io, const void* const* image_in,
                     void* const* echo_out, int n_swaths, void* stream);

/* Exact number of (pixel, ping, element) terms with g = 1 for each swath,
 * from the same per-row cone intervals the image kernels use. Writes
 * counts[s] (host memory) and synchronises the stream. */
int sas_bp_useful_updates(sas_bp_plan_t plan, const sas_bp_swath_io* io, int n_swaths,
                          void* stream, int64_t* counts);

/* Image sharpness S = sum|I|^4 / (sum|I|^2)^2 over n_pix complex64 pixels
 * (the autofocus objective) and, if grad_image is not NULL, its cotangent
 * Gbar = 4 I (|I|^2/B^2 - A/B^3) with A = sum|I|^4, B = sum|I|^2. Sums are
 * FP64 in a fixed order (bitwise reproducible). out_S is a device pointer to
 * one double; the plan lends its workspace for the partial sums. Asynchronous. */
int sas_bp_sharpness(sas_bp_plan_t plan, const void* image, int64_t n_pix, double* out_S,
                     void* grad_image, void* stream);

/* Allocation-free variant of sas_bp_sharpness, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same S and cotangent, computed by the
 * same kernels in the same fixed order (bitwise equal to sas_bp_sharpness), with
 * the partial sums in a fixed array of 2 x 1024 + 2 doubles (16.4 KB) that the
 * library keeps on every device it runs on until the process ends. Needs no
 * plan; runs on the calling thread's current device (stream must belong to it);
 * calls no allocating routine. The array's address is looked up on the first
 * call on each device. n_pix in [1, SAS_BP_SHARPNESS_STATIC_MAX_PIX]; larger
 * sizes return SAS_BP_EINVAL. Every call on one device shares the array (each
 * call overwrites all of it before reading it): calls that overlap on one
 * device, on different streams or threads, race. Pointers as for
 * sas_bp_sharpness (device memory, 8-byte aligned). Asynchronous on `stream`. */
#define SAS_BP_SHARPNESS_STATIC_MAX_PIX (1ll << 34)
int sas_bp_sharpness_static(const void* image, int64_t n_pix, double* out_S, void* grad_image, void* stream);

/* Range compression and basebanding of swath `swath`'s echo cube, in place:
 * the matched filter with the transmitted waveform q of Eq. 1 (Sec. II-A),
 * which yields the compressed complex baseband echo the image reads. For each
 * (ping, element) row x[k] of N_s samples at t_k = t0 + k / f_s (the swath's
 * t0 and f_s):
 *   b[k] = x[k] exp(-j 2 pi f_c t_k)          (mix != 0: x is the analytic
 *                                              received signal; mix == 0: x is
 *                                              already at baseband, b = x)
 *   y[n] = sum_{m<M} b[n + m] conj(q[m]) / sum_m |q[m]|^2,  b[k] = 0 for k >= N_s,
 * so a delayed copy of q compresses to a peak of one at its delay.
 * echo: complex64 [P][E][N_s] with the swath's sizes, device memory, 8-byte
 * aligned, overwritten with y. replica: complex64 q[0..n_taps) device memory,
 * the waveform's baseband samples at f_s from the start of transmission,
 * 1 <= n_taps <= N_s; a replica of zero energy gives zeros. Fast correlation
 * with FP32 transforms; the carrier phase is reduced in FP64 and the replica
 * energy summed in FP64. n_taps <= 2048: one fused kernel (overlap-save in
 * 4096-point segments, transforms in LDS, one workgroup per row); the plan
 * keeps a 64 KiB + 8 N_s byte workspace. Longer replicas: rocFFT (through
 * hipFFT) over rows zero-padded to a length L >= N_s + n_taps - 1 with only
 * the factors 2, 3 and 5, in batches of at most 1024 rows and 256 MiB; the
 * plan keeps those transforms and an 8 B L (rows per batch + 1) + 8 N_s byte
 * workspace of the last call's size (remade when the size changes). Calls
 * on one plan must be ordered on one stream. Asynchronous on `stream`. */
int sas_bp_range_compress(sas_bp_plan_t plan, int swath, void* echo, const void* replica, int32_t n_taps,
                          int mix, void* stream);

/* Time-delay estimation between consecutive pings for the displaced-phase-
 * centre motion estimate (Sec. II-D: the measured delay of Eq. 4 from
 * overlapped coherent looks of the seafloor). For every ping pair (i, i + 1)
 * and window k (samples [k hop, k hop + win), K = (N_s - win) / hop + 1
 * windows, reference time t0 + (k hop + win / 2) / f_s), with the n_pairs
 * element pairs (e1 of ping i, e2 of ping i + 1) whose phase centres overlap:
 *   r(l) = sum_j sum_n echo[i][e1_j][n] conj(echo[i + 1][e2_j][n + l]),
 *          |l| <= max_lag, samples outside the record read zero;
 *   l* = first maximum of |r| over |l| < max_lag; mu = (m_- - m_+) /
 *   (2 (m_- - 2 m_0 + m_+)) from |r| at l* - 1, l*, l* + 1 (0 on a flat top);
 *   out[i][k] = { (l* + mu) / f_s  (coarse delay of ping i + 1 after ping i, s),
 *                 arg of the quadratic interpolation of r at l* + mu (rad; for a
 *                 common return delayed by delta it is 2 pi f_c delta mod 2 pi),
 *                 rho = |r(l*)| / sqrt(sum |a|^2 sum |b(l*)|^2),  l* }.
 * echo: complex64 [P][E][N_s] with the swath's sizes (device, 8-byte aligned);
 * pairs: host int32 [n_pairs][2], 1 <= n_pairs <= 256, elements in [0, E);
 * 2 <= win <= min(2048, N_s); hop >= 1; 1 <= max_lag <= 64; out: device float
 * [P - 1][K][4], 16-byte aligned. Correlations accumulate in FP32, the peak
 * step is FP64. The plan keeps a 2 KiB pair buffer and pinned staging (the
 * caller's pairs array may be reused on return). Asynchronous on `stream`. */
int sas_bp_dpc_tde(sas_bp_plan_t plan, int swath, const void* echo, const int32_t* pairs, int n_pairs,
                   int32_t win, int32_t hop, int32_t max_lag, float* out, void* stream);

/* Motion estimate of Sec. II-D from the measured delays (Eqs. 3-8): the
 * per-ping sway and heave velocities v_y, v_z (the surge v_x is known)
 * minimising L = sum w h(g / sigma) + lambda_smooth sum (v'')^2 +
 * lambda_dvl sum (z_i - z_DVL[i])^2, with the Eq. 4 residual of ping pair i
 * and window k
 *   g = c^-1 mean_j (|TX_i - p_s| + |p_s - RX_i,e1j(t_k)| - |TX_i+1 - p_s| - |p_s - RX_i+1,e2j(t_k)|) + delay,
 * positions integrated from the velocities, p_i(0) = p0 + sum_{n<i} v_n dt_n,
 * moving on during reception (p_i(t) = p_i(0) + v_i t), TX = p + lever_tx,
 * RX_e = p + lever_rx[e] (fixed attitude), z_i = p_z,i(0), h the square
 * (robust = 0, Eq. 5) or the Huber function of Eq. 3 (robust = 1). */
typedef struct {
    int32_t n_ping;        /* P, 2..65536 (the solve: 2..4096)                  */
    int32_t n_window;      /* K >= 1 windows per ping pair                      */
    int32_t n_pairs;       /* J, 1..256 element pairs (e1 of ping i, e2 of ping i + 1) */
    int32_t n_elem;        /* elements with lever arms                          */
    int32_t robust;        /* 0: h(a) = a^2; 1: Huber (Eq. 3)                   */
    int32_t max_iter;      /* Levenberg-Marquardt iterations, 1..1000           */
    double c;              /* sound speed, m/s                                  */
    double sigma;          /* residual scale, s (> 0)                           */
    double lambda_smooth;  /* Eq. 6 weight (>= 0)                               */
    double lambda_dvl;     /* Eq. 7 weight (>= 0)                               */
    double p0[3];          /* platform position at ping 0's transmission        */
    double lever_tx[3];    /* transmitter lever arm                             */
} sas_bp_dpc_desc;

/* Footprints p_s [P-1][K][3] (host) from a nominal navigation (host vel_nominal
 * [P][3], dt [P-1]): for ping pair i the point of the flat seafloor z = z_floor
 * abeam (same x) of the pairs' mean phase centre of ping i on the look side
 * (look = +1: +y, -1: -y) whose two-way time from it is t_ref[k]. Host only. */
int sas_bp_dpc_footprints(const sas_bp_dpc_desc* desc, const double* vel_nominal, const double* dt,
                          const double* lever_rx, const int32_t* pairs, const double* t_ref, double z_floor,
                          double look, double* out);

/* The Eq. 4 residual of every (ping pair, window) and its derivatives, FP64
 * on the GPU: rows[i][k][7] = { g, dg/dP_i (y, z), dg/dv_i (y, z), dg/dv_i+1
 * (y, z) } with P_i ping i's position (dg/dv_n = dt_n dg/dP_i for n < i), and
 * pos_out [P][3] the integrated positions. All pointers are device memory:
 * vel [P][3], dt [P-1], lever_rx [E][3], pairs int32 [J][2], t_ref [K],
 * footprint [P-1][K][3], delay [P-1][K]. Asynchronous on `stream`. */
int sas_bp_dpc_residual(const sas_bp_dpc_desc* desc, const double* vel, const double* dt, const double* lever_rx,
                        const int32_t* pairs, const double* t_ref, const double* footprint, const double* delay,
                        double* pos_out, double* rows, void* stream);

/* Fine delays (Sec. II-D, the second step of the estimate): the correlation
 * phase of every (ping pair, window) unwrapped around the delay a first motion
 * solution predicts. tde: device float [n][4] as written by sas_bp_dpc_tde
 * (its phase, element 1, is used); rows: device double [n][7], the
 * sas_bp_dpc_residual rows of the first solution evaluated with a zero
 * measured delay, so that -rows[r][0] is the delay the solution predicts;
 * writes out[r] = (phi + 2 pi m) / (2 pi f_c) (device double [n], seconds),
 * m the integer nearest f_c (-rows[r][0]) - phi / (2 pi). The fine delays then
 * replace the coarse ones in a second sas_bp_dpc_solve. FP64; n in [1, 2^31];
 * f_c > 0 (the swath's carrier); tde 16-byte aligned. Asynchronous on
 * `stream`. */
int sas_bp_dpc_fine_delay(const float* tde, const double* rows, int64_t n, double f_c, double* out, void* stream);

/* Levenberg-Marquardt solve of the motion estimate (host arrays: vx [P], dt
 * [P-1], lever_rx [E][3], pairs [J][2], t_ref [K], footprint [P-1][K][3],
 * delay and weight [P-1][K], z_dvl [P]; vyz [P][2] holds the start and
 * receives the solution; *loss_out (optional) the final L). Residuals and
 * Jacobians on the GPU of `device` each pass; the normal equations, built from
 * per-pair sums (the integration makes dg/dv_n = dt_n dg/dP_i for every
 * n < i), and a dense Cholesky solve on the host; the Huber case by iteratively
 * reweighted least squares. Damping starts at 1e-3 (x1/3 on success, x4 on a
 * rejected step, 10 tries); stops on no improvement or a step below 1e-12 of
 * the solution. Synchronous; allocates and frees its device workspace. */
int sas_bp_dpc_solve(const sas_bp_dpc_desc* desc, const double* vx, const double* dt, const double* lever_rx,
                     const int32_t* pairs, const double* t_ref, const double* footprint, const double* delay,
                     const double* weight, const double* z_dvl, double* vyz, double* loss_out, int device);

/* Spectral whitening of swath `swath`'s echo cube, in place (Eq. 9, Sec.
 * II-E): with X the DFT of each (ping, element) row of N_s samples, the power
 * estimate P^(f) = mean over rows of |X(f)|^2 and the power gain
 * G(f) = h(1 / (gamma mean_f P^ + P^(f))), h the normalisation to max G = 1
 * (0 dB smallest attenuation); every row's spectrum is multiplied by
 * sqrt(G(f)) and transformed back. echo is complex64 [P][E][N_s] with the
 * swath's sizes. gamma >= 0. Rows of 4096, 8192 or 16384 samples use the
 * library's own transforms (FP32, in LDS; per-bin power summed in FP32 over
 * each workgroup's run of rows, then in FP64 over the runs in a fixed order);
 * other lengths use rocFFT through hipFFT (FP64 power sums in a fixed order),
 * whose FFT plan the plan makes on the first call. The plan allocates a
 * workspace of at most 34 MB on the first call. Asynchronous on `stream`. */
int sas_bp_whiten(sas_bp_plan_t plan, int swath, void* echo, double gamma, void* stream);

/* Time-varying gain of swath `swath`'s echo cube, in place (Eq. 10, Sec.
 * II-E): per sample time t, P~(t) = the population median of |E|^2 over all
 * (ping, element) (the element of rank floor((P E - 1) / 2)), and the power
 * gain G(t) = (alpha mean_t P~ + P~(t))^-1, applied as sqrt(G(t)) to the
 * complex samples; a time whose G is not finite (alpha = 0 and a zero
 * median) is left unchanged. echo is complex64 [P][E][N_s] with the swath's
 * sizes, whatever the plan's echo dtype (the gain conditions the echo before
 * any 16-bit storage). If gain_out is not NULL it receives G as f32[N_s]
 * (device memory). alpha >= 0. The medians are exact radix selections on the
 * FP32 squared magnitudes. The plan allocates 8 N_s bytes of workspace on
 * the first call. Asynchronous on `stream`. */
int sas_bp_tvg(sas_bp_plan_t plan, int swath, void* echo, double alpha, float* gain_out, void* stream);

/* Echo envelope of swath `swath` for the incoherent stage of the sharpness
 * autofocus (Sec. II-A's delay-and-sum with the carrier phase removed: its
 * sharpness varies on the scale of the range resolution, not the
 * wavelength): every sample e of the cube [P][E][N_s] becomes (|e|, 0), in
 * the swath's echo storage format (complex64, or FP16/BF16 pairs; per-ping
 * scales unchanged). |e| = sqrt(re^2 + im^2) in FP32, correctly rounded, then
 * rounded to nearest-even for 16-bit storage (a magnitude beyond the format's
 * range becomes infinite). echo and out are device memory, 8-byte (complex64)
 * or 4-byte aligned, equal (in place) or disjoint. Asynchronous on `stream`. */
int sas_bp_envelope(sas_bp_plan_t plan, int swath, const void* echo, void* out, void* stream);

/* Dynamic range compression of an image for display (Eqs. 11-12, Sec.
 * II-E). x = |I| / max |I| over the n_pix complex64 pixels of image; each
 * pixel maps to out[i] = q x / ((q - 1) x + 1) (FP32, n_pix floats), with
 * q = (b - b x~) / (x~ - b x~) so that the median x~ (the element of rank
 * floor((n_pix - 1) / 2)) maps to the brightness b in (0, 1). Degenerate
 * images: all zero -> zeros (q = 1); x~ = 0 -> every non-zero pixel to 1
 * (q = +inf); x~ = 1 -> every pixel below the maximum to 0 (q = 0). The
 * median is an exact radix selection on the FP32 squared magnitudes. If
 * params is not NULL it receives (device memory, 3 doubles) max |I|, x~ and
 * q. n_pix in [1, 2^31]. The plan lends a small workspace; asynchronous. */
int sas_bp_drc(sas_bp_plan_t plan, const void* image, int64_t n_pix, double brightness, float* out,
               double* params, void* stream);

/* Sticky device-detected status of the plan (SAS_BP_OK, SAS_BP_ENAV, or
 * SAS_BP_ECONVERGE when no navigation fault was seen); synchronises with the
 * device and clears it. */
int sas_bp_plan_status(sas_bp_plan_t plan);

/* Chosen tiling, for reporting: tile_x, tile_y, tile_z, pings_per_chunk
 * (adjoint), window samples, image LDS bytes per workgroup, image workgroups
 * launched, threads per workgroup, image records per chunk, image workgroups
 * resident per CU. */
int sas_bp_plan_info(sas_bp_plan_t plan, int64_t info[10]);

/* Autotuner (tile shape and chunk size). Times every candidate tiling of the
 * lane-layout menu (2D layouts for images, 3D ones for volumes) with the
 * automatic chunk, 1, 2, 4 and 8 pings per chunk and 3/4, 1/2 and 1/4 of a
 * ping's elements per chunk, each that fits the device, running the image of
 * these swaths on the caller's buffers (io: as for sas_bp_image; the images
 * are overwritten) on `stream`: one warm-up and `reps` timed launches each,
 * measured with HIP events. Writes the fastest candidate's options to *best
 * (device and workspace_limit copied from `base`, which may be NULL) and its
 * mean time to *best_ms (host memory). The choice is stored per shape class
 * (see sas_bp_tune_mode) in the process cache and, when base->tune_cache is
 * set, in that file: unless base->tune_mode is SEARCH, a later call for the
 * same class, in this process or (through the file) in another, returns it
 * without timing, with *best_ms = 0. The returned options carry tune_mode
 * DEFAULT and base's device, workspace_limit, no_cull and tune_cache.
 * Synchronous; creates and destroys one plan per candidate. */
int sas_bp_autotune(const sas_bp_swath_desc* desc, int n_swaths, const sas_bp_swath_io* io,
                    const sas_bp_options* base, int reps, void* stream, sas_bp_options* best, double* best_ms);

/* The block-cull predicates of the image kernels (Sec. II-C: a block of pixels
 * is kept for a ping when its pixels may lie inside the beam; Sec. III-B: the
 * transmitter and each receiver are tested as separate apexes), evaluated on
 * the host for one cone apex and one axis-aligned box of pixel centres
 * [box_lo, box_hi] (metres). The cone is |x - apex_x| <= tan(half_angle) rho,
 * rho the (y, z) distance to the apex, which is the gate |dx| <= sin(half_angle)
 * |p - apex| rearranged. Writes
 *   *record_class : 0 every point of the box is outside the cone, 1 every point
 *                   is inside, 2 neither can be shown (decided per pixel row);
 *                   the class each (tile, ping, element) record gets;
 *   *may_hit      : 0 only if no point of the box is inside (the per-(tile, ping)
 *                   test of the cull pass; a conservative superset of class != 0).
 * Both are exact for the box: a box that the beam crosses without holding any
 * of the box's corners is class 2 and may_hit 1. half_angle in (0, pi/2).
 * Host only; needs no device. */
int sas_bp_gate_class(const double apex[3], const double box_lo[3], const double box_hi[3], double half_angle,
                      int32_t* record_class, int32_t* may_hit);

/* Per-launch timing of the main kernel, for measuring it against its
 * roofline. With enable != 0, sas_bp_image and sas_bp_adjoint enqueue their
 * kernels directly (not through the captured graph) and bracket the
 * persistent image or adjoint kernel with a pair of HIP events on the
 * caller's stream; enable = 0 restores graph launches and drops pending
 * pairs. sas_bp_kernel_time waits for the recorded pairs, writes the sum of
 * their durations in milliseconds to *ms_total and their number to
 * *launches (host memory), and starts a new count. */
int sas_bp_set_kernel_timing(sas_bp_plan_t plan, int enable);
int sas_bp_kernel_time(sas_bp_plan_t plan, double* ms_total, int64_t* launches);

void sas_bp_destroy(sas_bp_plan_t plan);

const char* sas_bp_error_string(int status);
const char* sas_bp_last_error_detail(void);
int sas_bp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SAS_BP_H */
