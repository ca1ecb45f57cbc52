// Plan, workspace slab, graph capture/replay and the exported C ABI.
//
// A plan is made once per set of swath shapes. It validates the descriptors on
// the host, picks the tile shape and the records staged per pass, sizes one
// device slab for every buffer the kernels need (one allocation, the slab
// scheme of Sec. II-C), and captures the launch sequence
//     init -> cull -> cost order -> persistent image kernel
// into a HIP graph. The per-swath pointers and constants live in the slab, so
// the graph stays valid when callers pass new buffers or move the navigation
// and sound speed (device memory read at every replay).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "sas_bp.h"
#include "tdbp_dev.h"
#include "tdbp_geom.h"

namespace sasbp {
typedef void (*ImageKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);
ImageKernelFn image_kernel_for(int layout, bool gate, int dt, int interp);
int image_lds_bytes(int RC, int E, int W, int ROWS, bool gate, bool motion);
hipError_t launch_init(const Workspace& ws, hipStream_t st);
hipError_t launch_cull(const Workspace& ws, int n_tiles, int TX, int TY, int TZ, int bucket_shift, hipStream_t st);
hipError_t launch_order(const Workspace& ws, int n_tiles, int bucket_shift, hipStream_t st);
hipError_t launch_track_stats(const Workspace& ws, int swath, int n_ping, hipStream_t st);
hipError_t launch_image(ImageKernelFn fn, const Workspace& ws, int n_tiles, int grid, int threads, int lds_bytes,
                        hipStream_t st);
hipError_t image_occupancy(ImageKernelFn fn, int threads, int lds_bytes, int* blocks_per_cu);
hipError_t set_image_lds_limit(ImageKernelFn fn, int lds_bytes);

typedef void (*AdjointKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);
AdjointKernelFn adjoint_kernel_for(int layout, bool gate, int dt);
int adjoint_lds_bytes(int CP, int E, int W, int ROWS, bool gate, int threads);
hipError_t launch_adjoint(AdjointKernelFn fn, const Workspace& ws, int n_tiles, int grid, int threads, int lds_bytes,
                          hipStream_t st);
hipError_t adjoint_occupancy(AdjointKernelFn fn, int threads, int lds_bytes, int* blocks_per_cu);
hipError_t set_adjoint_lds_limit(AdjointKernelFn fn, int lds_bytes);

typedef void (*RefractKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);
RefractKernelFn refract_kernel_for(int layout, bool gate, int dt);
typedef void (*ReprojectKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);
ReprojectKernelFn reproject_kernel_for(int layout, bool gate);
hipError_t launch_reproject(ReprojectKernelFn fn, const Workspace& ws, int n_tiles, int grid, int threads,
                            int lds_bytes, hipStream_t st);
hipError_t launch_zero_rows(void* p, long long n, hipStream_t st);
hipError_t reproject_occupancy(ReprojectKernelFn fn, int threads, int lds_bytes, int* blocks_per_cu);
hipError_t set_reproject_lds_limit(ReprojectKernelFn fn, int lds_bytes);
hipError_t launch_drc(const void* image, long long n, double brightness, float* out, double* params, void* work,
                      hipStream_t st);
size_t drc_work_bytes();
hipError_t launch_envelope(const void* in, void* out, long long n, int dt, hipStream_t st);
hipError_t launch_tvg(void* echo, long long rows, int Ns, double alpha, float* work, float* gain_out,
                      hipStream_t st);
size_t whiten_work_bytes(int Ns);
int launch_whiten(void* fft_plan, void* echo, long long rows, int Ns, double gamma, void* work, hipStream_t st);
bool whiten_hand_written(int Ns);
int make_fft_plan(int Ns, long long rows, void** out);
void destroy_fft_plan(void* p);
int rc_transform_length(long long n);
int tde_max_lag();
hipError_t launch_dpc_residual(int P, int K, int J, const double* pos, const double* vel, const double* dt,
                               const double* lever_tx, const double* lever_rx, const int* pairs, const double* t_ref,
                               const double* ps, const double* delay, double c, double* rows, hipStream_t st);
hipError_t launch_dpc_fine_delay(long long n, const float* tde, const double* rows, double fc, double* out,
                                 hipStream_t st);
hipError_t launch_dpc_positions(int P, const double* vel, const double* dt, const double* p0, double* pos,
                                hipStream_t st);
size_t tde_lds_bytes(int W, int L, int J);
hipError_t launch_dpc_tde(const void* echo, int P, int E, int Ns, const int* pairs, int J, int W, int hop, int L,
                          double fs, float* out, hipStream_t st);
int rc_fused_taps();
int launch_range_compress_fused(void* echo, long long rows, int Ns, const void* replica, int M, double fc, double t0,
                                double fs, int apply_mix, void* filt, void* tw, void* mixtab, void* energy,
                                hipStream_t st);
int rc_make_plans(int L, int B, void** batch, void** single);
int launch_range_compress(void* batch_plan, void* single_plan, void* echo, long long rows, int Ns, int L, int B,
                          const void* replica, int M, double fc, double t0, double fs, int apply_mix, void* buf,
                          void* filt, void* mixtab, void* energy, hipStream_t st);
hipError_t launch_adjoint_reduce(const Workspace& ws, int n_swaths, int max_p, hipStream_t st);
hipError_t launch_count(const Workspace& ws, int s, int P, int E, int rows, unsigned long long* out, hipStream_t st);
hipError_t launch_sharpness(const void* image, long long n, double* partials, double* out_S, void* grad,
                            hipStream_t st);
}  // namespace sasbp

using namespace sasbp;

namespace {

thread_local std::string g_detail;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_detail = buf;
  return status;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(SAS_BP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));      \
  } while (0)

constexpr double kDefaultCmin = 1400.0;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Tiling {
  int layout, K, LX, LY, LZ, TX, TY, TZ, NT;
};

constexpr int kLdsMax = 160 * 1024;

struct SwathPlan {
  sas_bp_swath_desc d;
  int ntx, nty, ntz, ntiles, tile0;
  int W, CP, RC, SC;
  int no_cull;
  double half_diag, c_min;
  size_t tstats_off = 0;   // first ping of this swath's position-table statistics (motion = TABLE)
};

struct Layout {
  size_t swaths, prange, order, counters, bucket, tile_swath, scratch, drc, tstats, geo, total;
  size_t geo_stride;   // bytes of geometry scratch per resident workgroup
  int geo_slots;       // resident workgroups the geometry scratch serves
  size_t n_partials;   // adjoint records, allocated on the first adjoint call
};

// Compute units the geometry scratch is sized for (an MI355X has 256); a
// device with more runs at most this many times the per-CU occupancy.
constexpr int kMaxCUs = 256;

}  // namespace

struct sas_bp_plan_s {
  int device = 0;
  int n_swaths = 0;
  int n_tiles = 0;
  Tiling tiling{};
  bool gate_any = false;
  int dtype = 0;
  int interp = 0;                  // SAS_BP_INTERP_*, shared by all swaths of the plan
  int motion = 0;                  // continuous receiver motion, shared by all swaths of the plan
  int refract = 0;                 // sediment refraction, shared by all swaths of the plan
  int bucket_shift = 0;
  int lds_bytes = 0, adj_lds_bytes = 0;
  int image_launch_lds = 0;        // dynamic LDS of the image kernel's launch (0 for refraction)
  int grid = 0, adj_grid = 0;
  int occ = 0;                     // image workgroups resident per CU
  bool adj_ok = false;             // the adjoint's whole-ping chunks fit the device
  int max_pe = 0;
  int max_p = 0;
  bool use_graph = true;
  void* adj_buf = nullptr;   // adjoint partials + sound-speed partials
  void* tvg_buf = nullptr;   // time-varying gain: medians and factors per sample time
  void* whiten_buf = nullptr;          // whitening: partial power sums, estimate, factors
  std::vector<void*> fft_plans;        // per swath, made on the first whitening call
  struct {                             // range compression: transforms and buffers of the last call's size
    int L = 0, B = 0;                  // transform length, rows per batch
    void* batch = nullptr;             // FFT plans: B rows, one row
    void* single = nullptr;
    void* buf = nullptr;               // B x L complex rows
    size_t buf_bytes = 0;
    void* small = nullptr;             // filter (L), twiddles, mix table (N_s), replica energy
    size_t small_bytes = 0;
  } rc;
  int* tde_pairs = nullptr;            // time-delay estimation: element pairs on the device (kMaxTdePairs)
  int* tde_pairs_host = nullptr;       // pinned staging for them
  hipEvent_t tde_copied = nullptr;     // the last staging copy has been consumed
  std::vector<SwathPlan> sw;
  Layout lay{};
  unsigned char* slab = nullptr;
  float4* tstats = nullptr;        // per-ping position-table statistics (motion = TABLE), in the slab
  Workspace ws{};
  ImageKernelFn image_fn = nullptr;
  AdjointKernelFn adjoint_fn = nullptr;
  ReprojectKernelFn reproject_fn = nullptr;
  int rep_grid = 0;
  SwathDev* host_sw = nullptr;     // pinned mirror of ws.swaths
  std::vector<SwathDev> last_sw;   // what the device copy currently holds
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool timing = false;
  bool tuned_from_cache = false;   // the tiling came from the tuning cache
  std::vector<hipEvent_t> events;  // pairs bracketing the main kernel
  size_t n_timed = 0;              // pairs recorded since the last read
};

namespace {

bool finite(double v) { return std::isfinite(v); }

int validate(const sas_bp_swath_desc* d, int i) {
  if (d->n_ping < 1) return fail(SAS_BP_EINVAL, "swath %d: n_ping must be >= 1", i);
  if (d->n_elem < 1 || d->n_elem > kMaxElem) return fail(SAS_BP_EINVAL, "swath %d: n_elem must be in [1, %d]", i, kMaxElem);
  if (d->n_sample < 2) return fail(SAS_BP_EINVAL, "swath %d: n_sample must be >= 2", i);
  if (d->echo_dtype < 0 || d->echo_dtype > 2) return fail(SAS_BP_EUNSUPPORTED, "swath %d: unknown echo dtype %d", i, d->echo_dtype);
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 1) return fail(SAS_BP_EINVAL, "swath %d: n[%d] must be >= 1", i, a);
    if (d->n[a] > (1 << 20)) return fail(SAS_BP_EUNSUPPORTED, "swath %d: n[%d] too large", i, a);
    if (!finite(d->origin[a])) return fail(SAS_BP_EINVAL, "swath %d: origin[%d] not finite", i, a);
    if (!(d->spacing[a] > 0.0) || !finite(d->spacing[a])) {
      if (a < 2 || d->n[2] > 1) return fail(SAS_BP_EINVAL, "swath %d: spacing[%d] must be > 0", i, a);
    }
  }
  if ((long long)d->n[0] * d->n[1] * d->n[2] > (1ll << 34)) return fail(SAS_BP_EUNSUPPORTED, "swath %d: image too large", i);
  if (!(d->f_s > 0.0) || !finite(d->f_s)) return fail(SAS_BP_EINVAL, "swath %d: f_s must be > 0", i);
  if (!(d->f_c >= 0.0) || !finite(d->f_c)) return fail(SAS_BP_EINVAL, "swath %d: f_c must be >= 0", i);
  if (!finite(d->t0)) return fail(SAS_BP_EINVAL, "swath %d: t0 not finite", i);
  if (!(d->gate_half_angle >= 0.0) || !(d->gate_half_angle < 1.5707963267948966))
    return fail(SAS_BP_EINVAL, "swath %d: gate_half_angle must be in [0, pi/2)", i);
  if (!(d->c_min >= 0.0) || !finite(d->c_min)) return fail(SAS_BP_EINVAL, "swath %d: c_min must be >= 0", i);
  if (d->interp != SAS_BP_INTERP_LINEAR && d->interp != SAS_BP_INTERP_SINC8)
    return fail(SAS_BP_EINVAL, "swath %d: unknown interpolator %d", i, d->interp);
  if (d->motion < 0 || d->motion > 2) return fail(SAS_BP_EINVAL, "swath %d: motion must be 0, 1 or 2", i);
  if (d->motion == SAS_BP_MOTION_TABLE &&
      (d->track_n < 2 || d->track_n > (1 << 24) || !(d->track_dt > 0.0) || !finite(d->track_dt)))
    return fail(SAS_BP_EINVAL, "swath %d: a position table needs track_n in [2, 2^24] and track_dt > 0", i);
  if (d->motion && d->interp != SAS_BP_INTERP_LINEAR)
    return fail(SAS_BP_EUNSUPPORTED, "swath %d: continuous motion is built for linear interpolation only", i);
  if (d->refract != 0 && d->refract != 1) return fail(SAS_BP_EINVAL, "swath %d: refract must be 0 or 1", i);
  if (d->refract && (d->interp != SAS_BP_INTERP_LINEAR || d->motion))
    return fail(SAS_BP_EUNSUPPORTED, "swath %d: refraction is built for linear interpolation without motion", i);
  if (d->refract && (!(d->c_sediment > 0.0) || !finite(d->c_sediment) || !finite(d->z_interface)))
    return fail(SAS_BP_EINVAL, "swath %d: c_sediment must be > 0 and z_interface finite", i);
  return SAS_BP_OK;
}

// Tile shape from the lane-layout menu. An explicit tile (and optionally the
// threads per workgroup) must match a menu entry; otherwise 2D images use
// 64 x 32 pixel tiles (16 x 32 for small images, so that they still give
// enough tiles to occupy the GPU) and 3D volumes use 32 x 8 x 4 voxel tiles,
// all on 256 threads.
int choose_tiling(const sas_bp_swath_desc* d, int n, const sas_bp_options* o, Tiling* t) {
  bool any3d = false;
  long long pix = 0;
  for (int i = 0; i < n; ++i) {
    any3d |= d[i].n[2] > 1;
    pix += (long long)d[i].n[0] * d[i].n[1] * d[i].n[2];
  }
  int layout = any3d ? 6 : (pix < (1ll << 20) ? 0 : 2);
  if (o && (o->tile_x || o->tile_y || o->tile_z || o->threads)) {
    layout = -1;
    for (int l = 0; l < kNumLayouts && layout < 0; ++l) {
      const LaneLayout& L = kLayouts[l];
      const int tx = L.LX * L.K, ty = L.LY, tz = L.LZ, nt = L.LX * L.LY * L.LZ;
      if (o->tile_x && o->tile_x != tx) continue;
      if (o->tile_y && o->tile_y != ty) continue;
      if (o->tile_z && o->tile_z != tz) continue;
      if (!o->tile_z && (tz > 1) != any3d) continue;
      if (o->threads && o->threads != nt) continue;
      layout = l;
    }
    if (layout < 0)
      return fail(SAS_BP_EUNSUPPORTED, "no tiling with tile %dx%dx%d and %d threads", o->tile_x, o->tile_y,
                  o->tile_z, o->threads);
  }
  const LaneLayout& L = kLayouts[layout];
  t->layout = layout;
  t->K = L.K;
  t->LX = L.LX;
  t->LY = L.LY;
  t->LZ = L.LZ;
  t->TX = L.LX * L.K;
  t->TY = L.LY;
  t->TZ = L.LZ;
  t->NT = L.LX * L.LY * L.LZ;
  return SAS_BP_OK;
}

constexpr int kLdsBudget = 64 * 1024;

// LDS per workgroup that still lets the image kernel reach the occupancy its
// register budget allows (kImageWaves waves per SIMD, four SIMDs per CU). A
// plan with fewer tiles than that many workgroups over the device's CUs never
// fills those slots (each workgroup holds one tile at a time), so its chunks
// may take the LDS of the workgroups a CU actually runs (at least two): on
// 512 tiles over 256 CUs, two pings of 16 elements per chunk instead of one
// ran the image in 3.55 ms against 3.80 and the adjoint in 7.11 against 7.50.
int image_lds_target(int threads, long long tiles, int cus) {
  int per_cu = std::max(1, kImageWaves * 4 * 64 / threads);
  if (cus > 0 && tiles > 0) per_cu = (int)std::min<long long>(per_cu, std::max(2ll, (tiles + cus - 1) / cus));
  return kLdsMax / per_cu - 512;
}

// Compute units of the plan's device; 0 when they cannot be queried.
int device_cus(const sas_bp_options* o) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, o ? o->device : 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cus;
}

int build_swaths(const sas_bp_swath_desc* d, int n, const sas_bp_options* o, const Tiling& t,
                 std::vector<SwathPlan>* out, int* n_tiles) {
  out->clear();
  int tiles = 0;
  const int rows = t.TY * t.TZ;
  long long all_tiles = 0;
  for (int i = 0; i < n; ++i)
    all_tiles += ((d[i].n[0] + t.TX - 1) / t.TX) * ((d[i].n[1] + t.TY - 1) / t.TY) * ((d[i].n[2] + t.TZ - 1) / t.TZ);
  const int cus = device_cus(o);
  for (int i = 0; i < n; ++i) {
    SwathPlan s;
    s.d = d[i];
    s.no_cull = (o && o->no_cull) ? 1 : 0;
    s.ntx = (int)((d[i].n[0] + t.TX - 1) / t.TX);
    s.nty = (int)((d[i].n[1] + t.TY - 1) / t.TY);
    s.ntz = (int)((d[i].n[2] + t.TZ - 1) / t.TZ);
    const long long nt = (long long)s.ntx * s.nty * s.ntz;
    if (nt + tiles > (1ll << 30)) return fail(SAS_BP_EUNSUPPORTED, "too many tiles");
    s.ntiles = (int)nt;
    s.tile0 = tiles;
    tiles += s.ntiles;
    const double ex = (t.TX - 1) * d[i].spacing[0];
    const double ey = (t.TY - 1) * d[i].spacing[1];
    const double ez = d[i].n[2] > 1 ? (t.TZ - 1) * d[i].spacing[2] : 0.0;
    s.half_diag = 0.5 * std::sqrt(ex * ex + ey * ey + ez * ez);
    s.c_min = d[i].c_min > 0.0 ? d[i].c_min : kDefaultCmin;
    // window: delay offsets within the tile are bounded by +-2 r (triangle
    // inequality on both legs). With the window start rounded down to an even
    // sample (the staging load width), entries up to 4 r f_s / c + 4 are read;
    // one more entry of margin for FP32 rounding of the sample position.
    // Continuous motion moves a pixel's delay by at most one sample from the
    // tile centre's (the record build refuses more) and starts the window one
    // sample earlier: two more entries.
    s.W = (int)std::ceil(4.0 * s.half_diag * d[i].f_s / s.c_min) + 6 + (d[i].motion ? 2 : 0);
    if (s.W > 8192) return fail(SAS_BP_EUNSUPPORTED, "swath %d: tile spans %d samples; use a smaller tile", i, s.W);
    const int E = d[i].n_elem;
    const int ppc = (o && o->pings_per_chunk > 0) ? o->pings_per_chunk : 0;
    const int epc = (o && o->elems_per_chunk > 0) ? std::min(o->elems_per_chunk, E) : 0;
    const bool gate = d[i].gate_half_angle > 0.0;
    const bool mot = d[i].motion != 0;
    // adjoint chunk: whole pings
    int cp = ppc;
    if (cp == 0) {
      cp = 1;
      // (a plan too small to fill three workgroups per CU may use more)
      const int budget = std::max(kLdsBudget, image_lds_target(t.NT, all_tiles, cus));
      while (cp < 8 && image_lds_bytes(cp * 2 * E, E, s.W, rows, gate, false) <= budget) cp *= 2;
    }
    if (ppc > 0 && image_lds_bytes(cp * E, E, s.W, rows, gate, mot) > kLdsMax - 1024)
      return fail(SAS_BP_EUNSUPPORTED, "swath %d: %d pings x %d elements x %d samples exceed LDS", i, cp, E, s.W);
    s.CP = cp;   // if even one whole ping does not fit, the plan has no adjoint
    // image chunk in records: explicit elements (part of a ping), explicit
    // pings, or the largest of 8, 4, 2, 1 pings and then of E - 1, E - 2, ...
    // records whose LDS lets the kernel reach its register-bound occupancy
    // (such a chunk may straddle two pings)
    int rc = 0;
    if (epc > 0 && epc < E) rc = epc;
    else if (ppc > 0) rc = ppc * E;
    else {
      const int target = image_lds_target(t.NT, all_tiles, cus);
      rc = 8 * E;
      while (rc > E && image_lds_bytes(rc, E, s.W, rows, gate, mot) > target) rc /= 2;
      while (rc > 1 && image_lds_bytes(rc, E, s.W, rows, gate, mot) > target) --rc;
      // part of a ping: a whole number of quarter pings where possible (measured
      // faster than the largest fitting count on both the 2D and 3D workloads)
      if (rc < E && E >= 4 && rc >= E / 4) rc = rc / (E / 4) * (E / 4);
    }
    // the geometry build keeps its list of partially gated records (one int
    // each) in the window area, which must hold at least one ping's list
    rc = std::max(rc, (E + 4 * (s.W + 1) - 1) / (4 * (s.W + 1)));
    if (image_lds_bytes(rc, E, s.W, rows, gate, mot) > kLdsMax - 1024)
      return fail(SAS_BP_EUNSUPPORTED, "swath %d: %d records x %d samples exceed LDS", i, rc, s.W);
    s.RC = rc;
    const int cap = (int)std::min<long long>(32, 4ll * rc * (s.W + 1) / E);   // pings whose list fits
    if (cp > cap) {
      if (ppc > 0) return fail(SAS_BP_EUNSUPPORTED, "swath %d: %d pings per chunk need a larger image chunk", i, cp);
      cp = cap;
      s.CP = cp;
    }
    // pings whose FP64 geometry is built at once: enough (ping, element)
    // records to keep every thread of the workgroup busy, a multiple of the
    // adjoint chunk, and a partial-record list that fits the window area of
    // both kernels
    int sc = std::max(1, std::min(32, 1024 / E));
    sc = std::min(sc, cap);
    sc = std::max(cp, sc / cp * cp);
    s.SC = sc;
    out->push_back(s);
  }
  *n_tiles = tiles;
  return SAS_BP_OK;
}

Layout make_layout(int n_swaths, int n_tiles, size_t n_partials, size_t geo_stride, int geo_slots,
                   size_t n_track_pings) {
  Layout L{};
  size_t o = 0;
  L.swaths = o;     o = align_up(o + sizeof(SwathDev) * n_swaths);
  L.prange = o;     o = align_up(o + sizeof(PingRange) * n_tiles);
  L.order = o;      o = align_up(o + sizeof(int) * n_tiles);
  L.counters = o;   o = align_up(o + sizeof(unsigned) * kCounterWords);
  L.bucket = o;     o = align_up(o + sizeof(unsigned) * kBuckets);
  L.tile_swath = o; o = align_up(o + sizeof(int) * n_tiles);
  L.scratch = o;    o = align_up(o + sizeof(double) * (kSharpScratch + 16));
  L.drc = o;        o = align_up(o + drc_work_bytes());
  L.tstats = o;     o = align_up(o + sizeof(float4) * n_track_pings);
  L.geo = o;        o = align_up(o + geo_stride * (size_t)geo_slots);
  L.geo_stride = geo_stride;
  L.geo_slots = geo_slots;
  L.n_partials = n_partials;
  L.total = o;
  return L;
}

// Adjoint partials: one record per (tile, ping, element) of the tile's ping range.
size_t adjoint_partials(const std::vector<SwathPlan>& sw) {
  size_t n = 0;
  for (const auto& s : sw) n += (size_t)s.ntiles * s.d.n_ping * s.d.n_elem;
  return n;
}

SwathDev make_dev(const SwathPlan& s) {
  SwathDev v;
  std::memset(&v, 0, sizeof v);
  v.P = s.d.n_ping;
  v.E = s.d.n_elem;
  v.Ns = s.d.n_sample;
  v.dtype = s.d.echo_dtype;
  v.interp = s.d.interp;
  v.motion = s.d.motion;
  v.track_n = s.d.motion == SAS_BP_MOTION_TABLE ? s.d.track_n : 0;
  v.track_h = s.d.motion == SAS_BP_MOTION_TABLE ? s.d.track_dt : 0.0;
  v.refract = s.d.refract;
  v.no_cull = s.no_cull;
  v.c_sed = s.d.refract ? s.d.c_sediment : 0.0;
  v.z_int = s.d.refract ? s.d.z_interface : 0.0;
  v.nx = (int)s.d.n[0];
  v.ny = (int)s.d.n[1];
  v.nz = (int)s.d.n[2];
  v.ntx = s.ntx;
  v.nty = s.nty;
  v.ntz = s.ntz;
  v.tile0 = s.tile0;
  v.W = s.W;
  v.CP = s.CP;
  v.RC = s.RC;
  v.SC = s.SC;
  for (int a = 0; a < 3; ++a) {
    v.o[a] = s.d.origin[a];
    v.d[a] = (a == 2 && s.d.n[2] == 1 && !(s.d.spacing[2] > 0.0)) ? 1.0 : s.d.spacing[a];
  }
  v.fc = s.d.f_c;
  v.fs = s.d.f_s;
  v.t0 = s.d.t0;
  v.tan_g = s.d.gate_half_angle > 0.0 ? std::tan(s.d.gate_half_angle) : 0.0;
  v.sin_g = s.d.gate_half_angle > 0.0 ? std::sin(s.d.gate_half_angle) : 0.0;
  v.c_min = s.c_min;
  v.half_diag = s.half_diag;
  return v;
}

int check_io(const sas_bp_plan_s* p, const sas_bp_swath_io* io, int n) {
  if (!io) return fail(SAS_BP_EINVAL, "io is NULL");
  if (n != p->n_swaths) return fail(SAS_BP_EINVAL, "plan has %d swaths, got %d", p->n_swaths, n);
  for (int i = 0; i < n; ++i) {
    const auto& s = p->sw[i];
    if (!io[i].echo || !io[i].tx_pos || !io[i].rx_pos || !io[i].c || !io[i].image)
      return fail(SAS_BP_EINVAL, "swath %d: NULL pointer", i);
    if (((uintptr_t)io[i].echo & 15u) != 0) return fail(SAS_BP_EINVAL, "swath %d: echo not 16-byte aligned", i);
    if (((uintptr_t)io[i].image & 7u) != 0) return fail(SAS_BP_EINVAL, "swath %d: image not 8-byte aligned", i);
    if (((uintptr_t)io[i].tx_pos & 7u) || ((uintptr_t)io[i].rx_pos & 7u) || ((uintptr_t)io[i].c & 7u))
      return fail(SAS_BP_EINVAL, "swath %d: navigation not 8-byte aligned", i);
    if (s.d.echo_dtype != SAS_BP_ECHO_C64 && !io[i].echo_scale)
      return fail(SAS_BP_EINVAL, "swath %d: echo_scale required for 16-bit echoes", i);
    if (s.d.motion == SAS_BP_MOTION_VELOCITY && (!io[i].rx_vel || ((uintptr_t)io[i].rx_vel & 7u)))
      return fail(SAS_BP_EINVAL, "swath %d: continuous motion needs an 8-byte aligned rx_vel", i);
    if (s.d.motion == SAS_BP_MOTION_TABLE && (!io[i].rx_track || ((uintptr_t)io[i].rx_track & 7u)))
      return fail(SAS_BP_EINVAL, "swath %d: a position table needs an 8-byte aligned rx_track", i);
  }
  return SAS_BP_OK;
}

// Copy the per-swath descriptors (with the caller's pointers) to the slab if
// they changed since the last call. The pinned staging buffer is reused only
// after the previous copy has completed.
int upload(sas_bp_plan_s* p, const std::vector<SwathDev>& v, hipStream_t st) {
  if (v.size() == p->last_sw.size() && std::memcmp(v.data(), p->last_sw.data(), v.size() * sizeof(SwathDev)) == 0)
    return SAS_BP_OK;
  if (p->upload_pending) HIP_TRY(hipEventSynchronize(p->upload_done));
  std::memcpy(p->host_sw, v.data(), v.size() * sizeof(SwathDev));
  HIP_TRY(hipMemcpyAsync(p->ws.swaths, p->host_sw, v.size() * sizeof(SwathDev), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(p->upload_done, st));
  p->upload_pending = true;
  p->last_sw = v;
  return SAS_BP_OK;
}

// Event pair for the next timed launch (created on first use, then reused).
int timing_pair(sas_bp_plan_s* p, hipEvent_t* a, hipEvent_t* b) {
  while (p->events.size() < 2 * (p->n_timed + 1)) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreate(&e));
    p->events.push_back(e);
  }
  *a = p->events[2 * p->n_timed];
  *b = p->events[2 * p->n_timed + 1];
  return SAS_BP_OK;
}

int enqueue_image(sas_bp_plan_s* p, hipStream_t st) {
  HIP_TRY(launch_init(p->ws, st));
  if (p->motion == SAS_BP_MOTION_TABLE)
    for (int i = 0; i < p->n_swaths; ++i) HIP_TRY(launch_track_stats(p->ws, i, p->sw[i].d.n_ping, st));
  HIP_TRY(launch_cull(p->ws, p->n_tiles, p->tiling.TX, p->tiling.TY, p->tiling.TZ, p->bucket_shift, st));
  HIP_TRY(launch_order(p->ws, p->n_tiles, p->bucket_shift, st));
  hipEvent_t a = nullptr, b = nullptr;
  if (p->timing) {
    int rc = timing_pair(p, &a, &b);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(a, st));
  }
  HIP_TRY(launch_image(p->image_fn, p->ws, p->n_tiles, p->grid, p->tiling.NT, p->image_launch_lds, st));
  if (p->timing) {
    HIP_TRY(hipEventRecord(b, st));
    ++p->n_timed;
  }
  return SAS_BP_OK;
}

int capture_graph(sas_bp_plan_s* p) {
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_image(p, p->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
  if (rc != SAS_BP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(SAS_BP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(SAS_BP_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  p->graph = g;
  p->graph_exec = ex;
  return SAS_BP_OK;
}

void release(sas_bp_plan_s* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->upload_done) {
    (void)hipEventSynchronize(p->upload_done);
    (void)hipEventDestroy(p->upload_done);
  }
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  if (p->host_sw) (void)hipHostFree(p->host_sw);
  if (p->adj_buf) (void)hipFree(p->adj_buf);
  if (p->tvg_buf) (void)hipFree(p->tvg_buf);
  if (p->whiten_buf) (void)hipFree(p->whiten_buf);
  for (void* f : p->fft_plans) destroy_fft_plan(f);
  destroy_fft_plan(p->rc.batch);
  destroy_fft_plan(p->rc.single);
  if (p->rc.buf) (void)hipFree(p->rc.buf);
  if (p->rc.small) (void)hipFree(p->rc.small);
  if (p->tde_copied) {
    (void)hipEventSynchronize(p->tde_copied);
    (void)hipEventDestroy(p->tde_copied);
  }
  if (p->tde_pairs) (void)hipFree(p->tde_pairs);
  if (p->tde_pairs_host) (void)hipHostFree(p->tde_pairs_host);
  if (p->slab) (void)hipFree(p->slab);
  (void)hipSetDevice(cur);
  delete p;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int plan_sizes(const sas_bp_swath_desc* desc, int n, const sas_bp_options* o, Tiling* t,
               std::vector<SwathPlan>* sw, int* n_tiles, Layout* lay) {
  if (!desc) return fail(SAS_BP_EINVAL, "desc is NULL");
  if (n < 1 || n > 4096) return fail(SAS_BP_EINVAL, "n_swaths must be in [1, 4096]");
  if (o && (o->tune_mode < SAS_BP_TUNE_DEFAULT || o->tune_mode > SAS_BP_TUNE_SEARCH))
    return fail(SAS_BP_EINVAL, "tune_mode must be DEFAULT, CACHED or SEARCH");
  if (o && o->no_cull != 0 && o->no_cull != 1) return fail(SAS_BP_EINVAL, "no_cull must be 0 or 1");
  for (int i = 0; i < n; ++i) {
    int rc = validate(&desc[i], i);
    if (rc) return rc;
  }
  int rc = choose_tiling(desc, n, o, t);
  if (rc) return rc;
  rc = build_swaths(desc, n, o, *t, sw, n_tiles);
  if (rc) return rc;
  // geometry scratch: one region per resident workgroup, as many as the
  // smaller of the two kernels' LDS footprints lets a CU hold
  bool gate_any = false;
  for (const auto& s : *sw) gate_any |= s.d.gate_half_angle > 0.0;
  const int rows = t->TY * t->TZ;
  size_t stride = 0;
  int lds = 0;
  for (const auto& s : *sw) {
    stride = std::max(stride, (size_t)geo_layout(s.SC, s.d.n_elem, rows, gate_any, s.d.motion != 0).bytes);
    lds = std::max(lds, std::min(image_lds_bytes(s.RC, s.d.n_elem, s.W, rows, gate_any, s.d.motion != 0),
                                 adjoint_lds_bytes(s.CP, s.d.n_elem, s.W, rows, gate_any, t->NT)));
  }
  const int per_cu = std::max(1, std::min(8, kLdsMax / std::max(1, lds)));
  const int slots = (int)std::min<long long>(*n_tiles, (long long)kMaxCUs * per_cu);
  size_t track_pings = 0;
  for (auto& s : *sw) {
    s.tstats_off = track_pings;
    if (s.d.motion == SAS_BP_MOTION_TABLE) track_pings += (size_t)s.d.n_ping;
  }
  *lay = make_layout(n, *n_tiles, adjoint_partials(*sw), stride, slots, track_pings);
  return SAS_BP_OK;
}

}  // namespace

// Tuning cache, keyed by shape class: a process-wide map, and optionally a
// JSON file shared between processes.
namespace {

std::mutex g_tune_mutex;
std::map<std::string, sas_bp_options> g_tune_cache;

int log2_bucket(long long v) {
  int b = 0;
  while (v > 1) { v >>= 1; ++b; }
  return b;
}

// The shape class of these swaths on `device` (see sas_bp_tune_mode), from the
// automatic tiling's window lengths.
int shape_class(const sas_bp_swath_desc* desc, int n, int device, std::string* key) {
  Tiling t;
  std::vector<SwathPlan> sw;
  int n_tiles = 0;
  Layout lay;
  int rc = plan_sizes(desc, n, nullptr, &t, &sw, &n_tiles, &lay);
  if (rc) return rc;
  bool any3d = false, gate = false;
  int E = 0, W = 0;
  long long pix = 0;
  for (const auto& s : sw) {
    any3d |= s.d.n[2] > 1;
    gate |= s.d.gate_half_angle > 0.0;
    E = std::max(E, s.d.n_elem);
    W = std::max(W, s.W);
    pix += s.d.n[0] * s.d.n[1] * s.d.n[2];
  }
  std::string arch = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  } else {
    (void)hipGetLastError();
  }
  static const char* kDtype[] = {"c64", "f16", "bf16"};
  char buf[256];
  snprintf(buf, sizeof buf, "%s|%s|%s|interp%d|motion%d|refract%d|%s|e%d|w%d|p%d", arch.c_str(),
           any3d ? "3d" : "2d", kDtype[sw[0].d.echo_dtype], sw[0].d.interp, sw[0].d.motion, sw[0].d.refract,
           gate ? "gate" : "nogate", log2_bucket(E), log2_bucket(W), log2_bucket(pix));
  *key = buf;
  return SAS_BP_OK;
}

// Fields of a tiling stored in the cache.
const char* kTuneFields[] = {"tile_x", "tile_y", "tile_z", "threads", "pings_per_chunk", "elems_per_chunk"};

int32_t* tune_field(sas_bp_options* o, int i) {
  int32_t* f[] = {&o->tile_x, &o->tile_y, &o->tile_z, &o->threads, &o->pings_per_chunk, &o->elems_per_chunk};
  return f[i];
}

struct TuneEntry {
  std::string key;
  sas_bp_options opt;
  double ms;
};

// Entries of a cache file written by write_tune_file: one object per entry,
// {"class": "...", "tile_x": 64, ..., "ms": 21.9}. Anything unreadable is skipped.
std::vector<TuneEntry> read_tune_file(const char* path) {
  std::vector<TuneEntry> out;
  FILE* f = fopen(path, "rb");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 24)) text.append(buf, got);
  fclose(f);
  size_t pos = 0;
  const std::string tag = "\"class\"";
  while ((pos = text.find(tag, pos)) != std::string::npos) {
    const size_t end = text.find('}', pos);
    if (end == std::string::npos) break;
    const std::string obj = text.substr(pos, end - pos);
    pos = end;
    const size_t colon0 = obj.find(':');
    if (colon0 == std::string::npos) continue;
    const size_t q0 = obj.find('"', colon0 + 1);
    if (q0 == std::string::npos) continue;
    const size_t q1 = obj.find('"', q0 + 1);
    if (q1 == std::string::npos) continue;
    TuneEntry e;
    e.key = obj.substr(q0 + 1, q1 - q0 - 1);
    std::memset(&e.opt, 0, sizeof e.opt);
    e.ms = 0.0;
    bool ok = true;
    for (int i = 0; i < 6 && ok; ++i) {
      const std::string k = std::string("\"") + kTuneFields[i] + "\"";
      const size_t at = obj.find(k);
      if (at == std::string::npos) { ok = false; break; }
      const size_t colon = obj.find(':', at + k.size());
      if (colon == std::string::npos) { ok = false; break; }
      char* stop = nullptr;
      const long v = strtol(obj.c_str() + colon + 1, &stop, 10);
      if (stop == obj.c_str() + colon + 1 || v < 0 || v > 1 << 20) { ok = false; break; }
      *tune_field(&e.opt, i) = (int32_t)v;
    }
    const size_t at = obj.find("\"ms\"");
    if (at != std::string::npos) {
      const size_t colon = obj.find(':', at);
      if (colon != std::string::npos) e.ms = strtod(obj.c_str() + colon + 1, nullptr);
    }
    if (ok) out.push_back(e);
  }
  return out;
}

bool write_tune_file(const char* path, const std::vector<TuneEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  fprintf(f, "{\"format\": \"sas_bp tuning cache\", \"version\": 1, \"entries\": [\n");
  for (size_t i = 0; i < entries.size(); ++i) {
    const TuneEntry& e = entries[i];
    fprintf(f, "  {\"class\": \"%s\"", e.key.c_str());
    for (int j = 0; j < 6; ++j)
      fprintf(f, ", \"%s\": %d", kTuneFields[j], *tune_field(const_cast<sas_bp_options*>(&e.opt), j));
    fprintf(f, ", \"ms\": %.6g}%s\n", e.ms, i + 1 < entries.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  const bool ok = fflush(f) == 0;
  fclose(f);
  return ok && rename(tmp.c_str(), path) == 0;
}

// Stored tiling for a class: the process cache, then the file.
bool tune_lookup(const std::string& key, const char* path, sas_bp_options* out) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  auto it = g_tune_cache.find(key);
  if (it != g_tune_cache.end()) {
    *out = it->second;
    return true;
  }
  if (!path) return false;
  for (const TuneEntry& e : read_tune_file(path)) {
    if (e.key == key) {
      g_tune_cache[key] = e.opt;
      *out = e.opt;
      return true;
    }
  }
  return false;
}

void tune_store(const std::string& key, const sas_bp_options& opt, double ms, const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  sas_bp_options o;
  std::memset(&o, 0, sizeof o);
  for (int i = 0; i < 6; ++i) *tune_field(&o, i) = *tune_field(const_cast<sas_bp_options*>(&opt), i);
  g_tune_cache[key] = o;
  if (!path) return;
  std::vector<TuneEntry> entries = read_tune_file(path);
  bool found = false;
  for (TuneEntry& e : entries) {
    if (e.key == key) {
      e.opt = o;
      e.ms = ms;
      found = true;
    }
  }
  if (!found) entries.push_back(TuneEntry{key, o, ms});
  (void)write_tune_file(path, entries);
}

// The options a plan is made with: for CACHED and SEARCH, the stored tiling of
// the shape class replaces the tile and chunk fields (when one is stored).
int resolve_options(const sas_bp_swath_desc* desc, int n, const sas_bp_options* o, sas_bp_options* out,
                    bool* used) {
  *used = false;
  if (!o) return SAS_BP_OK;
  *out = *o;
  if (o->tune_mode != SAS_BP_TUNE_CACHED && o->tune_mode != SAS_BP_TUNE_SEARCH) return SAS_BP_OK;
  std::string key;
  int rc = shape_class(desc, n, o->device, &key);
  if (rc) return rc;
  sas_bp_options stored;
  if (tune_lookup(key, o->tune_cache, &stored)) {
    for (int i = 0; i < 6; ++i) *tune_field(out, i) = *tune_field(&stored, i);
    *used = true;
  } else {
    for (int i = 0; i < 6; ++i) *tune_field(out, i) = 0;   // the automatic choice
  }
  return SAS_BP_OK;
}

}  // namespace

namespace {

int check_dpc_desc(const sas_bp_dpc_desc* d) {
  if (!d) return fail(SAS_BP_EINVAL, "desc is NULL");
  if (d->n_ping < 2 || d->n_ping > 65536) return fail(SAS_BP_EINVAL, "n_ping must lie in [2, 65536]");
  if (d->n_window < 1) return fail(SAS_BP_EINVAL, "n_window must be >= 1");
  if (d->n_pairs < 1 || d->n_pairs > 256) return fail(SAS_BP_EINVAL, "n_pairs must lie in [1, 256]");
  if (d->n_elem < 1 || d->n_elem > kMaxElem) return fail(SAS_BP_EINVAL, "n_elem must lie in [1, %d]", kMaxElem);
  if (!(d->c > 0.0) || !finite(d->c)) return fail(SAS_BP_EINVAL, "c must be > 0");
  for (int a = 0; a < 3; ++a)
    if (!finite(d->p0[a]) || !finite(d->lever_tx[a])) return fail(SAS_BP_EINVAL, "p0 and lever_tx must be finite");
  return SAS_BP_OK;
}

// Dense Cholesky solve of A x = b (A symmetric positive definite, n x n, row
// major, overwritten by its factor). Returns false if A is not positive definite.
bool cholesky_solve(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int j = 0; j < n; ++j) {
    double* rj = &A[(size_t)j * n];
    double djj = rj[j];
    for (int k = 0; k < j; ++k) djj -= rj[k] * rj[k];
    if (!(djj > 0.0)) return false;
    djj = std::sqrt(djj);
    rj[j] = djj;
    const double inv = 1.0 / djj;
    for (int i = j + 1; i < n; ++i) {
      double* ri = &A[(size_t)i * n];
      double v = ri[j];
      for (int k = 0; k < j; ++k) v -= ri[k] * rj[k];
      ri[j] = v * inv;
    }
  }
  for (int i = 0; i < n; ++i) {   // L y = b
    const double* ri = &A[(size_t)i * n];
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= ri[k] * b[k];
    b[i] = v / ri[i];
  }
  for (int i = n - 1; i >= 0; --i) {   // L^T x = y
    double v = b[i];
    for (int k = i + 1; k < n; ++k) v -= A[(size_t)k * n + i] * b[k];
    b[i] = v / A[(size_t)i * n + i];
  }
  return true;
}

double huber(double a) {
  a = std::fabs(a);
  return a <= 1.0 ? 0.5 * a * a : a - 0.5;
}

}  // namespace

extern "C" {

int sas_bp_dpc_footprints(const sas_bp_dpc_desc* d, const double* vel_nominal, const double* dt,
                          const double* lever_rx, const int32_t* pairs, const double* t_ref, double z_floor,
                          double look, double* out) {
  int rc = check_dpc_desc(d);
  if (rc) return rc;
  if (!vel_nominal || !dt || !lever_rx || !pairs || !t_ref || !out) return fail(SAS_BP_EINVAL, "NULL argument");
  if (look != 1.0 && look != -1.0) return fail(SAS_BP_EINVAL, "look must be +1 or -1");
  const int P = d->n_ping, K = d->n_window, J = d->n_pairs;
  double pc_off[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < J; ++j) {
    const int e = pairs[2 * j];
    if (e < 0 || e >= d->n_elem) return fail(SAS_BP_EINVAL, "pair %d names an element outside [0, %d)", j, d->n_elem);
    for (int a = 0; a < 3; ++a) pc_off[a] += lever_rx[3 * e + a];
  }
  for (int a = 0; a < 3; ++a) pc_off[a] = 0.5 * (d->lever_tx[a] + pc_off[a] / J);
  double pos[3] = {d->p0[0], d->p0[1], d->p0[2]};
  for (int i = 0; i < P - 1; ++i) {
    const double pc[3] = {pos[0] + pc_off[0], pos[1] + pc_off[1], pos[2] + pc_off[2]};
    for (int k = 0; k < K; ++k) {
      const double slant = 0.5 * d->c * t_ref[k], dz = z_floor - pc[2];
      const double ground = std::sqrt(std::max(slant * slant - dz * dz, 0.0));
      double* o = out + ((size_t)i * K + k) * 3;
      o[0] = pc[0];
      o[1] = pc[1] + look * ground;
      o[2] = z_floor;
    }
    for (int a = 0; a < 3; ++a) pos[a] += vel_nominal[3 * i + a] * dt[i];
  }
  return SAS_BP_OK;
}

int sas_bp_dpc_residual(const sas_bp_dpc_desc* d, const double* vel, const double* dt, const double* lever_rx,
                        const int32_t* pairs, const double* t_ref, const double* footprint, const double* delay,
                        double* pos_out, double* rows, void* stream) {
  int rc = check_dpc_desc(d);
  if (rc) return rc;
  if (!vel || !dt || !lever_rx || !pairs || !t_ref || !footprint || !delay || !pos_out || !rows)
    return fail(SAS_BP_EINVAL, "NULL argument");
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_dpc_positions(d->n_ping, vel, dt, d->p0, pos_out, st));
  HIP_TRY(launch_dpc_residual(d->n_ping, d->n_window, d->n_pairs, pos_out, vel, dt, d->lever_tx, lever_rx, pairs,
                              t_ref, footprint, delay, d->c, rows, st));
  return SAS_BP_OK;
}

int sas_bp_dpc_fine_delay(const float* tde, const double* rows, int64_t n, double f_c, double* out, void* stream) {
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (!tde || !rows || !out) return fail(SAS_BP_EINVAL, "NULL pointer");
  if (n < 1 || n > (1ll << 31)) return fail(SAS_BP_EINVAL, "n must be in [1, 2^31]");
  if (!(f_c > 0.0) || !std::isfinite(f_c)) return fail(SAS_BP_EINVAL, "f_c must be > 0");
  if (((uintptr_t)tde & 15u) || ((uintptr_t)rows & 7u) || ((uintptr_t)out & 7u))
    return fail(SAS_BP_EINVAL, "tde must be 16-byte aligned, rows and out 8-byte aligned");
  HIP_TRY(launch_dpc_fine_delay((long long)n, tde, rows, f_c, out, reinterpret_cast<hipStream_t>(stream)));
  return SAS_BP_OK;
}

int sas_bp_dpc_solve(const sas_bp_dpc_desc* d, const double* vx, const double* dt, const double* lever_rx,
                     const int32_t* pairs, const double* t_ref, const double* footprint, const double* delay,
                     const double* weight, const double* z_dvl, double* vyz, double* loss_out, int device) {
  int rc = check_dpc_desc(d);
  if (rc) return rc;
  if (!vx || !dt || !lever_rx || !pairs || !t_ref || !footprint || !delay || !weight || !z_dvl || !vyz)
    return fail(SAS_BP_EINVAL, "NULL argument");
  if (d->n_ping > 4096) return fail(SAS_BP_EUNSUPPORTED, "the dense normal equations are built for <= 4096 pings");
  if (!(d->sigma > 0.0) || !(d->lambda_smooth >= 0.0) || !(d->lambda_dvl >= 0.0))
    return fail(SAS_BP_EINVAL, "sigma must be > 0 and the regularisation weights >= 0");
  if (d->max_iter < 1 || d->max_iter > 1000) return fail(SAS_BP_EINVAL, "max_iter must lie in [1, 1000]");
  for (int j = 0; j < 2 * d->n_pairs; ++j)
    if (pairs[j] < 0 || pairs[j] >= d->n_elem) return fail(SAS_BP_EINVAL, "a pair names an element outside [0, %d)",
                                                          d->n_elem);
  const int P = d->n_ping, K = d->n_window, J = d->n_pairs, n = 2 * P;
  const size_t R = (size_t)(P - 1) * K;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (hipSetDevice(device) != hipSuccess) return fail(SAS_BP_EINVAL, "device %d not available", device);
  (void)hipGetLastError();
  // device copies of the fixed inputs; velocities, positions and rows per pass
  const size_t b_vel = sizeof(double) * 3 * P, b_dt = sizeof(double) * (P - 1), b_lr = sizeof(double) * 3 * d->n_elem;
  const size_t b_pairs = sizeof(int) * 2 * J, b_t = sizeof(double) * K, b_ps = sizeof(double) * 3 * R;
  const size_t b_del = sizeof(double) * R, b_rows = sizeof(double) * 7 * R;
  const size_t offs[] = {0, b_vel, b_dt, b_lr, b_pairs, b_t, b_ps, b_del, b_vel, b_rows};
  size_t total = 0, at[10];
  for (int q = 0; q < 10; ++q) {
    total = align_up(total + offs[q]);
    at[q] = total;
  }
  unsigned char* buf = nullptr;
  if (hipMalloc(&buf, total + kAlign) != hipSuccess) {
    (void)hipSetDevice(cur);
    return fail(SAS_BP_ENOMEM, "motion-estimate workspace of %zu bytes could not be allocated", total);
  }
  double* g_vel = reinterpret_cast<double*>(buf + at[0]);
  double* g_dt = reinterpret_cast<double*>(buf + at[1]);
  double* g_lr = reinterpret_cast<double*>(buf + at[2]);
  int* g_pairs = reinterpret_cast<int*>(buf + at[3]);
  double* g_t = reinterpret_cast<double*>(buf + at[4]);
  double* g_ps = reinterpret_cast<double*>(buf + at[5]);
  double* g_del = reinterpret_cast<double*>(buf + at[6]);
  double* g_pos = reinterpret_cast<double*>(buf + at[7]);
  double* g_rows = reinterpret_cast<double*>(buf + at[8]);
  int status = SAS_BP_OK;
  std::vector<double> vel(3 * P), rows(7 * R), x(n), N((size_t)n * n), grad(n);
  for (int i = 0; i < P; ++i) {
    x[2 * i] = vyz[2 * i];
    x[2 * i + 1] = vyz[2 * i + 1];
  }
  auto evaluate = [&](const std::vector<double>& xv, double* loss) -> bool {
    for (int i = 0; i < P; ++i) {
      vel[3 * i] = vx[i];
      vel[3 * i + 1] = xv[2 * i];
      vel[3 * i + 2] = xv[2 * i + 1];
    }
    if (hipMemcpy(g_vel, vel.data(), b_vel, hipMemcpyHostToDevice) != hipSuccess) return false;
    if (launch_dpc_positions(P, g_vel, g_dt, d->p0, g_pos, nullptr) != hipSuccess) return false;
    if (launch_dpc_residual(P, K, J, g_pos, g_vel, g_dt, d->lever_tx, g_lr, g_pairs, g_t, g_ps, g_del, d->c, g_rows,
                            nullptr) != hipSuccess)
      return false;
    if (hipMemcpy(rows.data(), g_rows, b_rows, hipMemcpyDeviceToHost) != hipSuccess) return false;
    double L = 0.0;
    for (size_t r = 0; r < R; ++r) {
      const double a = rows[7 * r] / d->sigma;
      L += weight[r] * (d->robust ? huber(a) : a * a);
    }
    for (int i = 1; i + 1 < P; ++i)
      for (int c = 0; c < 2; ++c) {
        const double sv = xv[2 * (i - 1) + c] - 2.0 * xv[2 * i + c] + xv[2 * (i + 1) + c];
        L += d->lambda_smooth * sv * sv;
      }
    double z = d->p0[2];
    for (int i = 0; i < P; ++i) {
      const double dv = z - z_dvl[i];
      L += d->lambda_dvl * dv * dv;
      if (i + 1 < P) z += xv[2 * i + 1] * dt[i];
    }
    *loss = L;
    return true;
  };
  do {
    if (hipMemcpy(g_dt, dt, b_dt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g_lr, lever_rx, b_lr, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g_pairs, pairs, b_pairs, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g_t, t_ref, b_t, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g_ps, footprint, b_ps, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g_del, delay, b_del, hipMemcpyHostToDevice) != hipSuccess) {
      status = fail(SAS_BP_EDEVICE, "upload of the motion-estimate inputs failed");
      break;
    }
    double cur_loss = 0.0;
    if (!evaluate(x, &cur_loss)) {
      status = fail(SAS_BP_EDEVICE, "residual pass failed");
      break;
    }
    double lam = 1e-3;
    std::vector<double> Saa(4 * (P - 1)), Sab(4 * (P - 1)), Sac(4 * (P - 1)), Sbb(4 * (P - 1)), Sbc(4 * (P - 1)),
        Scc(4 * (P - 1)), Ga(2 * (P - 1)), Gb(2 * (P - 1)), Gc(2 * (P - 1)), Taa(4 * P), Tga(2 * P);
    for (int it = 0; it < d->max_iter; ++it) {
      // weighted normal equations of the stacked residuals at x (rows hold the current pass)
      std::fill(Saa.begin(), Saa.end(), 0.0);
      std::fill(Sab.begin(), Sab.end(), 0.0);
      std::fill(Sac.begin(), Sac.end(), 0.0);
      std::fill(Sbb.begin(), Sbb.end(), 0.0);
      std::fill(Sbc.begin(), Sbc.end(), 0.0);
      std::fill(Scc.begin(), Scc.end(), 0.0);
      std::fill(Ga.begin(), Ga.end(), 0.0);
      std::fill(Gb.begin(), Gb.end(), 0.0);
      std::fill(Gc.begin(), Gc.end(), 0.0);
      for (int i = 0; i < P - 1; ++i)
        for (int k = 0; k < K; ++k) {
          const double* o = &rows[7 * ((size_t)i * K + k)];
          const double a = o[0] / d->sigma;
          double om = weight[(size_t)i * K + k];
          if (d->robust) om *= 0.5 * (std::fabs(a) <= 1.0 ? 1.0 : 1.0 / std::fabs(a));
          const double f = om / (d->sigma * d->sigma), gr = om * a / d->sigma;
          const double va[2] = {o[1], o[2]}, vb[2] = {o[3], o[4]}, vc[2] = {o[5], o[6]};
          for (int p = 0; p < 2; ++p) {
            for (int q = 0; q < 2; ++q) {
              Saa[4 * i + 2 * p + q] += f * va[p] * va[q];
              Sab[4 * i + 2 * p + q] += f * va[p] * vb[q];
              Sac[4 * i + 2 * p + q] += f * va[p] * vc[q];
              Sbb[4 * i + 2 * p + q] += f * vb[p] * vb[q];
              Sbc[4 * i + 2 * p + q] += f * vb[p] * vc[q];
              Scc[4 * i + 2 * p + q] += f * vc[p] * vc[q];
            }
            Ga[2 * i + p] += gr * va[p];
            Gb[2 * i + p] += gr * vb[p];
            Gc[2 * i + p] += gr * vc[p];
          }
        }
      // suffix sums over pairs i > m: Taa[m] = sum Saa[i], Tga[m] = sum Ga[i]
      std::fill(Taa.begin(), Taa.end(), 0.0);
      std::fill(Tga.begin(), Tga.end(), 0.0);
      for (int m = P - 2; m >= 0; --m)
        for (int q = 0; q < 4; ++q) Taa[4 * m + q] = Taa[4 * (m + 1) + q] + (m + 1 < P - 1 ? Saa[4 * (m + 1) + q] : 0.0);
      for (int m = P - 2; m >= 0; --m)
        for (int q = 0; q < 2; ++q) Tga[2 * m + q] = Tga[2 * (m + 1) + q] + (m + 1 < P - 1 ? Ga[2 * (m + 1) + q] : 0.0);
      std::fill(N.begin(), N.end(), 0.0);
      auto add = [&](int nb, int mb, int p, int q, double v) { N[(size_t)(2 * nb + p) * n + 2 * mb + q] += v; };
      for (int m = 0; m < P; ++m)
        for (int nb = 0; nb <= m; ++nb)
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
              double v = 0.0;
              if (m < P - 1 && nb < P - 1) v += dt[nb] * dt[m] * Taa[4 * m + 2 * p + q];   // pairs i > m
              if (nb < m && m < P - 1) v += dt[nb] * Sab[4 * m + 2 * p + q];                 // pair i = m
              if (m >= 1 && nb < m - 1) v += dt[nb] * Sac[4 * (m - 1) + 2 * p + q];          // pair i = m - 1
              if (m >= 1 && nb == m - 1) v += Sbc[4 * (m - 1) + 2 * p + q];
              if (nb == m) {
                if (m < P - 1) v += Sbb[4 * m + 2 * p + q];
                if (m >= 1) v += Scc[4 * (m - 1) + 2 * p + q];
              }
              add(nb, m, p, q, v);
            }
      for (int nb = 0; nb < P; ++nb)
        for (int p = 0; p < 2; ++p) {
          double v = 0.0;
          if (nb < P - 1) v += dt[nb] * Tga[2 * nb + p] + Gb[2 * nb + p];
          if (nb >= 1) v += Gc[2 * (nb - 1) + p];
          grad[2 * nb + p] = v;
        }
      // the DPC part was built on the upper block triangle: mirror it
      for (int m = 0; m < P; ++m)
        for (int nb = 0; nb < m; ++nb)
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) N[(size_t)(2 * m + q) * n + 2 * nb + p] = N[(size_t)(2 * nb + p) * n + 2 * m + q];
      // Eq. 6: lambda_1 (v[i-1] - 2 v[i] + v[i+1])^2 per component
      const double cf[3] = {1.0, -2.0, 1.0};
      for (int i = 1; i + 1 < P; ++i)
        for (int c = 0; c < 2; ++c) {
          const double sv = x[2 * (i - 1) + c] - 2.0 * x[2 * i + c] + x[2 * (i + 1) + c];
          for (int u = 0; u < 3; ++u) {
            grad[2 * (i - 1 + u) + c] += d->lambda_smooth * cf[u] * sv;
            for (int w = 0; w < 3; ++w) add(i - 1 + u, i - 1 + w, c, c, d->lambda_smooth * cf[u] * cf[w]);
          }
        }
      // Eq. 7: lambda_2 (z_i - z_DVL[i])^2, dz_i / dv_z[n] = dt_n for n < i
      {
        std::vector<double> dres(P), tail(P + 1, 0.0);
        double z = d->p0[2];
        for (int i = 0; i < P; ++i) {
          dres[i] = z - z_dvl[i];
          if (i + 1 < P) z += x[2 * i + 1] * dt[i];
        }
        for (int i = P - 1; i >= 0; --i) tail[i] = tail[i + 1] + dres[i];
        for (int nb = 0; nb < P - 1; ++nb) {
          grad[2 * nb + 1] += d->lambda_dvl * dt[nb] * tail[nb + 1];
          for (int m = 0; m < P - 1; ++m)
            add(nb, m, 1, 1, d->lambda_dvl * dt[nb] * dt[m] * (double)(P - 1 - std::max(nb, m)));
        }
      }
      bool improved = false;
      double snorm = 0.0, xnorm = 0.0;
      for (int tries = 0; tries < 10; ++tries) {
        std::vector<double> A(N), rhs(n);
        for (int q = 0; q < n; ++q) {
          A[(size_t)q * n + q] += lam * (N[(size_t)q * n + q] + 1e-12);
          rhs[q] = -grad[q];
        }
        if (!cholesky_solve(A, rhs, n)) {
          lam *= 4.0;
          continue;
        }
        std::vector<double> xt(n);
        snorm = 0.0;
        xnorm = 0.0;
        for (int q = 0; q < n; ++q) {
          xt[q] = x[q] + rhs[q];
          snorm += rhs[q] * rhs[q];
          xnorm += x[q] * x[q];
        }
        double tl = 0.0;
        if (!evaluate(xt, &tl)) {
          status = fail(SAS_BP_EDEVICE, "residual pass failed");
          break;
        }
        if (tl < cur_loss) {
          x = xt;
          cur_loss = tl;
          lam = std::max(lam / 3.0, 1e-12);
          improved = true;
          break;
        }
        lam *= 4.0;
      }
      if (status != SAS_BP_OK) break;
      if (!improved) break;
      if (std::sqrt(snorm) < 1e-12 * (1.0 + std::sqrt(xnorm))) break;
    }
    if (status != SAS_BP_OK) break;
    for (int q = 0; q < n; ++q) vyz[q] = x[q];
    if (loss_out) *loss_out = cur_loss;
  } while (false);
  (void)hipFree(buf);
  (void)hipSetDevice(cur);
  return status;
}

}  // extern "C"

extern "C" {

int sas_bp_abi_version(void) { return SAS_BP_ABI_VERSION; }

const char* sas_bp_error_string(int status) {
  switch (status) {
    case SAS_BP_OK: return "success";
    case SAS_BP_EINVAL: return "invalid argument";
    case SAS_BP_EUNSUPPORTED: return "unsupported configuration";
    case SAS_BP_ENOMEM: return "out of device memory or over the workspace limit";
    case SAS_BP_EDEVICE: return "HIP runtime error";
    case SAS_BP_ENAV: return "non-finite navigation or sound speed below c_min";
    case SAS_BP_ECONVERGE: return "a refracted leg's crossing did not converge within the step cap";
    default: return "unknown status";
  }
}

const char* sas_bp_last_error_detail(void) { return g_detail.c_str(); }

int sas_bp_workspace_size(const sas_bp_swath_desc* desc, int n_swaths, const sas_bp_options* options,
                          size_t* bytes) {
  if (!bytes) return fail(SAS_BP_EINVAL, "bytes is NULL");
  sas_bp_options ro;
  bool cached = false;
  int rc = resolve_options(desc, n_swaths, options, &ro, &cached);
  if (rc) return rc;
  if (options) options = &ro;
  Tiling t;
  std::vector<SwathPlan> sw;
  int n_tiles = 0;
  Layout lay;
  rc = plan_sizes(desc, n_swaths, options, &t, &sw, &n_tiles, &lay);
  if (rc) return rc;
  *bytes = lay.total;
  return SAS_BP_OK;
}

int sas_bp_plan(const sas_bp_swath_desc* desc, int n_swaths, const sas_bp_options* options, sas_bp_plan_t* out) {
  if (!out) return fail(SAS_BP_EINVAL, "out is NULL");
  *out = nullptr;
  sas_bp_options ro;
  bool cached = false;
  int rc = resolve_options(desc, n_swaths, options, &ro, &cached);
  if (rc) return rc;
  if (options) options = &ro;
  Tiling t;
  std::vector<SwathPlan> sw;
  int n_tiles = 0;
  Layout lay;
  rc = plan_sizes(desc, n_swaths, options, &t, &sw, &n_tiles, &lay);
  if (rc) return rc;
  if (options && options->workspace_limit && lay.total > options->workspace_limit)
    return fail(SAS_BP_ENOMEM, "workspace needs %zu bytes, limit is %zu", lay.total, options->workspace_limit);
  const int device = options ? options->device : 0;
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev <= 0) return fail(SAS_BP_EDEVICE, "no HIP device");
  if (device < 0 || device >= n_dev) return fail(SAS_BP_EINVAL, "device %d out of range", device);
  DeviceGuard guard(device);

  sas_bp_plan_s* p = new (std::nothrow) sas_bp_plan_s;
  if (!p) return fail(SAS_BP_ENOMEM, "host allocation failed");
  p->device = device;
  p->n_swaths = n_swaths;
  p->n_tiles = n_tiles;
  p->tiling = t;
  p->sw = sw;
  p->lay = lay;
  p->use_graph = options ? options->use_graph != 0 : true;
  p->tuned_from_cache = cached;
  p->dtype = sw[0].d.echo_dtype;
  p->interp = sw[0].d.interp;
  p->motion = sw[0].d.motion;
  p->refract = sw[0].d.refract;
  int max_pe = 1, max_lds = 0, max_adj_lds = 0;
  for (const auto& s : sw) {
    const bool gate = s.d.gate_half_angle > 0.0;
    p->gate_any |= gate;
    if (s.d.echo_dtype != p->dtype) {
      release(p);
      return fail(SAS_BP_EUNSUPPORTED, "all swaths of a plan must share one echo dtype");
    }
    if (s.d.interp != p->interp) {
      release(p);
      return fail(SAS_BP_EUNSUPPORTED, "all swaths of a plan must share one interpolator");
    }
    if (s.d.motion != p->motion) {
      release(p);
      return fail(SAS_BP_EUNSUPPORTED, "all swaths of a plan must share one motion model");
    }
    if (s.d.refract != p->refract) {
      release(p);
      return fail(SAS_BP_EUNSUPPORTED, "all swaths of a plan must share one propagation model");
    }
    max_pe = std::max(max_pe, s.d.n_ping * s.d.n_elem);
    p->max_p = std::max(p->max_p, s.d.n_ping);
  }
  for (const auto& s : sw) {
    max_lds = std::max(max_lds, image_lds_bytes(s.RC, s.d.n_elem, s.W, t.TY * t.TZ, p->gate_any, p->motion != 0));
    max_adj_lds = std::max(max_adj_lds, adjoint_lds_bytes(s.CP, s.d.n_elem, s.W, t.TY * t.TZ, p->gate_any, t.NT));
  }
  p->max_pe = max_pe;
  int shift = 0;
  while ((max_pe >> shift) >= kBuckets) ++shift;
  p->bucket_shift = shift;
  p->lds_bytes = max_lds;
  p->adj_lds_bytes = max_adj_lds;
  p->image_fn = p->refract ? refract_kernel_for(t.layout, p->gate_any, p->dtype)
                           : image_kernel_for(t.layout, p->gate_any, p->dtype,
                                              p->motion == SAS_BP_MOTION_TABLE ? 3 : p->motion ? 2 : p->interp);
  p->adjoint_fn = adjoint_kernel_for(t.layout, p->gate_any, p->dtype);
  p->reproject_fn = reproject_kernel_for(t.layout, p->gate_any);
  if (!p->image_fn || !p->adjoint_fn || !p->reproject_fn) {
    release(p);
    return fail(SAS_BP_EUNSUPPORTED, "no kernel for tiling %d", t.layout);
  }
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e == hipSuccess && (size_t)max_lds + 1024 > prop.sharedMemPerBlock) {
    release(p);
    return fail(SAS_BP_EUNSUPPORTED, "tiling needs %d bytes of LDS, the device allows %zu per workgroup", max_lds,
                (size_t)prop.sharedMemPerBlock);
  }
  p->adj_ok = e == hipSuccess && (size_t)max_adj_lds + 1024 <= prop.sharedMemPerBlock;
  // the refraction kernel reads the echo from global memory: no dynamic LDS,
  // so that its occupancy is set by its registers alone
  const int image_lds = p->refract ? 0 : max_lds;
  p->image_launch_lds = image_lds;
  if (e == hipSuccess) e = set_image_lds_limit(p->image_fn, image_lds);
  if (e == hipSuccess && p->adj_ok) e = set_adjoint_lds_limit(p->adjoint_fn, max_adj_lds);
  if (e == hipSuccess) e = set_reproject_lds_limit(p->reproject_fn, max_lds);   // same layout as the image
  int occ = 0, adj_occ = 1, rep_occ = 0;
  if (e == hipSuccess) e = image_occupancy(p->image_fn, t.NT, image_lds, &occ);
  if (e == hipSuccess && p->adj_ok) e = adjoint_occupancy(p->adjoint_fn, t.NT, max_adj_lds, &adj_occ);
  if (e == hipSuccess) e = reproject_occupancy(p->reproject_fn, t.NT, max_lds, &rep_occ);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release(p);
    return fail(SAS_BP_EDEVICE, "kernel setup failed: %s", hipGetErrorString(e));
  }
  if (occ < 1 || adj_occ < 1 || rep_occ < 1) {
    release(p);
    return fail(SAS_BP_EUNSUPPORTED, "tiling needs %d bytes of LDS; no workgroup fits", max_lds);
  }
  p->occ = occ;
  // the refraction kernel keeps its references in static LDS, not in the
  // geometry scratch: its resident workgroups are set by its occupancy alone
  p->grid = std::max(1, std::min(std::min(n_tiles, occ * prop.multiProcessorCount),
                                 p->refract ? n_tiles : lay.geo_slots));
  p->adj_grid = std::max(1, std::min(std::min(n_tiles, adj_occ * prop.multiProcessorCount), lay.geo_slots));
  p->rep_grid = std::max(1, std::min(std::min(n_tiles, rep_occ * prop.multiProcessorCount), lay.geo_slots));

  e = hipMalloc(&p->slab, lay.total);
  if (e != hipSuccess) {
    p->slab = nullptr;
    release(p);
    return fail(SAS_BP_ENOMEM, "hipMalloc(%zu) failed: %s", lay.total, hipGetErrorString(e));
  }
  p->ws.swaths = reinterpret_cast<SwathDev*>(p->slab + lay.swaths);
  p->ws.prange = reinterpret_cast<PingRange*>(p->slab + lay.prange);
  p->ws.order = reinterpret_cast<int*>(p->slab + lay.order);
  p->ws.counters = reinterpret_cast<unsigned*>(p->slab + lay.counters);
  p->ws.bucket = reinterpret_cast<unsigned*>(p->slab + lay.bucket);
  p->ws.tile_swath = reinterpret_cast<int*>(p->slab + lay.tile_swath);
  p->ws.partials = nullptr;
  p->ws.cpart = nullptr;
  p->ws.scratch64 = reinterpret_cast<double*>(p->slab + lay.scratch);
  p->ws.geo = p->slab + lay.geo;
  p->tstats = reinterpret_cast<float4*>(p->slab + lay.tstats);
  p->ws.geo_stride = (long long)lay.geo_stride;

  std::vector<int> tile_swath(n_tiles);
  for (int i = 0; i < n_swaths; ++i)
    for (int k = 0; k < sw[i].ntiles; ++k) tile_swath[sw[i].tile0 + k] = i;
  std::vector<unsigned> zeros(kCounterWords, 0u);
  e = hipMemcpy(p->ws.tile_swath, tile_swath.data(), sizeof(int) * n_tiles, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->ws.counters, zeros.data(), sizeof(unsigned) * kCounterWords, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&p->host_sw), sizeof(SwathDev) * n_swaths, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    release(p);
    return fail(SAS_BP_EDEVICE, "plan setup failed: %s", hipGetErrorString(e));
  }
  if (p->use_graph) {
    rc = capture_graph(p);
    if (rc) {
      release(p);
      return rc;
    }
  }
  *out = p;
  return SAS_BP_OK;
}

int sas_bp_image(sas_bp_plan_t p, const sas_bp_swath_io* io, int n_swaths, void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  int rc = check_io(p, io, n_swaths);
  if (rc) return rc;
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<SwathDev> v(n_swaths);
  for (int i = 0; i < n_swaths; ++i) {
    v[i] = make_dev(p->sw[i]);
    v[i].echo = io[i].echo;
    v[i].scale = io[i].echo_scale;
    v[i].tx = io[i].tx_pos;
    v[i].rx = io[i].rx_pos;
    v[i].vel = io[i].rx_vel;
    v[i].track = io[i].rx_track;
    v[i].tstats = p->tstats + p->sw[i].tstats_off;
    v[i].c = io[i].c;
    v[i].image = reinterpret_cast<float2*>(io[i].image);
  }
  rc = upload(p, v, st);
  if (rc) return rc;
  if (p->use_graph && !p->timing) {
    HIP_TRY(hipGraphLaunch(p->graph_exec, st));
    return SAS_BP_OK;
  }
  return enqueue_image(p, st);
}

int sas_bp_adjoint(sas_bp_plan_t p, const sas_bp_swath_io* io, const void* const* grad_image,
                   double* const* grad_tx, double* const* grad_rx, double* const* grad_c, int n_swaths,
                   void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  int rc = check_io(p, io, n_swaths);
  if (rc) return rc;
  if (!grad_image || !grad_tx || !grad_rx || !grad_c) return fail(SAS_BP_EINVAL, "gradient array is NULL");
  if (p->interp != SAS_BP_INTERP_LINEAR || p->motion || p->refract)
    return fail(SAS_BP_EUNSUPPORTED, "the adjoint is built for linear interpolation, stop-and-hop positions and "
                "straight paths only");
  if (!p->adj_ok)
    return fail(SAS_BP_EUNSUPPORTED, "the adjoint stages whole pings and needs %d bytes of LDS with this tiling; "
                "plan with a smaller tile", p->adj_lds_bytes);
  for (int i = 0; i < n_swaths; ++i) {
    if (!grad_image[i] || !grad_tx[i] || !grad_rx[i] || !grad_c[i])
      return fail(SAS_BP_EINVAL, "swath %d: NULL gradient pointer", i);
    if (((uintptr_t)grad_image[i] & 7u) || ((uintptr_t)grad_tx[i] & 7u) || ((uintptr_t)grad_rx[i] & 7u) ||
        ((uintptr_t)grad_c[i] & 7u))
      return fail(SAS_BP_EINVAL, "swath %d: gradient pointer not 8-byte aligned", i);
  }
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<SwathDev> v(n_swaths);
  long long off = 0;
  for (int i = 0; i < n_swaths; ++i) {
    v[i] = make_dev(p->sw[i]);
    v[i].echo = io[i].echo;
    v[i].scale = io[i].echo_scale;
    v[i].tx = io[i].tx_pos;
    v[i].rx = io[i].rx_pos;
    v[i].vel = io[i].rx_vel;
    v[i].track = io[i].rx_track;
    v[i].tstats = p->tstats + p->sw[i].tstats_off;
    v[i].c = io[i].c;
    v[i].image = reinterpret_cast<float2*>(io[i].image);
    v[i].gimage = reinterpret_cast<const float2*>(grad_image[i]);
    v[i].grad_tx = grad_tx[i];
    v[i].grad_rx = grad_rx[i];
    v[i].grad_c = grad_c[i];
    v[i].part_off = off;
    off += (long long)p->sw[i].ntiles * p->sw[i].d.n_ping * p->sw[i].d.n_elem;
  }
  if (!p->adj_buf) {
    const size_t bytes = sizeof(double) * ((size_t)p->lay.n_partials * kPartial + (size_t)n_swaths * p->max_p);
    if (hipMalloc(&p->adj_buf, bytes) != hipSuccess) {
      p->adj_buf = nullptr;
      return fail(SAS_BP_ENOMEM, "adjoint workspace of %zu bytes could not be allocated", bytes);
    }
    p->ws.partials = reinterpret_cast<double*>(p->adj_buf);
    p->ws.cpart = p->ws.partials + (size_t)p->lay.n_partials * kPartial;
  }
  rc = upload(p, v, st);
  if (rc) return rc;
  HIP_TRY(launch_init(p->ws, st));
  HIP_TRY(launch_cull(p->ws, p->n_tiles, p->tiling.TX, p->tiling.TY, p->tiling.TZ, p->bucket_shift, st));
  HIP_TRY(launch_order(p->ws, p->n_tiles, p->bucket_shift, st));
  hipEvent_t ea = nullptr, eb = nullptr;
  if (p->timing) {
    rc = timing_pair(p, &ea, &eb);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ea, st));
  }
  HIP_TRY(launch_adjoint(p->adjoint_fn, p->ws, p->n_tiles, p->adj_grid, p->tiling.NT, p->adj_lds_bytes, st));
  if (p->timing) {
    HIP_TRY(hipEventRecord(eb, st));
    ++p->n_timed;
  }
  HIP_TRY(launch_adjoint_reduce(p->ws, n_swaths, p->max_p, st));
  return SAS_BP_OK;
}

int sas_bp_reproject(sas_bp_plan_t p, const sas_bp_swath_io* io, const void* const* image_in,
                     void* const* echo_out, int n_swaths, void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  int rc = check_io(p, io, n_swaths);
  if (rc) return rc;
  if (!image_in || !echo_out) return fail(SAS_BP_EINVAL, "image_in or echo_out is NULL");
  if (p->interp != SAS_BP_INTERP_LINEAR || p->motion || p->refract)
    return fail(SAS_BP_EUNSUPPORTED, "reprojection is built for linear interpolation, stop-and-hop positions and "
                "straight paths only");
  for (int i = 0; i < n_swaths; ++i) {
    if (!image_in[i] || !echo_out[i]) return fail(SAS_BP_EINVAL, "swath %d: NULL image_in or echo_out", i);
    if (((uintptr_t)image_in[i] & 7u) || ((uintptr_t)echo_out[i] & 7u))
      return fail(SAS_BP_EINVAL, "swath %d: image_in or echo_out not 8-byte aligned", i);
  }
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<SwathDev> v(n_swaths);
  for (int i = 0; i < n_swaths; ++i) {
    v[i] = make_dev(p->sw[i]);
    v[i].echo = io[i].echo;
    v[i].scale = io[i].echo_scale;
    v[i].tx = io[i].tx_pos;
    v[i].rx = io[i].rx_pos;
    v[i].vel = io[i].rx_vel;
    v[i].track = io[i].rx_track;
    v[i].tstats = p->tstats + p->sw[i].tstats_off;
    v[i].c = io[i].c;
    v[i].image = reinterpret_cast<float2*>(io[i].image);
    v[i].gimage = reinterpret_cast<const float2*>(image_in[i]);
    v[i].gecho = reinterpret_cast<float2*>(echo_out[i]);
  }
  rc = upload(p, v, st);
  if (rc) return rc;
  for (int i = 0; i < n_swaths; ++i) {
    const auto& d = p->sw[i].d;
    HIP_TRY(launch_zero_rows(echo_out[i], (long long)d.n_ping * d.n_elem * d.n_sample, st));
  }
  HIP_TRY(launch_init(p->ws, st));
  HIP_TRY(launch_cull(p->ws, p->n_tiles, p->tiling.TX, p->tiling.TY, p->tiling.TZ, p->bucket_shift, st));
  HIP_TRY(launch_order(p->ws, p->n_tiles, p->bucket_shift, st));
  hipEvent_t ea = nullptr, eb = nullptr;
  if (p->timing) {
    rc = timing_pair(p, &ea, &eb);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ea, st));
  }
  HIP_TRY(launch_reproject(p->reproject_fn, p->ws, p->n_tiles, p->rep_grid, p->tiling.NT, p->lds_bytes, st));
  if (p->timing) {
    HIP_TRY(hipEventRecord(eb, st));
    ++p->n_timed;
  }
  return SAS_BP_OK;
}

int sas_bp_drc(sas_bp_plan_t p, const void* image, int64_t n_pix, double brightness, float* out, double* params,
               void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (!image || !out) return fail(SAS_BP_EINVAL, "image or out is NULL");
  if (n_pix < 1 || n_pix > (int64_t)1 << 31) return fail(SAS_BP_EINVAL, "n_pix must be in [1, 2^31]");
  if (!(brightness > 0.0 && brightness < 1.0)) return fail(SAS_BP_EINVAL, "brightness must lie in (0, 1)");
  if (((uintptr_t)image & 7u) || ((uintptr_t)out & 3u) || ((uintptr_t)params & 7u))
    return fail(SAS_BP_EINVAL, "image, out or params misaligned");
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_drc(image, (long long)n_pix, brightness, out, params, p->slab + p->lay.drc, st));
  return SAS_BP_OK;
}

int sas_bp_whiten(sas_bp_plan_t p, int swath, void* echo, double gamma, void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (swath < 0 || swath >= p->n_swaths) return fail(SAS_BP_EINVAL, "swath %d out of range", swath);
  if (!echo) return fail(SAS_BP_EINVAL, "echo is NULL");
  if ((uintptr_t)echo & 7u) return fail(SAS_BP_EINVAL, "echo misaligned");
  if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(SAS_BP_EINVAL, "gamma must be finite and >= 0");
  const auto& d = p->sw[swath].d;
  const long long rows = (long long)d.n_ping * d.n_elem;
  if (rows > 0x7fffffffll) return fail(SAS_BP_EUNSUPPORTED, "too many rows for one batched transform");
  DeviceGuard guard(p->device);
  if (!p->whiten_buf) {
    size_t bytes = 0;
    for (const auto& s : p->sw) bytes = std::max(bytes, whiten_work_bytes(s.d.n_sample));
    if (hipMalloc(&p->whiten_buf, bytes) != hipSuccess) {
      p->whiten_buf = nullptr;
      return fail(SAS_BP_ENOMEM, "whitening workspace of %zu bytes could not be allocated", bytes);
    }
  }
  if (p->fft_plans.empty()) p->fft_plans.assign(p->n_swaths, nullptr);
  if (!whiten_hand_written(d.n_sample) && !p->fft_plans[swath] &&
      make_fft_plan(d.n_sample, rows, &p->fft_plans[swath]) != 0) {
    p->fft_plans[swath] = nullptr;
    return fail(SAS_BP_EDEVICE, "FFT plan for %d x %lld samples could not be made", d.n_sample, rows);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int rc = launch_whiten(p->fft_plans[swath], echo, rows, d.n_sample, gamma, p->whiten_buf, st);
  if (rc) return fail(SAS_BP_EDEVICE, "whitening failed (%s)", rc == 2 ? "FFT" : rc == 1 ? "FFT stream" : "kernel");
  return SAS_BP_OK;
}

int sas_bp_range_compress(sas_bp_plan_t p, int swath, void* echo, const void* replica, int32_t n_taps, int mix,
                          void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (swath < 0 || swath >= p->n_swaths) return fail(SAS_BP_EINVAL, "swath %d out of range", swath);
  if (!echo || !replica) return fail(SAS_BP_EINVAL, "echo or replica is NULL");
  if (((uintptr_t)echo & 7u) || ((uintptr_t)replica & 7u)) return fail(SAS_BP_EINVAL, "echo or replica misaligned");
  const auto& d = p->sw[swath].d;
  if (n_taps < 1 || n_taps > d.n_sample)
    return fail(SAS_BP_EINVAL, "n_taps %d must lie in [1, %d] (the swath's samples)", (int)n_taps, d.n_sample);
  const long long rows = (long long)d.n_ping * d.n_elem;
  const bool fused = n_taps <= rc_fused_taps();
  const int L = fused ? 4096 : rc_transform_length((long long)d.n_sample + n_taps - 1);
  if (L < 0) return fail(SAS_BP_EUNSUPPORTED, "transform length beyond 2^31");
  DeviceGuard guard(p->device);
  auto& rc = p->rc;
  // small buffer: filter (L), twiddle table (4080), mix table (N_s), replica energy
  const size_t tw_off = align_up(8u * (size_t)L), mix_off = tw_off + align_up(8u * 4080);
  const size_t eq_off = mix_off + align_up(8u * (size_t)d.n_sample), small_bytes = eq_off + kAlign;
  if (rc.small_bytes < small_bytes) {
    if (rc.small) (void)hipFree(rc.small);
    rc.small_bytes = 0;
    if (hipMalloc(&rc.small, small_bytes) != hipSuccess) {
      rc.small = nullptr;
      return fail(SAS_BP_ENOMEM, "range compression filter of %zu bytes could not be allocated", small_bytes);
    }
    rc.small_bytes = small_bytes;
  }
  unsigned char* sm = static_cast<unsigned char*>(rc.small);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (fused) {
    const int r = launch_range_compress_fused(echo, rows, d.n_sample, replica, n_taps, d.f_c, d.t0, d.f_s, mix ? 1 : 0,
                                              sm, sm + tw_off, sm + mix_off, sm + eq_off, st);
    if (r) return fail(SAS_BP_EDEVICE, "range compression kernel launch failed");
    return SAS_BP_OK;
  }
  // Rows per batch: a padded batch of at most 256 MiB and 1024 rows.
  long long B = (256ll << 20) / (8ll * L);
  B = std::max(1ll, std::min(B, std::min(1024ll, rows)));
  if (rc.L != L || rc.B != (int)B) {
    destroy_fft_plan(rc.batch);
    destroy_fft_plan(rc.single);
    rc.batch = rc.single = nullptr;
    rc.L = rc.B = 0;
    if (rc_make_plans(L, (int)B, &rc.batch, &rc.single) != 0)
      return fail(SAS_BP_EDEVICE, "FFT plans of length %d could not be made", L);
    rc.L = L;
    rc.B = (int)B;
  }
  const size_t buf_bytes = 8u * (size_t)B * L;
  if (rc.buf_bytes < buf_bytes) {
    if (rc.buf) (void)hipFree(rc.buf);
    rc.buf_bytes = 0;
    if (hipMalloc(&rc.buf, buf_bytes) != hipSuccess) {
      rc.buf = nullptr;
      return fail(SAS_BP_ENOMEM, "range compression workspace of %zu bytes could not be allocated", buf_bytes);
    }
    rc.buf_bytes = buf_bytes;
  }
  const int r = launch_range_compress(rc.batch, rc.single, echo, rows, d.n_sample, L, (int)B, replica, n_taps, d.f_c,
                                      d.t0, d.f_s, mix ? 1 : 0, rc.buf, sm, sm + mix_off, sm + eq_off, st);
  if (r) return fail(SAS_BP_EDEVICE, "range compression failed (%s)", r == 2 ? "FFT" : r == 1 ? "FFT stream" : "kernel");
  return SAS_BP_OK;
}

int sas_bp_dpc_tde(sas_bp_plan_t p, int swath, const void* echo, const int32_t* pairs, int n_pairs, int32_t win,
                   int32_t hop, int32_t max_lag, float* out, void* stream) {
  constexpr int kMaxTdePairs = 256;
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (swath < 0 || swath >= p->n_swaths) return fail(SAS_BP_EINVAL, "swath %d out of range", swath);
  if (!echo || !pairs || !out) return fail(SAS_BP_EINVAL, "echo, pairs or out is NULL");
  if (((uintptr_t)echo & 7u) || ((uintptr_t)out & 15u)) return fail(SAS_BP_EINVAL, "echo or out misaligned");
  const auto& d = p->sw[swath].d;
  if (d.echo_dtype != SAS_BP_ECHO_C64) return fail(SAS_BP_EUNSUPPORTED, "time-delay estimation reads complex64 echoes");
  if (d.n_ping < 2 || d.n_ping - 1 > 65535) return fail(SAS_BP_EUNSUPPORTED, "need 2..65536 pings, got %d", d.n_ping);
  if (n_pairs < 1 || n_pairs > kMaxTdePairs) return fail(SAS_BP_EINVAL, "n_pairs must lie in [1, %d]", kMaxTdePairs);
  if (win < 2 || win > 2048 || win > d.n_sample) return fail(SAS_BP_EINVAL, "win must lie in [2, min(2048, N_s)]");
  if (hop < 1) return fail(SAS_BP_EINVAL, "hop must be >= 1");
  if (max_lag < 1 || max_lag > tde_max_lag()) return fail(SAS_BP_EINVAL, "max_lag must lie in [1, %d]", tde_max_lag());
  for (int j = 0; j < n_pairs; ++j)
    if (pairs[2 * j] < 0 || pairs[2 * j] >= d.n_elem || pairs[2 * j + 1] < 0 || pairs[2 * j + 1] >= d.n_elem)
      return fail(SAS_BP_EINVAL, "pair %d names an element outside [0, %d)", j, d.n_elem);
  DeviceGuard guard(p->device);
  if (!p->tde_pairs) {
    if (hipMalloc(&p->tde_pairs, sizeof(int) * 2 * kMaxTdePairs) != hipSuccess) {
      p->tde_pairs = nullptr;
      return fail(SAS_BP_ENOMEM, "time-delay estimation pair buffer could not be allocated");
    }
    if (hipHostMalloc(&p->tde_pairs_host, sizeof(int) * 2 * kMaxTdePairs) != hipSuccess) {
      p->tde_pairs_host = nullptr;
      return fail(SAS_BP_ENOMEM, "time-delay estimation staging buffer could not be allocated");
    }
    HIP_TRY(hipEventCreateWithFlags(&p->tde_copied, hipEventDisableTiming));
  } else {
    HIP_TRY(hipEventSynchronize(p->tde_copied));   // the previous call's copy has left the staging buffer
  }
  std::memcpy(p->tde_pairs_host, pairs, sizeof(int) * 2 * n_pairs);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(p->tde_pairs, p->tde_pairs_host, sizeof(int) * 2 * n_pairs, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(p->tde_copied, st));
  HIP_TRY(launch_dpc_tde(echo, d.n_ping, d.n_elem, d.n_sample, p->tde_pairs, n_pairs, win, hop, max_lag, d.f_s, out,
                         st));
  return SAS_BP_OK;
}

int sas_bp_tvg(sas_bp_plan_t p, int swath, void* echo, double alpha, float* gain_out, void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (swath < 0 || swath >= p->n_swaths) return fail(SAS_BP_EINVAL, "swath %d out of range", swath);
  if (!echo) return fail(SAS_BP_EINVAL, "echo is NULL");
  if (((uintptr_t)echo & 7u) || ((uintptr_t)gain_out & 3u)) return fail(SAS_BP_EINVAL, "echo or gain_out misaligned");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SAS_BP_EINVAL, "alpha must be finite and >= 0");
  const auto& d = p->sw[swath].d;
  DeviceGuard guard(p->device);
  if (!p->tvg_buf) {
    int max_ns = 0;
    for (const auto& s : p->sw) max_ns = std::max(max_ns, s.d.n_sample);
    if (hipMalloc(&p->tvg_buf, sizeof(float) * 2 * (size_t)max_ns) != hipSuccess) {
      p->tvg_buf = nullptr;
      return fail(SAS_BP_ENOMEM, "time-varying gain workspace of %zu bytes could not be allocated",
                  sizeof(float) * 2 * (size_t)max_ns);
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_tvg(echo, (long long)d.n_ping * d.n_elem, d.n_sample, alpha, reinterpret_cast<float*>(p->tvg_buf),
                     gain_out, st));
  return SAS_BP_OK;
}

int sas_bp_envelope(sas_bp_plan_t p, int swath, const void* echo, void* out, void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (swath < 0 || swath >= p->n_swaths) return fail(SAS_BP_EINVAL, "swath %d out of range", swath);
  if (!echo || !out) return fail(SAS_BP_EINVAL, "echo or out is NULL");
  const auto& d = p->sw[swath].d;
  const unsigned align = d.echo_dtype == SAS_BP_ECHO_C64 ? 7u : 3u;
  if (((uintptr_t)echo & align) || ((uintptr_t)out & align)) return fail(SAS_BP_EINVAL, "echo or out misaligned");
  const long long n = (long long)d.n_ping * d.n_elem * d.n_sample;
  const size_t bytes = (size_t)n * (d.echo_dtype == SAS_BP_ECHO_C64 ? 8 : 4);
  const uintptr_t a = (uintptr_t)echo, b = (uintptr_t)out;
  if (a != b && a < b + bytes && b < a + bytes) return fail(SAS_BP_EINVAL, "echo and out overlap without being equal");
  DeviceGuard guard(p->device);
  HIP_TRY(launch_envelope(echo, out, n, d.echo_dtype, reinterpret_cast<hipStream_t>(stream)));
  return SAS_BP_OK;
}

int sas_bp_useful_updates(sas_bp_plan_t p, const sas_bp_swath_io* io, int n_swaths, void* stream, int64_t* counts) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (!counts) return fail(SAS_BP_EINVAL, "counts is NULL");
  int rc = check_io(p, io, n_swaths);
  if (rc) return rc;
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<SwathDev> v(n_swaths);
  for (int i = 0; i < n_swaths; ++i) {
    v[i] = make_dev(p->sw[i]);
    v[i].echo = io[i].echo;
    v[i].scale = io[i].echo_scale;
    v[i].tx = io[i].tx_pos;
    v[i].rx = io[i].rx_pos;
    v[i].vel = io[i].rx_vel;
    v[i].track = io[i].rx_track;
    v[i].tstats = p->tstats + p->sw[i].tstats_off;
    v[i].c = io[i].c;
    v[i].image = reinterpret_cast<float2*>(io[i].image);
  }
  rc = upload(p, v, st);
  if (rc) return rc;
  unsigned long long* dcount = reinterpret_cast<unsigned long long*>(p->ws.scratch64);
  for (int i = 0; i < n_swaths; ++i) {
    const auto& s = p->sw[i].d;
    if (s.gate_half_angle <= 0.0) {
      counts[i] = (int64_t)s.n[0] * s.n[1] * s.n[2] * s.n_ping * s.n_elem;
      continue;
    }
    HIP_TRY(launch_count(p->ws, i, s.n_ping, s.n_elem, (int)(s.n[1] * s.n[2]), dcount, st));
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, dcount, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    counts[i] = (int64_t)h;
  }
  return SAS_BP_OK;
}

int sas_bp_sharpness(sas_bp_plan_t p, const void* image, int64_t n_pix, double* out_S, void* grad_image,
                     void* stream) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (!image || !out_S) return fail(SAS_BP_EINVAL, "NULL pointer");
  if (n_pix < 1) return fail(SAS_BP_EINVAL, "n_pix must be >= 1");
  if (((uintptr_t)image & 7u) || ((uintptr_t)out_S & 7u) || ((uintptr_t)grad_image & 7u))
    return fail(SAS_BP_EINVAL, "pointer not 8-byte aligned");
  DeviceGuard guard(p->device);
  HIP_TRY(launch_sharpness(image, (long long)n_pix, p->ws.scratch64 + 16, out_S, grad_image,
                           reinterpret_cast<hipStream_t>(stream)));
  return SAS_BP_OK;
}

}  // extern "C"

// ------------------------------------------- allocation-free sharpness ---
// The partial sums of sas_bp_sharpness_static live in this fixed device array
// instead of a plan's workspace. In host code its name is only a stand-in for
// the device variable: the address each device holds it at is looked up once
// per device (hipGetSymbolAddress, with that device current) and only that
// address is passed to kernels.
static __device__ __align__(256) double scratch[kSharpScratch];

namespace {

constexpr int kStaticMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kStaticMaxDevices] = {};   // scratch's address on each device, once looked up

// scratch's device address on the current device (looked up on first use).
int static_scratch(int* device, double** out) {
  HIP_TRY(hipGetDevice(device));
  if (*device < 0 || *device >= kStaticMaxDevices)
    return fail(SAS_BP_EUNSUPPORTED, "device %d: at most %d devices", *device, kStaticMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[*device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SAS_BP_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", *device,
                  hipGetErrorString(e));
    g_scratch_ptr[*device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[*device];
  return SAS_BP_OK;
}

}  // namespace

extern "C" {

int sas_bp_sharpness_static(const void* image, int64_t n_pix, double* out_S, void* grad_image, void* stream) {
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  if (!image || !out_S) return fail(SAS_BP_EINVAL, "NULL pointer");
  if (n_pix < 1 || n_pix > SAS_BP_SHARPNESS_STATIC_MAX_PIX)
    return fail(SAS_BP_EINVAL, "n_pix must be in [1, %lld]", (long long)SAS_BP_SHARPNESS_STATIC_MAX_PIX);
  if (((uintptr_t)image & 7u) || ((uintptr_t)out_S & 7u) || ((uintptr_t)grad_image & 7u))
    return fail(SAS_BP_EINVAL, "pointer not 8-byte aligned");
  int device = 0;
  double* ptr = nullptr;
  int rc = static_scratch(&device, &ptr);
  if (rc) return rc;
  HIP_TRY(launch_sharpness(image, (long long)n_pix, ptr, out_S, grad_image, reinterpret_cast<hipStream_t>(stream)));
  return SAS_BP_OK;
}

int sas_bp_plan_status(sas_bp_plan_t p) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  DeviceGuard guard(p->device);
  unsigned h = 0;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(&h, p->ws.counters + 1, sizeof h, hipMemcpyDeviceToHost));
  const unsigned z = 0;
  HIP_TRY(hipMemcpy(p->ws.counters + 1, &z, sizeof z, hipMemcpyHostToDevice));
  if (h & kStatusNav) return SAS_BP_ENAV;
  return (h & kStatusConverge) ? SAS_BP_ECONVERGE : SAS_BP_OK;
}

int sas_bp_plan_info(sas_bp_plan_t p, int64_t info[10]) {
  if (!p || !info) return fail(SAS_BP_EINVAL, "NULL argument");
  info[0] = p->tiling.TX;
  info[1] = p->tiling.TY;
  info[2] = p->tiling.TZ;
  info[3] = p->sw[0].CP;
  info[4] = p->sw[0].W;
  info[5] = p->lds_bytes;
  info[6] = p->grid;
  info[7] = p->tiling.NT;
  info[8] = p->sw[0].RC;
  info[9] = p->occ;
  return SAS_BP_OK;
}

int sas_bp_set_kernel_timing(sas_bp_plan_t p, int enable) {
  if (!p) return fail(SAS_BP_EINVAL, "plan is NULL");
  p->timing = enable != 0;
  p->n_timed = 0;
  return SAS_BP_OK;
}

int sas_bp_kernel_time(sas_bp_plan_t p, double* ms_total, int64_t* launches) {
  if (!p || !ms_total || !launches) return fail(SAS_BP_EINVAL, "NULL argument");
  (void)hipGetLastError();   // an earlier failed runtime call must not be reported as ours
  DeviceGuard guard(p->device);
  double sum = 0.0;
  for (size_t i = 0; i < p->n_timed; ++i) {
    HIP_TRY(hipEventSynchronize(p->events[2 * i + 1]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, p->events[2 * i], p->events[2 * i + 1]));
    sum += (double)ms;
  }
  *ms_total = sum;
  *launches = (int64_t)p->n_timed;
  p->n_timed = 0;
  return SAS_BP_OK;
}

// ------------------------------------------------------------ autotune ---

int sas_bp_autotune(const sas_bp_swath_desc* desc, int n_swaths, const sas_bp_swath_io* io,
                    const sas_bp_options* base, int reps, void* stream, sas_bp_options* best, double* best_ms) {
  if (!best || !best_ms) return fail(SAS_BP_EINVAL, "best or best_ms is NULL");
  if (reps < 1 || reps > 1000) return fail(SAS_BP_EINVAL, "reps must be in [1, 1000]");
  if (base && (base->tune_mode < SAS_BP_TUNE_DEFAULT || base->tune_mode > SAS_BP_TUNE_SEARCH))
    return fail(SAS_BP_EINVAL, "tune_mode must be DEFAULT, CACHED or SEARCH");
  // validate with the default tiling, and get the shape class
  const int device = base ? base->device : 0;
  std::string key;
  int rc = shape_class(desc, n_swaths, device, &key);
  if (rc) return rc;
  bool any3d = false;
  int E = 0;
  for (int i = 0; i < n_swaths; ++i) {
    any3d |= desc[i].n[2] > 1;
    E = std::max(E, desc[i].n_elem);
  }
  const char* path = base ? base->tune_cache : nullptr;
  sas_bp_options cand;
  std::memset(&cand, 0, sizeof cand);
  if (base) {
    cand.device = base->device;
    cand.workspace_limit = base->workspace_limit;
    cand.no_cull = base->no_cull;
  }
  cand.use_graph = 1;
  cand.tune_mode = SAS_BP_TUNE_DEFAULT;   // candidates are timed as given, never looked up
  if (!base || base->tune_mode != SAS_BP_TUNE_SEARCH) {
    sas_bp_options stored;
    if (tune_lookup(key, path, &stored)) {
      *best = cand;
      for (int i = 0; i < 6; ++i) *tune_field(best, i) = *tune_field(&stored, i);
      best->tune_cache = path;
      *best_ms = 0.0;
      return SAS_BP_OK;
    }
  }
  DeviceGuard guard(cand.device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t ea = nullptr, eb = nullptr;
  HIP_TRY(hipEventCreate(&ea));
  if (hipEventCreate(&eb) != hipSuccess) {
    (void)hipEventDestroy(ea);
    return fail(SAS_BP_EDEVICE, "hipEventCreate failed");
  }
  double best_time = -1.0;
  sas_bp_options best_opt = cand;
  int last_err = SAS_BP_OK;
  // chunk candidates {pings, elements}: the automatic choice, whole pings,
  // and parts of a ping
  const int kChunks[][2] = {{0, 0}, {1, 0}, {2, 0}, {4, 0}, {8, 0}, {1, 3 * E / 4}, {1, E / 2}, {1, E / 4}};
  for (int l = 0; l < kNumLayouts; ++l) {
    const LaneLayout& L = kLayouts[l];
    if ((L.LZ > 1) != any3d) continue;
    for (const auto& ch : kChunks) {
      if (ch[1] != 0 && (ch[1] < 1 || ch[1] >= E)) continue;
      if (ch[1] == 3 * E / 4 && (ch[1] == E / 2 || ch[1] == E / 4)) continue;   // duplicate for tiny E
      sas_bp_options o = cand;
      o.tile_x = L.LX * L.K;
      o.tile_y = L.LY;
      o.tile_z = L.LZ;
      o.threads = L.LX * L.LY * L.LZ;
      o.pings_per_chunk = ch[0];
      o.elems_per_chunk = ch[1];
      sas_bp_plan_t p = nullptr;
      if (sas_bp_plan(desc, n_swaths, &o, &p) != SAS_BP_OK) continue;   // does not fit: skip
      int e = sas_bp_image(p, io, n_swaths, stream);
      float ms = 0.0f;
      if (e == SAS_BP_OK && hipEventRecord(ea, st) != hipSuccess) e = SAS_BP_EDEVICE;
      for (int r = 0; r < reps && e == SAS_BP_OK; ++r) e = sas_bp_image(p, io, n_swaths, stream);
      if (e == SAS_BP_OK && hipEventRecord(eb, st) != hipSuccess) e = SAS_BP_EDEVICE;
      if (e == SAS_BP_OK && hipEventSynchronize(eb) != hipSuccess) e = SAS_BP_EDEVICE;
      if (e == SAS_BP_OK && hipEventElapsedTime(&ms, ea, eb) != hipSuccess) e = SAS_BP_EDEVICE;
      release(p);
      if (e != SAS_BP_OK) {
        last_err = e;
        if (e == SAS_BP_EINVAL) break;    // the buffers do not match: no candidate can run
        continue;
      }
      const double mean = (double)ms / reps;
      if (best_time < 0.0 || mean < best_time) {
        best_time = mean;
        best_opt = o;
      }
    }
    if (last_err == SAS_BP_EINVAL) break;
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (best_time < 0.0) {
    if (last_err != SAS_BP_OK) return last_err;
    return fail(SAS_BP_EUNSUPPORTED, "no tiling candidate fits these swaths");
  }
  tune_store(key, best_opt, best_time, path);
  *best = best_opt;
  best->tune_cache = path;
  *best_ms = best_time;
  return SAS_BP_OK;
}

int sas_bp_gate_class(const double apex[3], const double box_lo[3], const double box_hi[3], double half_angle,
                      int32_t* record_class, int32_t* may_hit) {
  if (!apex || !box_lo || !box_hi || !record_class || !may_hit) return fail(SAS_BP_EINVAL, "NULL argument");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(apex[a]) || !std::isfinite(box_lo[a]) || !std::isfinite(box_hi[a]))
      return fail(SAS_BP_EINVAL, "apex and box must be finite");
    if (box_lo[a] > box_hi[a]) return fail(SAS_BP_EINVAL, "box_lo[%d] > box_hi[%d]", a, a);
  }
  if (!(half_angle > 0.0) || !(half_angle < 1.5707963267948966))
    return fail(SAS_BP_EINVAL, "half_angle must be in (0, pi/2)");
  const double tg = std::tan(half_angle);
  *record_class = gate_class(tg * tg, apex[0], apex[1], apex[2], box_lo[0], box_hi[0], box_lo[1], box_hi[1],
                             box_lo[2], box_hi[2]);
  *may_hit = cone_may_hit(tg, box_lo[0], box_hi[0], box_lo[1], box_hi[1], box_lo[2], box_hi[2], apex) ? 1 : 0;
  return SAS_BP_OK;
}

void sas_bp_destroy(sas_bp_plan_t p) { release(p); }

}  // extern "C"
