// Internal types shared by the TDBP kernels and the plan (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sasbp {

// Lane layouts of the image and adjoint kernels: a workgroup of
// LX * LY * LZ threads (256 or 512) owns a tile of (LX * K) x LY x LZ pixels;
// lane (lx, ly, lz) owns the K pixels lx + LX k of row (ly, lz).
struct LaneLayout {
  int K, LX, LY, LZ;
};
constexpr LaneLayout kLayouts[] = {
    {2, 8, 32, 1},   // 0: 16 x 32,     256 threads
    {4, 8, 32, 1},   // 1: 32 x 32,     256
    {8, 8, 32, 1},   // 2: 64 x 32,     256
    {4, 16, 32, 1},  // 3: 64 x 32,     512
    {8, 16, 32, 1},  // 4: 128 x 32,    512
    {4, 8, 64, 1},   // 5: 32 x 64,     512
    {4, 8, 8, 4},    // 6: 32 x 8 x 4,  256
    {4, 8, 16, 4},   // 7: 32 x 16 x 4, 512
    {8, 8, 8, 4},    // 8: 64 x 8 x 4,  256
};
constexpr int kNumLayouts = sizeof(kLayouts) / sizeof(kLayouts[0]);
constexpr int kThreads = 256;    // helper kernels (cull, order, count, sharpness)
// Waves per SIMD the image kernel's register budget is compiled for (512
// VGPRs per SIMD lane shared by the resident waves); the plan sizes LDS
// chunks so that this occupancy is not lost to LDS.
constexpr int kImageWaves = 3;
constexpr int kAdjointWaves = 3;   // the adjoint's register budget (its chunks stay whole pings)
constexpr int kMaxElem = 256;
constexpr int kSincHalf = 4;     // windowed-sinc interpolation: taps on each side

// Per-swath constants and pointers, stored in the plan's workspace so that a
// captured graph stays valid when the caller passes new buffers.
struct SwathDev {
  const void* echo;
  const float* scale;
  const double* tx;
  const double* rx;
  const double* c;
  float2* image;
  const float2* gimage;   // adjoint cotangent (complex64, image layout)
  double* grad_tx;        // adjoint outputs
  double* grad_rx;
  double* grad_c;
  float2* gecho;          // reprojection output (complex64, echo layout)
  const double* vel;      // receiver velocity during reception [P][3] (motion 1)
  const double* track;    // receiver displacement table [P][track_n][3] (motion 2)
  float4* tstats;         // per ping of the table: (largest displacement over the record,
                          // largest velocity change between segments, largest segment
                          // speed, 1 if not finite) (motion 2)
  double track_h;         // s between table samples (motion 2)
  int track_n;            // table samples per ping (motion 2)
  int P, E, Ns, dtype;
  int interp;             // 0 linear, 1 windowed sinc over 2 * kSincHalf samples
  int motion;             // 1: receivers move at vel during reception; 2: along the table
  int refract;            // 1: sediment below z_int refracts the legs (sound speed c_sed)
  int no_cull;            // 1: no block cull (every ping of every tile, every record decided per row)
  double c_sed, z_int;
  int nx, ny, nz;
  int ntx, nty, ntz;      // tiles per axis
  int tile0;              // index of this swath's first tile in the global tile list
  int W;                  // LDS window length per (ping, element), samples (without guard)
  int CP;                 // adjoint: pings staged per pass
  int RC;                 // image: (ping, element) records staged per pass
  int SC;                 // pings whose geometry is built at once (a multiple of CP)
  double o[3], d[3];
  double fc, fs, t0;
  double tan_g, sin_g;    // gate: tan and sin of the half-angle (0 = off)
  double c_min;
  double half_diag;       // distance from a tile's centre to its farthest pixel centre
  int64_t part_off;       // adjoint: offset of this swath's partials (in records)
};

// Per-tile ping interval found by the cull pass: pings outside [lo, hi] have
// no (element, pixel) inside both cones. lo > hi means the tile is empty.
struct PingRange {
  int lo, hi;
};

// Workspace layout (byte offsets into the plan's slab).
struct Workspace {
  SwathDev* swaths;       // [n_swaths]
  PingRange* prange;      // [n_tiles]
  int* order;             // [n_tiles] processing order (largest cost first)
  unsigned* counters;     // [0] work counter, [1] status word, [2..] sort scratch
  unsigned* bucket;       // [kBuckets] histogram / cursors for the cost ordering
  int* tile_swath;        // [n_tiles] swath of each tile
  double* partials;       // adjoint: kPartial doubles per (tile, ping, element), allocated on first use
  double* cpart;          // adjoint: per-(swath, ping) sound-speed partials
  double* scratch64;      // sharpness partial sums, counters
  unsigned char* geo;     // per-workgroup geometry of SC pings: geo + blockIdx.x * geo_stride
  long long geo_stride;   // bytes per workgroup
};

// Geometry of a run of SC pings of one tile, built once per run by the whole
// workgroup and then copied chunk by chunk into LDS (bytes from the start of
// the workgroup's region):
//   receiver records [SC][E] (48 B)   window starts [SC][E] (int)
//   transmitter records [SC] (32 B)   gate rows [SC][E][ROWS] (int, gate only)
//   continuous motion only: motion offsets at the tile centre [SC][E] (float),
//   per ping the straight line the receivers follow, R(t) = R + c + v t
//   (3 float4: (v, |v|^2), (c, |c|^2), (c.v, segment index as int bits, 0, 0);
//   c = 0 for a constant velocity; for a table, the segment that holds the
//   tile centre's delay)
constexpr int kRxRecBytes = 48;
constexpr int kMotionLineBytes = 48;
constexpr int kTxRecBytes = 32;

struct GeoLayout {
  long long rec, n0, tx, rows, dc, vel, bytes;
};

__host__ __device__ inline GeoLayout geo_layout(int SC, int E, int ROWS, bool gate, bool motion = false) {
  GeoLayout g;
  long long o = 0;
  g.rec = o;  o += (long long)SC * E * kRxRecBytes;
  g.n0 = o;   o += (long long)SC * E * 4;
  o = (o + 15) & ~15ll;
  g.tx = o;   o += (long long)SC * kTxRecBytes;
  g.rows = o; o += gate ? (long long)SC * E * ROWS * 4 : 0;
  o = (o + 15) & ~15ll;
  g.dc = o;   o += motion ? (long long)SC * E * 4 : 0;
  o = (o + 15) & ~15ll;
  g.vel = o;  o += motion ? (long long)SC * kMotionLineBytes : 0;
  g.bytes = (o + 255) & ~255ll;
  return g;
}

// Most pings that a chunk of RC consecutive (ping, element) records, starting
// at a multiple of RC, can touch when each ping has E records.
__host__ __device__ inline int chunk_pings(int RC, int E) {
  if (RC % E == 0) return RC / E;
  if (E % RC == 0) return 1;
  return (RC - 1) / E + 2;
}

constexpr int kBuckets = 64;

// The MI355X has 8 accelerator complex dies (XCDs), each with its own L2;
// the dispatcher hands workgroups to them round-robin by workgroup index.
// The image kernel keeps one tile queue per XCD (tiles of neighbouring
// along-track stripes read the same echo windows, so a stripe per XCD keeps
// them in one L2) and takes from the other queues once its own is empty.
// Layout of ws.counters: [0] work counter of the single-queue kernels,
// [1] status word, [kQueueCursor + x] next item of XCD x's queue,
// [kQueueStart + x] its first slot in ws.order, [kQueueLen + x] its length.
constexpr int kXcds = 8;
constexpr int kQueueCursor = 4, kQueueStart = 12, kQueueLen = 20, kCounterWords = 32;

// Next tile for a workgroup on XCD xcd: its own queue, then the others in
// turn; -1 once every queue is empty.
__device__ __forceinline__ int next_tile(const Workspace& ws, int xcd) {
  for (int k = 0; k < kXcds; ++k) {
    const int q = (xcd + k) % kXcds;
    const unsigned len = ws.counters[kQueueLen + q];
    const unsigned i = atomicAdd(&ws.counters[kQueueCursor + q], 1u);
    if (i < len) return (int)(ws.counters[kQueueStart + q] + i);
  }
  return -1;
}

// Sharpness: one partial (sum |I|^4, sum |I|^2) pair per block of a fixed grid,
// then the two sums; scratch of 2 kSharpBlocks + 2 doubles.
constexpr int kSharpBlocks = 1024;
constexpr int kSharpScratch = 2 * kSharpBlocks + 2;
constexpr int kPartial = 8;   // gR.xyz, gc, gT.xyz (element 0 only), pad

enum : unsigned { kStatusOk = 0u, kStatusNav = 1u, kStatusConverge = 2u };

}  // namespace sasbp
