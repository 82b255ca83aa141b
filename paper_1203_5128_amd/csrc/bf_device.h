// Device-side views shared by the kernels and the plan runtime of libbf.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "bf_internal.h"

namespace bfi {

// Non-local means: the 8-bit samples f(x + u_k) of a pixel's patch packed
// into one word (sample k in byte k, u_1 = 0 in byte 0), the element type the
// Toeplitz kernels read in place of the image.  Internal dtype code kDtPatch.
struct Patch8x4 {
  uint32_t v;
};
constexpr bf_dtype kDtPatch = (bf_dtype)3;

// bf_dtype of an element type
template <typename Tin>
constexpr bf_dtype dtype_of() {
  return std::is_same<Tin, Patch8x4>::value
             ? kDtPatch
             : (std::is_same<Tin, uint8_t>::value ? BF_U8 : (std::is_same<Tin, uint16_t>::value ? BF_U16 : BF_F32));
}

// Order table on the device (uploaded copy of OrderTable).
struct DevTables {
  const int32_t *idx_of_T;
  const OrderEntry *ent;
  const int32_t *pm;
  const float *pc;
  int32_t T_cap;
  // polynomial range kernel (8-bit input): per pair slot and intensity the
  // basis values of the smoothed images and the coefficients of the combine,
  // which take the place of cos/sin of the raised cosine (NULL otherwise)
  const float2 *lut_gen;
  const float2 *lut_comb;
};

// Per-image scalars written by the range stage and read by every later stage.
struct DevState {
  int32_t *T_used;            // integer T indexing the table (ceil for floats)
  unsigned long long *T_raw;  // bit pattern of the raw T as a non-negative double
  int32_t *flags;             // bit0 non-finite input, bit1 T above the table
  unsigned long long *q_nonpos;  // pixels whose denominator was not positive
};

// Geometry of one image inside the blocked recursive filter.
struct Geom {
  int H, W;
  int64_t pitch;      // input pitch (elements)
  int64_t opitch;     // output pitch (elements)
  int S, logS;        // threads per row group in the horizontal pass (power of two)
  int cC;             // pixels per thread in the horizontal pass (kCSmall or kCLarge)
  int Seff;           // threads of a row group that hold positions: ceil(W / cC) <= S;
                      // the others smooth zeros (the row's zero extension)
  int Spos;           // Seff * cC positions per padded row
  int vS, vC;         // vertical pass: threads per column (power of two), rows per thread
  int vppw;           // vertical pass: pairs per workgroup (one after another)
  // smoothed images of the recursive path, stored in tiles of zth = 2^zlog
  // rows: element (y, p) at ((y >> zlog) Spos + p) zth + (y mod zth), Hz rows
  // per pair (H rounded up to zth).  zth (columns per vertical workgroup)
  // = z_tile_words(vS), zth at least 1 (row-major): 16 elements (256 bytes)
  // for workgroups of 4 and 8 columns, so that each writes 256 contiguous
  // bytes per tile while the horizontal workgroups of neighbouring rows
  // share each line; 8 (one line) for the 2-column workgroups of images
  // taller than 2048 (32 rows per thread) and 4 for the 1-column workgroups
  // (taller than 4096, or 16 rows per thread above 2048), whose
  // horizontal workgroups hold one row each.
  // (Taller tiles make the vertical writes longer but leave each horizontal
  // workgroup a smaller share of the lines it reads; shorter ones scatter
  // the vertical writes.)
  int Hz, zlog;
  // horizontal pass: the pairs of a launch are split into hgroups groups of
  // hkpg pairs, each a row of workgroups with its own partial sums; a
  // workgroup takes hrows image rows (a power of two <= 256/S), each with
  // 256/(S hrows) pairs in flight
  int hgroups, hkpg, hrows;
  float center;       // intensity subtracted from f in the f*cos, f*sin images
  // Toeplitz path: smoothed images stored with a left pad of padl elements
  // (padl = R mod 8) and a row pitch of zpitch elements (multiple of 8)
  int64_t zpitch;
  int padl;
};



// FIR taps and tile shape of the Toeplitz path.
struct ToepCfg {
  const float *taps;  // device, 2R+1 floats, exp(-(d-R)^2 / 2 sigma_s^2)
  int R;
  int nks;            // K-steps of 32 taps: 32 nks >= 16 + 2R
  int rows;           // output rows per vertical tile (multiple of 16)
  int groups;         // pair groups of the horizontal pass (partial sums each)
  int kpg;            // pairs per group
};

// LDS of a gfx950 CU (all of it may go to one workgroup), and the largest
// dynamic tile of the Toeplitz kernels (room left for their static tables).
constexpr int kToepLdsMax = 160 * 1024;
constexpr int kToepDynMax = kToepLdsMax - 4 * 1024;

// Block coordinates handed to a kernel body: the launch's own blockIdx for a
// single image, or the coordinates inside one image's share of a grouped
// launch over several images.
struct Blk {
  int x, y, z;
};

// Grouped launches: one launch runs the same stage for several images.  Image
// i owns the launch's blocks [start[i], start[i+1]); each image's arguments
// carry its own grid (gx, gy, gz), into which its local block index is
// decomposed x-fastest.
struct GroupGrid {
  int gx, gy, gz;
};
__device__ __forceinline__ int group_find(const int *__restrict__ start, int n, int bid) {
  int lo = 0, hi = n - 1;  // largest i with start[i] <= bid (it owns bid)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= bid) lo = mid;
    else hi = mid - 1;
  }
  // the same for every lane of the workgroup: say so, so that the image's
  // arguments are read with scalar loads into scalar registers
  return __builtin_amdgcn_readfirstlane(lo);
}
__device__ __forceinline__ Blk group_blk(const GroupGrid &gg, int local) {
  // the division runs on the vector unit; its results are the same in every
  // lane, and saying so keeps what derives from them in scalar registers
  return Blk{__builtin_amdgcn_readfirstlane(local % gg.gx), __builtin_amdgcn_readfirstlane((local / gg.gx) % gg.gy),
             __builtin_amdgcn_readfirstlane(local / (gg.gx * gg.gy))};
}

// Offset of element (y, p) of one pair's smoothed images (recursive path).
__host__ __device__ constexpr int z_tile_words(int vS) { return vS >= 256 ? 4 : (vS >= 128 ? 8 : 16); }
__host__ __device__ inline size_t z_index(const Geom &g, int y, int p) {
  return (((size_t)(y >> g.zlog) * g.Spos + p) << g.zlog) + (y & ((1 << g.zlog) - 1));
}

// Per-image arguments of the kernels that also run as grouped launches.
struct ResetArgs {
  GroupGrid gg;
  DevState st;
  int32_t T_used;
  double T_raw;
};
struct RowmaxArgs {
  GroupGrid gg;
  const void *f;
  int64_t pitch;
  int H, W, R;
  void *rowmax;
  DevState st;
};
struct ColmaxArgs {
  GroupGrid gg;
  const void *f;
  int64_t pitch;
  const void *rowmax;
  int H, W, R;
  DevState st;
  int32_t T_cap;
};
// Per-image accumulators of the one-launch range stage: a running maximum
// (double bit pattern), the OR of the flags and the count of arrivals; a top
// slot and kRangeSubs sub-slots.  All zero between calls (the last arrival
// at each slot clears it).
constexpr int kRangeSubs = 32;
struct RangeAccSlot {
  unsigned long long T;
  int32_t flags;
  uint32_t count;
};
struct RangeAcc {
  RangeAccSlot *top;
  RangeAccSlot *sub;       // [kRangeSubs]
  unsigned long long *lb;  // [kRangeSubs] lower bounds of T from the tile statistics
                           // (double bit patterns, merged by tile index mod kRangeSubs)
};
struct RangeTileArgs {
  GroupGrid gg;
  const void *f;
  int64_t pitch;
  int H, W, R;
  DevState st;
  RangeAcc acc;
  int32_t T_cap;
  int2 *tstats;  // per 32 x 32 tile: (max key, min key) of f, written by the statistics
                 // pass; null: no statistics, every tile is computed
  int nwg;       // workgroups of the tile kernel for this image (tile t: workgroup t mod nwg)
};
// Workgroups of the tile kernel for an image of `tiles` tiles when a launch
// covers `total` tiles: about kRangeTileWgs in all, each image's tiles
// spread over its share.  (Range stage of the 64-image batch with about
// 256 / 512 / 1024 / 2048 / 4096 workgroups per launch: 148 / 118 / 110 /
// 125 / 163 us; one tile per workgroup: 272 us.)
constexpr int kRangeTileWgs = 1024;
__host__ __device__ inline int range_tile_wgs(int tiles, long long total) {
  const long long per = total > kRangeTileWgs ? total / kRangeTileWgs : 1;
  return (int)((tiles + per - 1) / per);
}
// Single images with fewer tiles run the tile kernel without statistics.
constexpr int kRangeStatsMinTiles = 1024;
// Grid of the statistics pass over a tile grid gt: (tile columns, strips of
// kStatTiles tiles).
constexpr int kStatTiles = 4;
__host__ __device__ inline GroupGrid range_stats_grid(const GroupGrid &gt) {
  return GroupGrid{gt.gx, (gt.gy + kStatTiles - 1) / kStatTiles, 1};
}

struct ToepVArgs {  // vertical pass: blocks (launch tile index, pair)
  GroupGrid gg;
  const void *f;
  Geom g;
  DevTables tab;
  DevState st;
  ToepCfg tc;
  int ntx, ntiles, per, k0;
  void *Z;
  size_t zplane;
};
struct ToepHArgs {  // horizontal pass + combine: blocks (launch tile index, pair group)
  GroupGrid gg;
  const void *f;
  float *out;
  Geom g;
  DevTables tab;
  DevState st;
  ToepCfg tc;
  int ntx, ntiles, per, k0, kcount;
  const void *Z;
  size_t zplane;
  float2 *PQ;
  int first, finish;
};
struct FinishArgs {  // sum of the groups' partial sums and the division
  GroupGrid gg;
  const void *f;
  float *out;
  Geom g;
  DevState st;
  const float2 *PQ;
  int groups;
  float rscale;  // out = center + rscale * P / Q
};

struct IirArgs {  // the two recursive-path kernels (each with its own grid)
  GroupGrid gg;
  const void *f;
  float *out;
  Geom g;
  DevTables tab;
  DevState st;
  const float *iir;
  int k0, kcount;
  float4 *Z;
  float2 *PQ;
  int first, last;
  float2 *glut;
};

// Optional recorder of stage boundaries (host side): called before and after
// each stage's launches on the launch stream.
struct StageRec {
  void (*mark)(void *ctx, int stage, hipStream_t s, bool end) = nullptr;
  void *ctx = nullptr;
  void begin(int stage, hipStream_t s) const { if (mark) mark(ctx, stage, s, false); }
  void end(int stage, hipStream_t s) const { if (mark) mark(ctx, stage, s, true); }
};

// ---- launch wrappers (bf_kernels.hip) ----
hipError_t launch_fill_checker(hipStream_t s, bf_dtype dt, void *f, int H, int W, double top);
hipError_t launch_reset(hipStream_t s, DevState st, int32_t T_used, double T_raw);
// Zero fill of `bytes` (a multiple of 4) at p, as a kernel.
hipError_t launch_zero(hipStream_t s, void *p, size_t bytes);
// Non-local means: the patch image (H x W words, row pitch W) of an 8-bit
// image, sample k at (clamp(y + dy[k]), clamp(x + dx[k])), k < p.
struct PatchArgs {
  const uint8_t *f;
  int64_t pitch;
  int H, W, p;
  int dy[4], dx[4];
  Patch8x4 *out;
};
hipError_t launch_patch_pack(hipStream_t s, const PatchArgs &a);
// Algorithm 1 for one image, with the state reset it needs (tile statistics
// and the one-launch tile kernel when range_tile_ok(R, dt), rowmax then
// holding the statistics; else reset + row pass + column pass, rowmax
// holding the row maxima).
hipError_t launch_range(hipStream_t s, bf_dtype dt, const void *f, const Geom &g, int R, void *rowmax,
                        DevState st, RangeAcc acc, int32_t T_cap, const StageRec &rec);
// Grids of the two-pass range stage for one image (R > 48), and the
// one-launch kernel's coverage.
GroupGrid range_row_grid(const Geom &g);
GroupGrid range_col_grid(const Geom &g);
bool range_tile_ok(int R, bf_dtype dt);
int range_tile_kr(int R);  // staged-block size class (32 or 48) of a tile-kernel image
GroupGrid range_tile_grid(const Geom &g);
// LDS of the tile kernel for radius R staged as block size kr (0: R's own)
size_t range_tile_lds(int R, bf_dtype dt, int kr = 0);
hipError_t launch_range_tile_group(hipStream_t s, bf_dtype dt, int kr, const RangeTileArgs *a, const int *start,
                                   int total, int n, size_t lds);
// Tile statistics of the one-launch kernel's images (same grid), which must
// precede it: a.tstats and a.acc.lb are written.
hipError_t launch_range_stats_group(hipStream_t s, bf_dtype dt, const RangeTileArgs *a, const int *start, int total,
                                    int n);
// Grouped launches over n images (device argument arrays and block starts).
hipError_t launch_reset_group(hipStream_t s, const ResetArgs *a, const int *start, int total, int n);
hipError_t launch_range_group(hipStream_t s, bf_dtype dt, const RowmaxArgs *ra, const int *rstart, int rtotal,
                              const ColmaxArgs *ca, const int *cstart, int ctotal, int n);
hipError_t launch_iir_chunk(hipStream_t s, bf_dtype dt, const void *f, float *out, const Geom &g,
                            DevTables tab, DevState st, const float *iir, int k0, int kcount,
                            float4 *Z, float2 *PQ, bool first, bool last, float2 *glut, const StageRec &rec);

// Arguments of the recursive-path kernels of one image ([0] vertical, [1]
// horizontal + combine) and of the sum of its pair groups when there are
// several.
void iir_args(const void *f, float *out, const Geom &g, DevTables tab, DevState st, const float *iir, int k0,
              int kcount, float4 *Z, float2 *PQ, bool first, bool last, float2 *glut, IirArgs a[2],
              FinishArgs &fa);
// Grouped launches over n images of one dtype: the vertical pass of images
// with SV threads per column and cV rows per thread; the horizontal pass (and
// the finishing sums) of images with S threads per row and cC columns per
// thread.
hipError_t launch_iir_v_group(hipStream_t s, bf_dtype dt, int SV, int cV, const IirArgs *a, const int *start,
                              int n, int total, const StageRec &rec);
hipError_t launch_iir_h_group(hipStream_t s, bf_dtype dt, int S, int cC, const IirArgs *a, const int *start,
                              int n, int total, const FinishArgs *fa, const int *fstart, int ftotal,
                              const StageRec &rec);
// Sum of the pair groups' partial sums and the division (one image, or
// grouped over n images of one dtype).
hipError_t launch_finish(hipStream_t s, bf_dtype dt, const FinishArgs *one, const FinishArgs *arr,
                         const int *start, int n, int total);

// ---- Toeplitz MFMA path (bf_toeplitz.hip) ----
// LDS bytes of the two kernels' dynamic tiles, and the horizontal tile width.
size_t toeplitz_v_lds(int variant, int rows, int nks);
size_t toeplitz_h_lds(int variant, int nks);
int toeplitz_h_tiles(int variant, int H, int W);
// Allow the Toeplitz kernels the LDS they may ask for (once per process).
hipError_t toeplitz_setup();
// Arguments of the Toeplitz kernels for one image and pairs [k0, k0+kcount);
// fa.gg.gx blocks of the finishing kernel are needed when the image splits its
// pairs into several groups and this is its last launch (ha.finish == 0).
void toeplitz_args(int variant, const void *f, float *out, const Geom &g, DevTables tab, DevState st,
                   const ToepCfg &tc, int k0, int kcount, void *Z, float2 *PQ, bool first, bool last,
                   ToepVArgs &va, ToepHArgs &ha, FinishArgs &fa);
// A grouped launch of the Toeplitz stages: device argument arrays, block
// starts (n+1 entries each), block totals and the largest dynamic LDS.
struct ToepGroup {
  int n;
  const ToepVArgs *va;
  const int *vstart;
  int vtotal;
  size_t vlds;
  const ToepHArgs *ha;
  const int *hstart;
  int htotal;
  size_t hlds;
  const FinishArgs *fa;
  const int *fstart;
  int ftotal;
};
hipError_t launch_toeplitz_group(hipStream_t s, bf_dtype dt, int variant, const ToepGroup &tg,
                                 const StageRec &rec);
hipError_t launch_toeplitz_chunk(hipStream_t s, bf_dtype dt, int variant, const void *f, float *out, const Geom &g,
                                 DevTables tab, DevState st, const ToepCfg &tc, int k0, int kcount, void *Z,
                                 float2 *PQ, bool first, bool last, const StageRec &rec);

}  // namespace bfi
