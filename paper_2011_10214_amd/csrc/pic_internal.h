// Internal declarations shared by the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace pic {

// Cells per tile edge. A workgroup of the step kernel owns one tile of
// kTile^3 cells; it stages node E and a private rho for the tile grown by one
// cell on every side (kReg cells, kRegN nodes per axis).
constexpr int kTile = 4;
constexpr int kTileShift = 2;
constexpr int kReg = kTile + 2;
constexpr int kRegN = kTile + 3;
constexpr int kRegNodes = kRegN * kRegN * kRegN;
constexpr int kBlock = 256;
constexpr int kNeighbours = 27;
constexpr int kCellBits = 10;  // packed cell: i | j << 10 | k << 20
constexpr int32_t kDeadCell = -1;
constexpr int kMaxDim = (1 << kCellBits) - 1;

// Device error flags (bitwise or).
enum : int32_t { kErrRange = 1 };

// Per-species particle arrays of one buffer. Positions: x/y/z (FP64, FP32
// absolute: cell units) or in-cell offsets (FP32 cell form, with `cell`).
struct PBuf {
  void *pos[3];
  void *vel[3];
  int32_t *cell;  // FP32 cell form only
  int64_t *ids;   // only when ids were loaded
};

struct Geom {
  int32_t kind;
  int32_t ci[3];    // floor of c (cell form)
  int32_t zfi;      // floor of z_flat (cell form)
  double c[3];      // sphere centre / crater (xc, yc, zc), cell units
  double cf[3];     // c - ci
  double r2;        // R^2 or Rc^2
  double z_flat;
  double zff;       // z_flat - zfi
};

struct StepParams {
  PBuf buf[PIC_MAX_SPECIES];
  const int64_t *off;      // [ns][ntiles + 1] particle range of each tile
  int32_t ns;
  int32_t nx, ny, nz;
  int32_t ntx, nty, ntz, ntiles;
  double qmdt[PIC_MAX_SPECIES];  // q/m*dt/h
  double chg[PIC_MAX_SPECIES];   // q*w
  int64_t chg_fixed[PIC_MAX_SPECIES];  // llrint(chg_T * 2^32), chg_T in the path's type
  double dt;
  Geom geom;
  const void *E;           // float4 / double4 per node
  void *rho;               // int64 / float / double per node
  int64_t *tally;          // [nbins][ns]
  int64_t *escaped;        // [6][ns]
  int64_t *stats;          // [0] particle-steps
  int32_t *err;
};

struct SortParams {
  PBuf src[PIC_MAX_SPECIES];
  PBuf dst[PIC_MAX_SPECIES];
  int64_t n_src[PIC_MAX_SPECIES];  // entries in the source buffer
  const int64_t *off_src;   // [ns][ntiles + 1] (sorted source) or null (unsorted)
  int64_t *off_dst;         // [ns][ntiles + 1]
  int32_t *count;           // [ns][ntiles]
  int32_t *cursor;          // [ns][ntiles]
  int32_t *hist;            // [ns][ntiles][27] per source tile
  int32_t ns;
  int32_t nx, ny, nz;
  int32_t ntx, nty, ntz, ntiles;
  int32_t has_ids;          // bit s: species s carries ids
};

struct LoadParams {
  const float *x[3];
  const float *v[3];
  const int64_t *ids;
  PBuf out;
  int64_t n;
  double origin[3];
  double h;
  int32_t nx, ny, nz;
  int32_t *bad;             // count of positions outside the box
};

// Launchers (return hipError_t of the launch).
hipError_t launch_step(int repr, int deposit, bool push, const StepParams &p, hipStream_t s);
hipError_t launch_sort_count(int repr, const SortParams &p, int64_t max_src, hipStream_t s);
hipError_t launch_sort_scan(const SortParams &p, hipStream_t s);
hipError_t launch_sort_scatter(int repr, const SortParams &p, int64_t max_src, hipStream_t s);
hipError_t launch_fill(void *ptr, int64_t bytes, hipStream_t s);
hipError_t launch_load_f32(int repr, const LoadParams &p, hipStream_t s);
hipError_t launch_find_ids(int repr, const PBuf &buf, int64_t n_buf, const int64_t *ids_sorted,
                           int64_t n_ids, int32_t *found, double *out6, hipStream_t s);
hipError_t launch_node_E_f32(int repr, const float *Ex, const float *Ey, const float *Ez,
                             void *E, int64_t nodes, int32_t *bad, hipStream_t s);

}  // namespace pic
