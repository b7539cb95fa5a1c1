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
// Largest workgroup count of a field-solve kernel (each strides over its
// grid's nodes; every consumer of a dot product adds this many partials)
constexpr int kFieldGroups = 2048;

// Workgroups of a field kernel over a grid of this many nodes: one node per
// thread up to kFieldGroups.
inline int32_t field_groups(int64_t nodes) {
  const int64_t g = (nodes + kBlock - 1) / kBlock;
  return (int32_t)(g < kFieldGroups ? g : kFieldGroups);
}
constexpr int kNeighbours = 27;
constexpr int kCellBits = 10;  // packed cell: i | j << 10 | k << 20
constexpr int32_t kDeadCell = -1;
constexpr int kMaxDim = (1 << kCellBits) - 1;

// FP32 cell form, stored offsets: an in-cell offset lies in [0, 1), so the two
// top bits of its FP32 pattern (the sign and the exponent's top bit) are
// zero. They carry the cell's coordinate within its tile along the same axis
// (0..kTile-1), so that a particle in a tile's region needs no stored cell
// index: the region gives the tile. The cell array holds full cells only
// where no region does: the overflow list and a freshly loaded buffer.
static_assert(kTile == 4, "two bits per axis hold the coordinate within a tile");
constexpr uint32_t kOffMask = 0x3fffffffu;
__host__ __device__ inline float off_pack(float o, int ci) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, o) |
                                       ((uint32_t)(ci & (kTile - 1)) << 30));
}
__host__ __device__ inline float off_value(float s) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, s) & kOffMask);
}
__host__ __device__ inline int off_sub(float s) {
  return (int)(__builtin_bit_cast(uint32_t, s) >> 30);
}

// Device flags (bitwise or).
enum : int32_t {
  kErrRange = 1,     // a particle position became non-finite / ran away
  kErrCapacity = 2,  // the overflow list itself overflowed (particles lost)
  kErrSurface = 4,   // a tally bin's collected charge reached 2^30 (surface source)
};

// Per-species particle arrays of one buffer. Positions: x/y/z (FP64, FP32
// absolute: cell units) or in-cell offsets (FP32 cell form: off_pack, with
// `cell` where no tile region implies the tile).
struct PBuf {
  void *pos[3];
  void *vel[3];
  int32_t *cell;  // FP32 cell form only
  int64_t *ids;   // only when ids were loaded
};

// Tile regions of the particle buffers, per species s and tile t (index
// s * ntiles + t). A layout (base, cap, sz) is fixed between re-bucketings and
// shared by both buffers; the counts describe one buffer's content:
//   [base, base + nst)              particles that stayed in the tile
//   [base + cap - arr, base + cap)   particles that arrived from other tiles
// with nst <= sz (stay zone) and arr <= cap - sz (arrival zone). Particles
// that found no room are kept in an overflow list at ovf_base[s].
struct Layout {
  int64_t *base;
  int32_t *cap;
  int32_t *sz;
};

struct Bins {
  Layout lay;               // the layout in use
  int32_t *nst[2];          // stayed counts, by buffer
  int32_t *arr[2];          // arrival counts, by buffer
  int32_t *ovf[2];          // [ns] overflow counts, by buffer; a species with a
                            // nonzero count ran out of spare room and wants
                            // its tile regions re-planned
  int64_t ovf_base[PIC_MAX_SPECIES];
  int32_t ovf_cap[PIC_MAX_SPECIES];
};

// Tile capacities after a re-bucketing of cnt particles: a stay zone with
// 1/16 spare and an arrival zone of 1/8 (+ constants for sparse tiles); the
// re-bucketing adds room for growth (sort_scan_kernel) when it fits.
__host__ __device__ inline int32_t stay_zone(int32_t cnt) { return cnt + cnt / 16 + 32; }
__host__ __device__ inline int32_t arrival_zone(int32_t cnt) { return cnt / 8 + 64; }
// Slots of one buffer for n particles over nt tiles (tile regions + overflow).
__host__ inline int64_t region_slots(int64_t n, int64_t nt) {
  return n + n / 16 + n / 8 + 96 * nt + 64;
}
__host__ inline int32_t overflow_slots(int64_t n) {
  const int64_t o = n / 32 + 4096;
  return (int32_t)(o > 0x3fffffff ? 0x3fffffff : o);
}

struct Geom {
  int32_t kind;
  int32_t patches;  // sphere surface patches per cube-face edge (0: one bin)
  int32_t ci[3];    // floor of c (cell form)
  int32_t zfi;      // floor of z_flat (cell form)
  double c[3];      // sphere centre / crater (xc, yc, zc), cell units
  double cf[3];     // c - ci
  double r2;        // R^2 or Rc^2
  double z_flat;
  double zff;       // z_flat - zfi
};

struct StepParams {
  PBuf buf[2][PIC_MAX_SPECIES];  // both particle buffers of every species
  Bins bins;
  int32_t cur;                // buffer holding the state at the start of the step
  int32_t remaining;          // batched runs: steps left (the step is skipped at 0)
  int32_t ovf_groups;         // workgroups that share the overflow list (ovf_groups_for)
  int32_t ns;
  int32_t nx, ny, nz;
  int32_t ntx, nty, ntz, ntiles;
  int32_t has_ids;            // bit s: species s carries ids
  int32_t reflect;            // bit f: box face f reflects
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

// Re-bucketing of the species in sel: every particle of the source (tile
// regions and overflow list, or an unsorted range [0, n_src) after a load) is
// written to the stay zone of its tile in the destination buffer, and the tile
// regions are re-planned; the commit pass then makes the new layout and stay
// counts those of the source buffer index (the host swaps the species' two
// buffers), so species outside sel are not touched at all.
struct SortParams {
  PBuf src[PIC_MAX_SPECIES];
  PBuf dst[PIC_MAX_SPECIES];
  int32_t sel;              // bit s: species s is re-bucketed
  int64_t n_src[PIC_MAX_SPECIES];  // unsorted source: entries
  int32_t unsorted;         // bit s: species s is an unsorted range [0, n_src)
  Bins bins;                // bins.lay: the source layout
  Layout dst_lay;           // the new layout, planned by the scan
  int32_t cur;              // buffer index of the source (its arr / ovf counters)
  int32_t *count;           // [ns][ntiles]
  int32_t *cursor;          // [ns][ntiles]
  int32_t *hist;            // [ns][ntiles + 1][27] per source tile (+ overflow block)
  int64_t region_cap[PIC_MAX_SPECIES];  // slots available for tile regions
  int32_t ns;
  int32_t nx, ny, nz;
  int32_t ntx, nty, ntz, ntiles;
  int32_t has_ids;          // bit s: species s carries ids
  int32_t *err;
  // [ns][ntiles] or null: particles that a source (photoemission) may add to
  // a tile in one step; the plan gives the tile's stay zone kInflowSteps
  // steps of it (the added particles stay) and its arrival zone two, when
  // that fits the buffer
  const int32_t *inflow;
};

// Step-kernel workgroups that share the overflow list (after the tiles'),
// each a contiguous part of it: one per 1000 tiles, 1 to 32 (small grids,
// which a batch runs by the dozen, keep a single one)
inline int32_t ovf_groups_for(int32_t ntiles) {
  const int32_t g = ntiles / 1000;
  return g < 1 ? 1 : (g > 32 ? 32 : g);
}

// Counters that many waves of one short launch add to are spread over this
// many slots (by workgroup), so that the atomics do not queue on one address.
constexpr int kCountSlots = 64;

// Steps of a source's inflow that a re-bucketing leaves room for.
constexpr int32_t kInflowSteps = 16;
__host__ __device__ inline int64_t inflow_room(int32_t per_step) {
  return (int64_t)per_step * (kInflowSteps + 2);
}
// Room for a tile that wanted a arrivals in the last step (a count of all
// attempts, overflowed ones included): its stay zone kDemandSteps more steps
// of them (they stay), its arrival zone twice as many, beyond the zones of
// its count.
constexpr int32_t kDemandSteps = 4;
__host__ __device__ inline int64_t demand_room(int32_t cnt, int32_t a) {
  const int64_t az = arrival_zone(cnt);
  return kDemandSteps * (int64_t)a + (2 * (int64_t)a > az ? 2 * (int64_t)a - az : 0);
}

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

// Injection of ambient particles through box faces (one thread per species,
// face, face cell and ghost slot), after the step kernel: appended to the
// arrival zones of the output buffer and deposited with global atomics.
// Photoemission from the crater terrain (cell units).
struct PhotoParams {
  int32_t s;                    // photoelectron species
  uint64_t seed;
  double sun[3];                // unit vector towards the Sun
  double rate;                  // (flux / w) h^2 dt: mean per column = rate I / n_z
  double vth;
  int64_t gmax;                 // slots per column: floor(largest mean) + 1
  double cx, cy, zc, rc, rc2, a2, z_flat;  // terrain
};

struct InjParams {
  PBuf out[PIC_MAX_SPECIES];  // the buffer the step wrote
  Bins bins;
  int32_t out_idx;            // its index (arrival / overflow counters)
  int32_t ns, nx, ny, nz, ntx, nty, ntiles;
  int32_t has_ids;
  int32_t step;
  uint64_t seed;
  double dt;
  double vth[PIC_MAX_SPECIES];     // cell units
  double u[PIC_MAX_SPECIES][3];    // cell units
  double L[PIC_MAX_SPECIES][6];    // ghost slab thickness
  double mean[PIC_MAX_SPECIES][6]; // ghosts per face cell
  int64_t gmax[PIC_MAX_SPECIES][6];  // ghost slots per face cell: floor(mean) + 1
  int64_t first[PIC_MAX_SPECIES * 6 + 1];  // thread prefix over (species, face)
  double chg[PIC_MAX_SPECIES];
  int64_t chg_fixed[PIC_MAX_SPECIES];
  Geom geom;
  void *rho;
  int64_t *tally;
  int64_t *injected;          // [ns][kCountSlots]: the host adds the slots
  int32_t *err;
  PhotoParams pe;             // photoemission (photo_kernel)
};

// Field solve on the nodes: Jacobi-preconditioned CG for the node-centred
// finite-volume Poisson operator (Dirichlet / zero-Neumann faces), then
// E = -grad phi into the context's node field.
struct FieldCtrl {
  int32_t converged;
  int32_t iters;
  double rr, bb;  // last squared residual norm, squared right-hand-side norm
};

// One level of the multigrid preconditioner (level 0: the PIC nodes; level
// l + 1 keeps every other node of level l, spacing doubled).
constexpr int kMaxLevels = 8;
constexpr int64_t kCoarseNodes = 1024;  // the coarsest level is solved exactly
struct MgLevel {
  int32_t n[3];
  int64_t sx, sy, nodes;
  int32_t mask;                // Dirichlet faces (homogeneous for corrections)
  double s;                    // eps / h_l^2
  double *e, *e2, *res, *rhs;  // correction (ping-pong), residual, right-hand side
  int32_t G;                   // workgroups of the level's kernels: one node per thread
  // object as an interface: level set and diagonal of A at the level's nodes;
  // side: 1 for a node whose six links lie outside the object (all of
  // permittivity eps), 2 for one whose links all lie inside, 0 for a node
  // with a link across the interface (only these read diag in the solve)
  double *psi, *diag;
  int8_t *side;
  double ih2;                  // 1 / h_l^2
  double scale;                // fine cells per cell of the level
};

// The object in the field problem (cell units of the PIC mesh).
struct FieldGeom {
  int32_t kind;                 // PIC_OBJ_SPHERE or PIC_OBJ_CRATER
  double c[3], r;               // sphere centre and radius; crater axis (c[0], c[1])
  double z_flat, a2, zc, rc2;   // crater: flat ground, rim radius^2, bowl centre, radius^2
  double rs;                    // sphere: radius of the surface points (sqrt of R^2)
  int32_t patches;
};

struct FieldParams {
  const void *rho;          // the deposit (raw: fixed int64 at 2^32, or float / double)
  double *x, *r, *z, *p, *Ap;
  double *part;             // [6][G]: pAp, rz0, rz1, rr0, rr1, bb
  FieldCtrl *ctrl;
  void *E;                  // float4 / double4 per node
  int32_t n[3];
  int64_t sx, sy, nodes;
  double h, eps, s;         // s = eps / h^2
  double rho_scale;         // raw deposit -> density (2^-32 / h^3 or 1 / h^3)
  int32_t mask;             // Dirichlet faces
  double g[6];
  double tol;
  int32_t max_iter;
  int32_t G;                // workgroups of the fine-grid kernels that form or use dot products (partials per sum)
  // multigrid preconditioner (levels >= 2: z = V-cycle(r)); 0 levels: Jacobi
  int32_t levels;
  MgLevel lv[kMaxLevels];
  const double *ainv;       // coarsest level: inverse operator on its m unknowns (m x m)
  const int32_t *umap;      // coarsest level: node of each unknown
  int32_t m;
  // object as an interface (iface): permittivities, level set and diagonal of
  // the fine level (= lv[0].psi / lv[0].diag), geometry; surface source
  int32_t iface;
  double e_in, e_out;
  const double *psi, *diag;
  const int8_t *side;
  double ih2;
  FieldGeom geo;
  const int64_t *rho_surf;  // fixed-point surface charge (nullable)
  // immersed finite elements on the fine grid (ife): per node the index of
  // its explicit row (-1: eps of its side times the reference links of its
  // parity), rows of 18 link coefficients c_pq = -A_pq and their sum; the
  // reference links of an interior node of parity 0 / 1 (eps = 1) and their
  // sums, over h^2
  int32_t ife;
  const int32_t *srow;
  const double *rows;
  double rl[2][18];
  double rld[2];
};

// The collected charge as a surface source: one thread per tally bin.
struct SurfParams {
  const int64_t *tally;     // [nbins][ns]
  double chg[PIC_MAX_SPECIES];  // q_s w_s
  int32_t ns;
  int64_t nbins;
  int32_t n[3];
  int64_t sx, sy;
  FieldGeom geo;
  int64_t *rho_surf;        // [nodes], cleared before
  int32_t *err;
};

// Batched runs: many contexts (slots) advanced by one launch per step. Work
// item b belongs to slot k with prefix[k] <= b < prefix[k + 1] (ntiles +
// ovf_groups items per slot); persistent workgroups take items from a counter. The slot
// descriptors live in device memory so that a captured graph can replay steps
// while the host changes the batch between replays.
struct BatchTable {
  StepParams *slots;       // [max_slots], ordered by step quota (descending)
  const int32_t *prefix;   // [nslots + 1]
  const int32_t *totals;   // [steps per run]: work items of each step (a prefix of the table)
  int32_t *istep;          // step of the run being executed
  int32_t *work;           // next work item of the current step
  int32_t nslots;
};

// Launchers (return hipError_t of the launch).
hipError_t launch_step(int repr, int deposit, bool push, const StepParams &p, hipStream_t s);
// one batched step: clear rho of every running slot, step them, advance them
// (refl: some slot has reflecting faces; else the kernel without that code)
hipError_t launch_batch_step(int repr, int deposit, bool refl, const BatchTable &t, int32_t grid,
                             hipStream_t s);
// the re-bucketing flags of the table's slots into out[nslots]
hipError_t launch_batch_flags(const BatchTable &t, int32_t *out, hipStream_t s);
hipError_t launch_sort_count(int repr, const SortParams &p, int64_t max_src, hipStream_t s);
hipError_t launch_sort_scan(const SortParams &p, hipStream_t s);
hipError_t launch_sort_scatter(int repr, const SortParams &p, int64_t max_src, hipStream_t s);
hipError_t launch_sort_commit(const SortParams &p, hipStream_t s);
hipError_t launch_fill(void *ptr, int64_t bytes, hipStream_t s);
// Zeroes rho (bytes) before a step and the overflow counts of the step's
// output buffer (ns of them), which the step's overflow workgroups add to.
hipError_t launch_step_clear(void *rho, int64_t bytes, int32_t *ovf_out, int32_t ns, hipStream_t s);
hipError_t launch_inject(int repr, int deposit, const InjParams &p, hipStream_t s);
hipError_t launch_photo(int repr, int deposit, const InjParams &p, hipStream_t s);
// field solve: init (+ initial convergence check), one CG iteration (parity o:
// the partials of the previous iteration), and E
hipError_t launch_field_init(int deposit, const FieldParams &p, hipStream_t s);
// (with levels >= 2 the multigrid form: z = V-cycle(r) between the update and
// the new direction)
hipError_t launch_field_iter(const FieldParams &p, int o, hipStream_t s);
// multigrid form, after init: z = V-cycle(r), p = z
hipError_t launch_field_mg_start(const FieldParams &p, hipStream_t s);
// object as an interface: level set of level l (once), diagonal of level l
hipError_t launch_field_psi(const FieldParams &p, int l, hipStream_t s);
hipError_t launch_field_diag(const FieldParams &p, int l, hipStream_t s);
hipError_t launch_surface_rho(const SurfParams &p, hipStream_t s);
// immersed finite elements: mark the nodes that need a row (count[0] += their
// number), then assemble the rows and the fine level's diagonal
hipError_t launch_ife_mark(const FieldParams &p, int32_t *srow, int32_t *count, hipStream_t s);
hipError_t launch_ife_rows(const FieldParams &p, int32_t *srow, double *rows, int32_t *next,
                           double *diag, hipStream_t s);
hipError_t launch_field_E(int repr, const FieldParams &p, hipStream_t s);
hipError_t launch_load_f32(int repr, const LoadParams &p, hipStream_t s);
// Sampled read-back: out6 receives, per found id, the position and velocity in
// cell units, or with phys (origin, h) the physical ones (origin + g h, u h).
struct PhysUnits {
  bool on;
  double origin[3];
  double h;
};
hipError_t launch_find_ids(int repr, const PBuf &buf, const Bins &bins, int32_t cur, int32_t s,
                           int32_t ntiles, int32_t ntx, int32_t nty, const int64_t *ids_sorted,
                           int64_t n_ids, int32_t *found, double *out6, const PhysUnits &phys,
                           hipStream_t st);

// Scratch of pic_get_particles_by_id_noalloc: a file-scope device array of
// kNoAllocBytes on every GPU the library runs on, laid out as the id list
// (8 B per id), the results (48 B per id) and the found flags (4 B per id),
// each at a fixed offset for PIC_NOALLOC_MAX_IDS ids.
constexpr int64_t kNoAllocIdsOff = 0;
constexpr int64_t kNoAllocOutOff = (int64_t)PIC_NOALLOC_MAX_IDS * 8;
constexpr int64_t kNoAllocFoundOff = (int64_t)PIC_NOALLOC_MAX_IDS * 56;
constexpr int64_t kNoAllocBytes = (int64_t)PIC_NOALLOC_MAX_IDS * 64;
// Its address on the current device (looked up once per device).
hipError_t noalloc_scratch(void **ptr);
hipError_t launch_node_E_f32(int repr, const float *Ex, const float *Ey, const float *Ez,
                             void *E, int64_t nodes, int32_t *bad, hipStream_t s);

}  // namespace pic
