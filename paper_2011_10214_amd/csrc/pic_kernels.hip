// HIP kernels of the particle-mesh hot path for gfx950 (CDNA4, wave64).
//
// step_kernel    one workgroup per tile of kTile^3 cells: stages the node field
//                of the tile grown by one cell in LDS, keeps a private rho for
//                the same region in LDS, and runs gather -> leapfrog push ->
//                box / object removal -> trilinear deposit for every particle
//                bucketed to the tile (the particle half of the PIC loop, §2.1;
//                removal at the outer boundary, §3.1.3; collection at the
//                object / terrain, §5.2.2). Particles that drifted outside the
//                staged region take the global-memory path.
// sort_*         re-bucket particles by tile every K steps (count -> scan ->
//                scatter), dropping removed particles. The order inside a tile
//                is whatever the atomics give: every result is invariant to it.
// inject, photo  ambient plasma entering at open faces and photoelectrons from
//                the sunlit terrain, appended to their tiles and deposited.
// batch_*        the step of many contexts in one persistent launch.
// load / node_E  convert caller arrays into the device representation.
// (The field solve is in pic_field.hip.)
//
// Arithmetic is written with explicit fma and compiled with contraction off, in
// the expression order of the method's definition, so that the FP64 form
// reproduces an FP64 CPU evaluation of the same definition bit for bit (and the
// FP32 forms an FP32 one).
#include <mutex>

#include "pic_device.h"

namespace pic {
namespace {

// Wave-aggregated LDS counter increment: every active lane adds 1 to
// ctr[key]; returns the counter value before the wave's adds plus the lane's
// rank among the active lanes with the same key. The loop runs over a
// wave-uniform mask of lanes still pending, one distinct key per iteration,
// so it terminates by construction (a loop that waits on a lane's own key
// equalling readfirstlane(key) would spin without side effects for the other
// lanes, and the compiler may assume it never does).
__device__ __forceinline__ int agg_add(int32_t *ctr, int key) {
  const int lane = __lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long pending = __ballot(1);
  int ret = 0;
  while (pending) {
    const int leader = __ffsll(pending) - 1;
    const int k0 = __shfl(key, leader);
    const unsigned long long m = __ballot(key == k0) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(&ctr[k0], (int)__popcll(m));
    base = __shfl(base, leader);
    if ((m >> lane) & 1ull) ret = base + (int)__popcll(m & below);
    pending &= ~m;
  }
  return ret;
}

// ------------------------------------------------------------------ geometry

template <class T>
struct GeomT {
  T c[3], r2, z_flat, cf[3], zff;
  int ci[3], zfi, kind, patches;
};

template <class T>
__device__ __forceinline__ GeomT<T> geom_of(const Geom &g) {
  GeomT<T> o;
  o.kind = g.kind;
  o.patches = g.patches;
  for (int d = 0; d < 3; ++d) {
    o.c[d] = (T)g.c[d];
    o.cf[d] = (T)g.cf[d];
    o.ci[d] = g.ci[d];
  }
  o.r2 = (T)g.r2;
  o.z_flat = (T)g.z_flat;
  o.zff = (T)g.zff;
  o.zfi = g.zfi;
  return o;
}

template <class T>
__device__ __forceinline__ T dist2(T dx, T dy, T dz) {
  return fmaT(dz, dz, fmaT(dy, dy, dx * dx));
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Surface patch of a collected particle at offset d from the sphere's centre,
// m patches per cube-face edge: the face of the largest |d_a| (ties to the
// lower axis; 2a for d_a < 0, else 2a + 1), the two other components in axis
// order divided by |d_a|, each cut into m equal intervals of [-1, 1].
template <class T>
__device__ __forceinline__ int sphere_patch(T dx, T dy, T dz, int m) {
  const T ax = dx < T(0) ? -dx : dx, ay = dy < T(0) ? -dy : dy, az = dz < T(0) ? -dz : dz;
  int a = 0;
  T big = ax, du = dy, dv = dz, dn = dx;
  if (ay > big) {
    a = 1;
    big = ay;
    du = dx;
    dv = dz;
    dn = dy;
  }
  if (az > big) {
    a = 2;
    big = az;
    du = dx;
    dv = dy;
    dn = dz;
  }
  const int face = 2 * a + (dn < T(0) ? 0 : 1);
  T su = T(0), sv = T(0);
  if (big > T(0)) {
    su = du / big;
    sv = dv / big;
  }
  const T half = (T)(0.5 * m);
  const int iu = clampi((int)floorT((su + T(1)) * half), 0, m - 1);
  const int iv = clampi((int)floorT((sv + T(1)) * half), 0, m - 1);
  return (face * m + iv) * m + iu;
}

// Object test on an absolute position (cell units); bin or -1.
template <class T>
__device__ __forceinline__ int hit_abs(const GeomT<T> &G, int nx, int ny, const T g[3]) {
  if (G.kind == PIC_OBJ_SPHERE) {
    const T dx = g[0] - G.c[0], dy = g[1] - G.c[1], dz = g[2] - G.c[2];
    if (!(dist2(dx, dy, dz) <= G.r2)) return -1;
    return G.patches ? sphere_patch(dx, dy, dz, G.patches) : 0;
  }
  if (G.kind == PIC_OBJ_CRATER) {
    bool hit = g[2] < T(0);
    if (!hit && g[2] <= G.z_flat) hit = dist2(g[0] - G.c[0], g[1] - G.c[1], g[2] - G.c[2]) >= G.r2;
    if (!hit) return -1;
    const int ix = clampi((int)floorT(g[0]), 0, nx - 1), iy = clampi((int)floorT(g[1]), 0, ny - 1);
    return ix + nx * iy;
  }
  return -1;
}

// Object test on a cell + offset position; a coordinate minus a constant
// c = ci + cf is (float)(i - ci) + (o - cf).
__device__ __forceinline__ int hit_cell(const GeomT<float> &G, int nx, int ny, const int i[3],
                                        const float o[3]) {
  if (G.kind == PIC_OBJ_SPHERE) {
    const float dx = (float)(i[0] - G.ci[0]) + (o[0] - G.cf[0]);
    const float dy = (float)(i[1] - G.ci[1]) + (o[1] - G.cf[1]);
    const float dz = (float)(i[2] - G.ci[2]) + (o[2] - G.cf[2]);
    if (!(dist2(dx, dy, dz) <= G.r2)) return -1;
    return G.patches ? sphere_patch(dx, dy, dz, G.patches) : 0;
  }
  if (G.kind == PIC_OBJ_CRATER) {
    bool hit = i[2] < 0;
    if (!hit) {
      const float zrel = (float)(i[2] - G.zfi) + (o[2] - G.zff);
      if (zrel <= 0.0f) {
        const float dx = (float)(i[0] - G.ci[0]) + (o[0] - G.cf[0]);
        const float dy = (float)(i[1] - G.ci[1]) + (o[1] - G.cf[1]);
        const float dz = (float)(i[2] - G.ci[2]) + (o[2] - G.cf[2]);
        hit = dist2(dx, dy, dz) >= G.r2;
      }
    }
    if (!hit) return -1;
    return clampi(i[0], 0, nx - 1) + nx * clampi(i[1], 0, ny - 1);
  }
  return -1;
}

// First box face crossed (x, y, z order, lower first) or -1. The crater's
// z-lower face is a collection, not an exit.
__device__ __forceinline__ int box_face(const int i[3], int nx, int ny, int nz, bool crater) {
  if (i[0] < 0) return 0;
  if (i[0] >= nx) return 1;
  if (i[1] < 0) return 2;
  if (i[1] >= ny) return 3;
  if (i[2] < 0 && !crater) return 4;
  if (i[2] >= nz) return 5;
  return -1;
}

template <class T>
__device__ __forceinline__ int box_face_abs(const T g[3], int nx, int ny, int nz, bool crater) {
  if (g[0] < T(0)) return 0;
  if (g[0] >= (T)nx) return 1;
  if (g[1] < T(0)) return 2;
  if (g[1] >= (T)ny) return 3;
  if (g[2] < T(0) && !crater) return 4;
  if (g[2] >= (T)nz) return 5;
  return -1;
}

// Mirror about the reflecting faces (bit f of mask), axes x, y, z in turn, with
// the normal velocity negated; a particle mirrored exactly onto a max face is
// put just inside (the largest value below n).
__device__ __forceinline__ float below(float x) { return __int_as_float(__float_as_int(x) - 1); }
__device__ __forceinline__ double below(double x) {
  return __longlong_as_double(__double_as_longlong(x) - 1);
}

template <class T>
__device__ __forceinline__ void reflect_abs(int mask, const int n[3], T g[3], T u[3]) {
  for (int d = 0; d < 3; ++d) {
    if (((mask >> (2 * d)) & 1) && g[d] < T(0)) {
      g[d] = -g[d];
      u[d] = -u[d];
    }
    if (((mask >> (2 * d + 1)) & 1) && g[d] >= (T)n[d]) {
      g[d] = (T)(2 * n[d]) - g[d];
      if (g[d] >= (T)n[d]) g[d] = below((T)n[d]);
      u[d] = -u[d];
    }
  }
}

// The same on a cell + offset position: m - (i + o) = (m - i - 1) + (1 - o).
__device__ __forceinline__ void reflect_cell(int mask, const int n[3], int i[3], float o[3],
                                             float u[3]) {
  for (int d = 0; d < 3; ++d) {
    const bool lo = ((mask >> (2 * d)) & 1) && i[d] < 0;
    const bool hi = ((mask >> (2 * d + 1)) & 1) && i[d] >= n[d];
    if (!lo && !hi) continue;
    const int m = lo ? 0 : 2 * n[d];
    if (o[d] == 0.0f) {
      i[d] = m - i[d];
    } else {
      i[d] = m - i[d] - 1;
      o[d] = 1.0f - o[d];
      if (o[d] == 1.0f) {
        o[d] = 0.0f;
        i[d] += 1;
      }
    }
    if (hi && i[d] >= n[d]) {
      i[d] = n[d] - 1;
      o[d] = below(1.0f);
    }
    u[d] = -u[d];
  }
}

// ------------------------------------------------------------------ injection random numbers

// SplitMix64 (Steele, Lea and Flood, 2014) used as a counter-based generator:
// draw d of a key is the output function applied to key + (d + 1) * gamma.
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// key of a face cell; its ghost j (j >= 1) or count draw (j = 0) has key
// sm_mix(cell key ^ j)
__device__ __forceinline__ uint64_t inj_cell_key(uint64_t seed, int32_t step, int s, int f,
                                                 int64_t cell) {
  uint64_t k = sm_mix(seed + kGamma);
  k = sm_mix(k ^ (uint64_t)(uint32_t)step);
  k = sm_mix(k ^ (uint64_t)(s * 8 + f));
  return sm_mix(k ^ (uint64_t)cell);
}

// uniform in [0, 1) on the 2^-53 grid
__device__ __forceinline__ double inj_uniform(uint64_t key, uint64_t d) {
  return (double)(sm_mix(key + (d + 1) * kGamma) >> 11) * 0x1.0p-53;
}

// ln x = e ln 2 + 2 atanh((m - 1)/(m + 1)), x = m 2^e, m in [sqrt(1/2), sqrt(2));
// atanh by its Taylor series to s^23 (correctly rounded operations only).
__device__ double ln_series(double x) {
  int e = 0;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double t = s * s;
  double p = 1.0 / 23.0;
#pragma unroll
  for (int k = 21; k >= 1; k -= 2) p = p * t + 1.0 / (double)k;
  return (double)e * 0.69314718055994530942 + 2.0 * s * p;
}

// One pair of standard normals by Marsaglia's polar method; *d counts the
// draws and *attempts the pairs tried (at most 64 over the three normals of a
// ghost; none left gives zeros).
__device__ void normal_pair(uint64_t key, uint64_t *d, int *attempts, double *z0, double *z1) {
  *z0 = 0.0;
  *z1 = 0.0;
  for (; *attempts < 64;) {
    ++*attempts;
    const double a = 2.0 * inj_uniform(key, (*d)++) - 1.0;
    const double b = 2.0 * inj_uniform(key, (*d)++) - 1.0;
    const double r = a * a + b * b;
    if (!(r > 0.0 && r < 1.0)) continue;
    const double f = __builtin_sqrt(-2.0 * ln_series(r) / r);
    *z0 = a * f;
    *z1 = b * f;
    return;
  }
}

// ------------------------------------------------------------------ tile regions

// Source range of a workgroup: a tile's stayed + arrived particles, or (t ==
// ntiles) the overflow list. Index k in [0, n1 + na) maps to base + off(k).
struct Src {
  int64_t base;
  int32_t n1;   // stayed (tile) / listed (overflow)
  int32_t na;   // arrived
  int32_t gap;  // offset of the arrival zone's first entry minus n1
};

__device__ __forceinline__ Src src_of(const Bins &B, int cur, int s, int t, int nt) {
  Src r;
  if (t < nt) {
    const int64_t i = (int64_t)s * nt + t;
    r.base = B.lay.base[i];
    const int32_t cap = B.lay.cap[i], sz = B.lay.sz[i];
    const int32_t n1 = B.nst[cur][i], na = B.arr[cur][i];
    r.n1 = n1 < sz ? n1 : sz;
    r.na = na < cap - sz ? na : cap - sz;
    r.gap = cap - r.na - r.n1;
  } else {
    r.base = B.ovf_base[s];
    const int32_t n = B.ovf[cur][s];
    r.n1 = n < B.ovf_cap[s] ? n : B.ovf_cap[s];
    r.na = 0;
    r.gap = 0;
  }
  return r;
}

__device__ __forceinline__ int32_t src_off(const Src &r, int32_t k) { return k < r.n1 ? k : k + r.gap; }

__device__ __forceinline__ int tile_of_cell(const int ci[3], int ntx, int nty) {
  return (ci[0] >> kTileShift) + ntx * ((ci[1] >> kTileShift) + nty * (ci[2] >> kTileShift));
}

template <class T>
struct Particle {
  int32_t cell;  // packed cell (cell form)
  T x[3];        // stored offsets (cell form: off_pack) or positions in cell units
  T u[3];
  int64_t id;
};

// Writes particle v to slot q of B. In the FP32 cell form v.x holds the
// stored offsets (off_pack: with the cell's coordinates within its tile), and
// the full cell is written too for a slot at or past full_from (the start of
// the overflow list, where no region implies the tile).
template <int R>
__device__ __forceinline__ void store_particle(const PBuf &B, int64_t q, const Particle<typename RealOf<R>::T> &v,
                                               bool ids, int64_t full_from) {
  using T = typename RealOf<R>::T;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ((T *)B.pos[d])[q] = v.x[d];
    ((T *)B.vel[d])[q] = v.u[d];
  }
  if constexpr (R == PIC_REPR_FP32_CELL) {
    if (q >= full_from) B.cell[q] = v.cell;
  }
  if (ids) B.ids[q] = v.id;
}

// Slot for a particle entering tile tn of the output buffer: its arrival zone,
// else the overflow list (whose nonzero count requests a re-bucketing). -1 if
// even the overflow list is full (the particle is lost; reported as an error).
__device__ __forceinline__ int64_t arrival_slot(const Bins &B, int out, int s, int tn, int nt,
                                                int32_t *err) {
  const int64_t i = (int64_t)s * nt + tn;
  const int32_t k = atomicAdd(&B.arr[out][i], 1);
  const int32_t cap = B.lay.cap[i], room = cap - B.lay.sz[i];
  if (k < room) return B.lay.base[i] + cap - 1 - k;
  const int32_t o = atomicAdd(&B.ovf[out][s], 1);
  if (o < B.ovf_cap[s]) return B.ovf_base[s] + o;
  atomicOr(err, kErrCapacity);
  return -1;
}

// ------------------------------------------------------------------ step kernel

// rint(a) for 0 <= a < 2^52 as an unsigned 64-bit integer, split exactly into
// 32-bit halves in the arithmetic type: hi = floor(r 2^-32), lo = r - hi 2^32
// (both exact: r is an integer with at most 24 / 53 significant bits).
template <class T>
__device__ __forceinline__ unsigned long long fix_mag(T a) {
  const T r = rintT(a);
  const T hf = floorT(r * T(2.3283064365386963e-10));
  const T lf = fmaT(hf, -two32<T>(), r);
  const unsigned hi = (unsigned)hf, lo = (unsigned)lf;
  return ((unsigned long long)hi << 32) | (unsigned long long)lo;
}

// One workgroup per tile (plus one for the overflow list). With PUSH, every
// particle is pushed and written to the output buffer: compacted into its
// tile's stay zone if it stayed in the tile, into the arrival zone of its new
// tile if it moved, nowhere if it was removed -- so the particles are
// re-bucketed by tile at every step, in the same pass. Without PUSH only the
// deposit of the current positions is made. REFL: the code of reflecting box
// faces is compiled in (taken where P.reflect sets a face); a context without
// them runs the kernel without it, which needs fewer registers.
template <int R, int D, bool PUSH, bool REFL = true>
__device__ __forceinline__ void step_block(const StepParams &P, const int block) {
  using T = typename RealOf<R>::T;
  using V4 = typename Vec4Of<T>::type;
  using A = typename AccOf<D>::type;
  constexpr bool kCell = R == PIC_REPR_FP32_CELL;
  constexpr bool kFixed = D == PIC_DEP_FIXED64;

  __shared__ V4 sE[PUSH ? kRegNodes : 1];
  // private rho of the staged region; the fixed-point mode keeps the charge
  // magnitudes of positive and negative species apart (no sign handling per
  // contribution) and subtracts them at the flush
  __shared__ A sAcc[kFixed ? 2 : 1][kRegNodes];
  __shared__ int32_t sEsc[6 * PIC_MAX_SPECIES];
  __shared__ int32_t sAbs[PIC_MAX_SPECIES];
  __shared__ int32_t sStay[PIC_MAX_SPECIES];
  __shared__ int32_t sAlive;
  __shared__ Src sSrc[PIC_MAX_SPECIES];
  __shared__ int32_t sTotal;
  // movers of the current species, staged so that they leave the workgroup as
  // contiguous runs per destination tile (one reservation per destination);
  // the rest of a tile's movers reserve one slot each. The 4-byte forms stage
  // as many as fit with five workgroups per CU (30.6 KB of LDS each).
  constexpr int kMovers = sizeof(T) == 4 ? 400 : 160;
  __shared__ Particle<T> sMv[PUSH ? kMovers : 1];
  __shared__ int32_t sMvDst[PUSH ? kMovers : 1];   // destination tile
  __shared__ int16_t sMvRel[PUSH ? kMovers : 1];   // its 27-neighbour index, or -1
  __shared__ int16_t sMvRank[PUSH ? kMovers : 1];  // rank among movers to it
  __shared__ int32_t sMvN;
  __shared__ int32_t sRelCnt[kNeighbours];
  __shared__ int32_t sRelRes[kNeighbours];

  const int nt = P.ntiles;
  const bool ovf_block = block >= nt;  // one of the P.ovf_groups overflow workgroups
  // workgroups take tiles in the order of their regions in memory, so the
  // workgroups resident at any time stream one contiguous window of HBM
  const int t = block;
  const int cur = P.cur, out = 1 - P.cur;
  if (threadIdx.x == 0) {
    int total = 0;
    for (int s = 0; s < P.ns; ++s) {
      Src r = src_of(P.bins, cur, s, ovf_block ? nt : t, nt);
      if (ovf_block) {  // part c of the list: [n c / K, n (c + 1) / K)
        const int64_t c = block - nt;
        const int32_t lo = (int32_t)((int64_t)r.n1 * c / P.ovf_groups);
        const int32_t hi = (int32_t)((int64_t)r.n1 * (c + 1) / P.ovf_groups);
        r.base += lo;
        r.n1 = hi - lo;
      }
      sSrc[s] = r;
      total += r.n1 + r.na;
    }
    sTotal = total;
  }
  __syncthreads();
  if (sTotal == 0) {  // uniform over the workgroup
    // nothing stayed: the output's stayed counts of this tile are zero
    if (PUSH && !ovf_block && threadIdx.x < P.ns) P.bins.nst[out][(int64_t)threadIdx.x * nt + t] = 0;
    return;
  }
  if (PUSH && !ovf_block && threadIdx.x == 0) {
    // the input counters are consumed: they count the next step's arrivals
    // (the overflow count, which every overflow workgroup reads, is cleared
    // before the next step instead)
    for (int s = 0; s < P.ns; ++s) P.bins.arr[cur][(int64_t)s * nt + t] = 0;
  }

  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int sx = nx + 1, sy = (nx + 1) * (ny + 1);
  int rx0, ry0, rz0;
  int tx = -4, ty = -4, tz = -4;  // no neighbours for the overflow list
  if (ovf_block) {  // nothing is staged: every access takes the global path
    rx0 = ry0 = rz0 = -(1 << 20);
  } else {
    tx = t % P.ntx;
    ty = (t / P.ntx) % P.nty;
    tz = t / (P.ntx * P.nty);
    rx0 = tx * kTile - 1;
    ry0 = ty * kTile - 1;
    rz0 = tz * kTile - 1;
  }
  const V4 *__restrict__ gE = (const V4 *)P.E;
  A *__restrict__ gRho = (A *)P.rho;

  for (int n = threadIdx.x; n < kRegNodes; n += kBlock) {
    const int a = n % kRegN, b = (n / kRegN) % kRegN, c = n / (kRegN * kRegN);
    const int gi = rx0 + a, gj = ry0 + b, gk = rz0 + c;
    if constexpr (PUSH) {
      V4 e;
      e.x = 0;
      e.y = 0;
      e.z = 0;
      e.w = 0;
      if (gi >= 0 && gi <= nx && gj >= 0 && gj <= ny && gk >= 0 && gk <= nz)
        e = gE[gi + sx * gj + sy * gk];
      sE[n] = e;
    }
    sAcc[0][n] = A(0);
    if constexpr (kFixed) sAcc[1][n] = A(0);
  }
  if (threadIdx.x < 6 * PIC_MAX_SPECIES) sEsc[threadIdx.x] = 0;
  if (threadIdx.x < PIC_MAX_SPECIES) {
    sAbs[threadIdx.x] = 0;
    sStay[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) {
    sAlive = 0;
    sMvN = 0;
  }
  if (threadIdx.x < kNeighbours) sRelCnt[threadIdx.x] = 0;
  __syncthreads();

  const GeomT<T> G = geom_of<T>(P.geom);
  const bool crater = P.geom.kind == PIC_OBJ_CRATER;
  // one sphere bin: counted per wave into LDS; patches: per particle
  const bool sphere = P.geom.kind == PIC_OBJ_SPHERE && P.geom.patches == 0;
  const T dt = (T)P.dt;
  const int lane = __lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  int alive_here = 0;

  for (int s = 0; s < P.ns; ++s) {
    const Src src = sSrc[s];
    const int32_t np = src.n1 + src.na;
    if (np == 0) continue;
    const T qmdt = (T)P.qmdt[s];
    const T chg = (T)P.chg[s];
    const bool neg = chg < T(0);
    // |chg| 2^32 (exact scaling), and llrint(|chg| 2^32)
    const T amag = absT(chg) * two32<T>();
    const unsigned long long fmag =
        (unsigned long long)(P.chg_fixed[s] < 0 ? -P.chg_fixed[s] : P.chg_fixed[s]);
    A *__restrict__ sTile = sAcc[kFixed && neg ? 1 : 0];
    const bool ids = (P.has_ids >> s) & 1;
    // uniform bases at the region start; lanes index with a 32-bit offset
    const PBuf In = P.buf[cur][s];
    const T *__restrict__ X0 = (const T *)In.pos[0] + src.base;
    const T *__restrict__ X1 = (const T *)In.pos[1] + src.base;
    const T *__restrict__ X2 = (const T *)In.pos[2] + src.base;
    const T *__restrict__ U0 = (const T *)In.vel[0] + src.base;
    const T *__restrict__ U1 = (const T *)In.vel[1] + src.base;
    const T *__restrict__ U2 = (const T *)In.vel[2] + src.base;
    // full cells only in the overflow list; a region implies its tile
    const int32_t *__restrict__ CELL = kCell && ovf_block ? In.cell + src.base : nullptr;
    const int64_t *__restrict__ ID = ids ? In.ids + src.base : nullptr;
    const int64_t sbase = ovf_block ? 0 : P.bins.lay.base[(int64_t)s * nt + t];
    const int32_t ssz = ovf_block ? 0 : P.bins.lay.sz[(int64_t)s * nt + t];

    auto load = [&](int32_t k) {
      const int32_t o = src_off(src, k);
      Particle<T> q;
      q.cell = kCell && ovf_block ? CELL[o] : 0;
      q.x[0] = X0[o];
      q.x[1] = X1[o];
      q.x[2] = X2[o];
      q.u[0] = U0[o];
      q.u[1] = U1[o];
      q.u[2] = U2[o];
      q.id = ids ? ID[o] : 0;
      return q;
    };

    auto process = [&](Particle<T> &q) {
      int ci[3];
      T f[3];  // in-cell offsets
      T *u = q.u;
      if constexpr (kCell) {
        if (ovf_block) {
          if (q.cell < 0) return;  // not a particle (defensive: never written)
          ci[0] = q.cell & kMaxDim;
          ci[1] = (q.cell >> kCellBits) & kMaxDim;
          ci[2] = q.cell >> (2 * kCellBits);
        } else {
          ci[0] = (tx << kTileShift) + off_sub(q.x[0]);
          ci[1] = (ty << kTileShift) + off_sub(q.x[1]);
          ci[2] = (tz << kTileShift) + off_sub(q.x[2]);
        }
        f[0] = off_value(q.x[0]);
        f[1] = off_value(q.x[1]);
        f[2] = off_value(q.x[2]);
      } else {
        if (q.x[0] < T(0)) return;
        for (int d = 0; d < 3; ++d) {
          ci[d] = (int)floorT(q.x[d]);
          f[d] = q.x[d] - (T)ci[d];
        }
      }
      ++alive_here;

      if constexpr (PUSH) {
        T W[8];
        weights(f, W);
        T Ep[3];
        const int li = ci[0] - rx0, lj = ci[1] - ry0, lk = ci[2] - rz0;
#define PIC_ACC(n, e)             \
  Ep[0] = fmaT(W[n], e.x, Ep[0]); \
  Ep[1] = fmaT(W[n], e.y, Ep[1]); \
  Ep[2] = fmaT(W[n], e.z, Ep[2]);
        if ((unsigned)li < (unsigned)kReg && (unsigned)lj < (unsigned)kReg &&
            (unsigned)lk < (unsigned)kReg) {
          const int l0 = li + kRegN * (lj + kRegN * lk);
          const V4 e0 = sE[l0], e1 = sE[l0 + 1], e2 = sE[l0 + kRegN], e3 = sE[l0 + kRegN + 1];
          const V4 e4 = sE[l0 + kRegN * kRegN], e5 = sE[l0 + kRegN * kRegN + 1];
          const V4 e6 = sE[l0 + kRegN * kRegN + kRegN], e7 = sE[l0 + kRegN * kRegN + kRegN + 1];
          Ep[0] = W[0] * e0.x;
          Ep[1] = W[0] * e0.y;
          Ep[2] = W[0] * e0.z;
          PIC_ACC(1, e1)
          PIC_ACC(2, e2)
          PIC_ACC(3, e3)
          PIC_ACC(4, e4)
          PIC_ACC(5, e5)
          PIC_ACC(6, e6)
          PIC_ACC(7, e7)
        } else {
          const int g0 = ci[0] + sx * ci[1] + sy * ci[2];
          const V4 e0 = gE[g0], e1 = gE[g0 + 1], e2 = gE[g0 + sx], e3 = gE[g0 + sx + 1];
          const V4 e4 = gE[g0 + sy], e5 = gE[g0 + sy + 1], e6 = gE[g0 + sy + sx],
                   e7 = gE[g0 + sy + sx + 1];
          Ep[0] = W[0] * e0.x;
          Ep[1] = W[0] * e0.y;
          Ep[2] = W[0] * e0.z;
          PIC_ACC(1, e1)
          PIC_ACC(2, e2)
          PIC_ACC(3, e3)
          PIC_ACC(4, e4)
          PIC_ACC(5, e5)
          PIC_ACC(6, e6)
          PIC_ACC(7, e7)
        }
#undef PIC_ACC
        // leapfrog: kick with the gathered field, then drift
        u[0] = fmaT(qmdt, Ep[0], u[0]);
        u[1] = fmaT(qmdt, Ep[1], u[1]);
        u[2] = fmaT(qmdt, Ep[2], u[2]);
        bool bad = false;
        if constexpr (kCell) {
          for (int d = 0; d < 3; ++d) {
            T op = fmaT(u[d], dt, f[d]);
            T sh = floorT(op);
            op = op - sh;
            if (op == T(1)) {  // a tiny negative offset rounded up to 1 after the shift
              op = T(0);
              sh = sh + T(1);
            }
            bad |= !(absT(sh) <= T(1048576));  // also catches NaN / Inf
            f[d] = op;
            ci[d] += bad ? 0 : (int)sh;
          }
          if (REFL && P.reflect && !bad) {
            const int dims[3] = {nx, ny, nz};
            reflect_cell(P.reflect, dims, ci, f, u);
          }
        } else {
          for (int d = 0; d < 3; ++d) {
            q.x[d] = fmaT(u[d], dt, q.x[d]);
            bad |= !finiteT(q.x[d]);
          }
          if (REFL && P.reflect && !bad) {
            const int dims[3] = {nx, ny, nz};
            reflect_abs(P.reflect, dims, q.x, u);
          }
        }
        int face = -1, bin = -1;
        if (!bad) {
          if constexpr (kCell) {
            face = box_face(ci, nx, ny, nz, crater);
            if (face < 0) bin = hit_cell(G, nx, ny, ci, f);
          } else {
            face = box_face_abs(q.x, nx, ny, nz, crater);
            if (face < 0) bin = hit_abs(G, nx, ny, q.x);
          }
        }
        if (bad) atomicOr(P.err, kErrRange);
        if (face >= 0) atomicAdd(&sEsc[face * PIC_MAX_SPECIES + s], 1);
        if (sphere) {  // wave reduction of the collected count
          const unsigned long long m = __ballot(bin >= 0);
          if (m && lane == __ffsll(__ballot(1)) - 1) atomicAdd(&sAbs[s], (int)__popcll(m));
        } else if (bin >= 0) {
          atomicAdd((unsigned long long *)&P.tally[(long long)bin * P.ns + s], 1ull);
        }
        const bool removed = bad || face >= 0 || bin >= 0;
        if constexpr (kCell) {
          q.x[0] = off_pack(f[0], ci[0]);
          q.x[1] = off_pack(f[1], ci[1]);
          q.x[2] = off_pack(f[2], ci[2]);
          q.cell = pack_cell(ci[0], ci[1], ci[2]);
        } else if (!removed) {
          for (int d = 0; d < 3; ++d) {
            ci[d] = (int)floorT(q.x[d]);
            f[d] = q.x[d] - (T)ci[d];
          }
        }
        // re-bucket: stayed particles are compacted into the tile's stay zone
        // (one LDS reservation per wave), movers go to their new tile
        const int tn = removed ? -1 : tile_of_cell(ci, P.ntx, P.nty);
        const bool stay = !ovf_block && tn == t;
        const unsigned long long ms = __ballot(stay);
        int64_t slot = -1;
        if (ms) {
          const int leader = __ffsll(__ballot(1)) - 1;
          int wbase = 0;
          if (lane == leader) wbase = atomicAdd(&sStay[s], (int)__popcll(ms));
          wbase = __shfl(wbase, leader);
          const int k = wbase + (int)__popcll(ms & below);
          if (stay && k < ssz) slot = sbase + k;
        }
        const bool mover = !removed && !stay;
        const unsigned long long mm = __ballot(mover);
        if (mm) {  // stage the wave's movers in LDS (one reservation per wave)
          const int leader = __ffsll(__ballot(1)) - 1;
          int wbase = 0;
          if (lane == leader) wbase = atomicAdd(&sMvN, (int)__popcll(mm));
          wbase = __shfl(wbase, leader);
          const int k = wbase + (int)__popcll(mm & below);
          if (mover && k < kMovers) {
            sMv[k] = q;
            sMvDst[k] = tn;
            int tc[3] = {ci[0] >> kTileShift, ci[1] >> kTileShift, ci[2] >> kTileShift};
            const int dx = tc[0] - tx, dy = tc[1] - ty, dz = tc[2] - tz;
            sMvRel[k] = (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1)
                            ? (int16_t)-1
                            : (int16_t)((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
            slot = -2;  // staged
          }
        }
        if (!removed && slot == -1) {
          if (stay) {  // the stay zone is full
            const int32_t o = atomicAdd(&P.bins.ovf[out][s], 1);
            if (o < P.bins.ovf_cap[s]) slot = P.bins.ovf_base[s] + o;
            else atomicOr(P.err, kErrCapacity);
          } else {  // the staging area is full: write it directly
            slot = arrival_slot(P.bins, out, s, tn, nt, P.err);
          }
        }
        if (slot >= 0) store_particle<R>(P.buf[out][s], slot, q, ids, P.bins.ovf_base[s]);
        if (removed) return;
      }

      // trilinear deposit at the (new) position (the cell form takes the
      // offsets back from the stored values, so that only those stay live
      // across the write)
      if constexpr (kCell && PUSH) {
        f[0] = off_value(q.x[0]);
        f[1] = off_value(q.x[1]);
        f[2] = off_value(q.x[2]);
      }
      T W[8];
      weights(f, W);
      const int li = ci[0] - rx0, lj = ci[1] - ry0, lk = ci[2] - rz0;
      const bool local = (unsigned)li < (unsigned)kReg && (unsigned)lj < (unsigned)kReg &&
                         (unsigned)lk < (unsigned)kReg;
      int idx[8];
      {
        const int b0 = local ? li + kRegN * (lj + kRegN * lk) : ci[0] + sx * ci[1] + sy * ci[2];
        const int ox = local ? kRegN : sx, oz = local ? kRegN * kRegN : sy;
        idx[0] = b0;
        idx[1] = b0 + 1;
        idx[2] = b0 + ox;
        idx[3] = b0 + ox + 1;
        idx[4] = b0 + oz;
        idx[5] = b0 + oz + 1;
        idx[6] = b0 + oz + ox;
        idx[7] = b0 + oz + ox + 1;
      }
      if constexpr (kFixed) {
        // magnitudes rint(|chg| W 2^32) (rounding is sign symmetric), the
        // remainder on corner 7; negative species go to the second tile
        unsigned long long C[8];
        unsigned long long sum = 0;
#pragma unroll
        for (int n = 0; n < 7; ++n) {
          C[n] = fix_mag<T>(amag * W[n]);
          sum += C[n];
        }
        C[7] = fmag - sum;
        if (local) {
#pragma unroll
          for (int n = 0; n < 8; ++n) atomicAdd(&sTile[idx[n]], C[n]);
        } else {
#pragma unroll
          for (int n = 0; n < 8; ++n) atomicAdd(&gRho[idx[n]], neg ? 0ull - C[n] : C[n]);
        }
      } else {
        A C[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) C[n] = (A)(chg * W[n]);
        if (local) {
          // workgroup-scope float add on the LDS tile (an LDS atomic; the
          // device-scope atomicAdd would go through the flat path)
#pragma unroll
          for (int n = 0; n < 8; ++n)
            __hip_atomic_fetch_add(&sTile[idx[n]], C[n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
#pragma unroll
          for (int n = 0; n < 8; ++n) unsafeAtomicAdd(&gRho[idx[n]], C[n]);
        }
      }
    };

    // two particles per lane per iteration: both loads are issued before
    // either is processed
    for (int32_t k = threadIdx.x; k < np; k += 2 * kBlock) {
      const int32_t k2 = k + kBlock;
      const bool two = k2 < np;
      Particle<T> a = load(k), b;
      if (two) b = load(k2);
      process(a);
      if (two) process(b);
    }

    if constexpr (PUSH) {
      // flush the staged movers: count them per destination, reserve one run
      // per destination in its arrival zone, write the runs
      __syncthreads();
      const int nm = sMvN < kMovers ? sMvN : kMovers;
      for (int i = threadIdx.x; i < nm; i += kBlock) {
        const int rel = sMvRel[i];
        if (rel >= 0) sMvRank[i] = (int16_t)agg_add(sRelCnt, rel);
      }
      __syncthreads();
      if (threadIdx.x < kNeighbours) {
        const int c = sRelCnt[threadIdx.x];
        int r = 0;
        if (c) {
          const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
          const int tn = (tx + dx) + P.ntx * ((ty + dy) + P.nty * (tz + dz));
          r = atomicAdd(&P.bins.arr[out][(int64_t)s * nt + tn], c);
        }
        sRelRes[threadIdx.x] = r;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < nm; i += kBlock) {
        const int rel = sMvRel[i], tn = sMvDst[i];
        int64_t slot;
        if (rel >= 0) {
          const int64_t j = (int64_t)s * nt + tn;
          const int32_t k = sRelRes[rel] + sMvRank[i];
          const int32_t cap = P.bins.lay.cap[j], room = cap - P.bins.lay.sz[j];
          if (k < room) {
            slot = P.bins.lay.base[j] + cap - 1 - k;
          } else {
            const int32_t o = atomicAdd(&P.bins.ovf[out][s], 1);
            slot = o < P.bins.ovf_cap[s] ? P.bins.ovf_base[s] + o : -1;
            if (slot < 0) atomicOr(P.err, kErrCapacity);
          }
        } else {
          slot = arrival_slot(P.bins, out, s, tn, nt, P.err);
        }
        if (slot >= 0) store_particle<R>(P.buf[out][s], slot, sMv[i], ids, P.bins.ovf_base[s]);
      }
      __syncthreads();
      if (threadIdx.x == 0) sMvN = 0;
      if (threadIdx.x < kNeighbours) sRelCnt[threadIdx.x] = 0;
      __syncthreads();
    }
  }

  atomicAdd(&sAlive, alive_here);
  __syncthreads();
  for (int n = threadIdx.x; n < kRegNodes; n += kBlock) {
    A v = sAcc[0][n];
    if constexpr (kFixed) v -= sAcc[1][n];
    if (v == A(0)) continue;
    const int a = n % kRegN, b = (n / kRegN) % kRegN, c = n / (kRegN * kRegN);
    const int gi = rx0 + a, gj = ry0 + b, gk = rz0 + c;
    if (gi < 0 || gi > nx || gj < 0 || gj > ny || gk < 0 || gk > nz) continue;
    if constexpr (kFixed) atomicAdd(&gRho[gi + sx * gj + sy * gk], v);
    else unsafeAtomicAdd(&gRho[gi + sx * gj + sy * gk], v);
  }
  if (threadIdx.x < 6 * PIC_MAX_SPECIES) {
    const int face = threadIdx.x / PIC_MAX_SPECIES, s = threadIdx.x % PIC_MAX_SPECIES;
    const int v = sEsc[threadIdx.x];
    if (v) atomicAdd((unsigned long long *)&P.escaped[face * P.ns + s], (unsigned long long)v);
  }
  if (sphere && threadIdx.x < PIC_MAX_SPECIES && sAbs[threadIdx.x])
    atomicAdd((unsigned long long *)&P.tally[threadIdx.x], (unsigned long long)sAbs[threadIdx.x]);
  if (PUSH && !ovf_block && threadIdx.x < P.ns) {
    const int32_t sz = P.bins.lay.sz[(int64_t)threadIdx.x * nt + t];
    const int32_t k = sStay[threadIdx.x];
    P.bins.nst[out][(int64_t)threadIdx.x * nt + t] = k < sz ? k : sz;
  }
  if (PUSH && threadIdx.x == 0 && sAlive)
    atomicAdd((unsigned long long *)&P.stats[0], (unsigned long long)sAlive);
}

// The FP32 cell form runs at 5 waves per SIMD (96 VGPRs, no spills): the
// step is bound by the latency of its particle stream, which more resident
// waves hide.
template <int R, int D, bool PUSH, bool REFL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R == PIC_REPR_FP32_CELL ? 5 : 1))) void step_kernel(StepParams P) {
  step_block<R, D, PUSH, REFL>(P, blockIdx.x);
}

// Batched step (persistent): workgroups take work items (slot, block) from a
// counter until the step's items are exhausted. Slots are ordered by quota, so
// the items of the slots still stepping are a prefix of the table.
// The slot table is not written while a step runs: read it through the
// constant address space, so that the compiler may keep the descriptor of the
// (wave-uniform) work item in scalar registers as it does for a kernel
// argument.
typedef const __attribute__((address_space(4))) StepParams ConstStep;
typedef const __attribute__((address_space(4))) int32_t ConstI32;

template <int R, int D, bool REFL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R == PIC_REPR_FP32_CELL ? 5 : 1))) void batch_step_kernel(BatchTable B) {
  __shared__ int32_t sItem;
  ConstStep *slots = (ConstStep *)B.slots;
  ConstI32 *prefix = (ConstI32 *)B.prefix;
  const int total = ((ConstI32 *)B.totals)[*(ConstI32 *)B.istep];
  for (;;) {
    if (threadIdx.x == 0) sItem = atomicAdd(B.work, 1);
    __syncthreads();
    const int b = __builtin_amdgcn_readfirstlane(sItem);
    __syncthreads();
    if (b >= total) return;  // uniform
    int lo = 0, hi = B.nslots - 1;  // last slot with prefix <= b
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= b) lo = mid;
      else hi = mid - 1;
    }
    const StepParams &P = *(const StepParams *)(slots + lo);
    if (P.remaining > 0) step_block<R, D, true, REFL>(P, b - prefix[lo]);
  }
}

// Clears rho and the output overflow counts of every slot that will step
// (blockIdx.y = slot) and resets the work counter of the step.
__global__ void batch_clear_kernel(BatchTable B, int64_t elem_bytes) {
  const int k = blockIdx.y;
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) *B.work = 0;
  if (k >= B.nslots) return;
  const StepParams &P = B.slots[k];
  if (P.remaining <= 0) return;
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)P.ns) P.bins.ovf[1 - P.cur][threadIdx.x] = 0;
  const int64_t n = (int64_t)(P.nx + 1) * (P.ny + 1) * (P.nz + 1) * elem_bytes / 4;
  uint32_t *r = (uint32_t *)P.rho;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = 0u;
}

// After a batched run: for every slot of the table, the species whose
// overflow list in the current buffer is not empty (bit s), for one read-back
// by the host.
__global__ void batch_flags_kernel(BatchTable B, int32_t *out) {
  for (int k = threadIdx.x; k < B.nslots; k += blockDim.x) {
    const StepParams &P = B.slots[k];
    int32_t m = 0;
    for (int s = 0; s < P.ns; ++s)
      if (P.bins.ovf[P.cur][s] > 0) m |= 1 << s;
    out[k] = m;
  }
}

// After a batched step: every slot that stepped moves to its other buffer.
__global__ void batch_advance_kernel(BatchTable B) {
  for (int k = threadIdx.x; k < B.nslots; k += blockDim.x) {
    StepParams &P = B.slots[k];
    if (P.remaining > 0) {
      P.cur = 1 - P.cur;
      P.remaining -= 1;
    }
  }
  if (threadIdx.x == 0) *B.istep += 1;
}

// ------------------------------------------------------------------ re-bucketing

// Tile of a particle's current cell, or -1 if it is not a particle. home:
// the tile whose region slot p belongs to, or -1 (the overflow list, a
// freshly loaded buffer); a region holds its own tile's particles only.
template <int R>
__device__ __forceinline__ int tile_at(const PBuf &B, int64_t p, int ntx, int nty, int home,
                                       int tc[3]) {
  using T = typename RealOf<R>::T;
  int i, j, k;
  if constexpr (R == PIC_REPR_FP32_CELL) {
    if (home >= 0) {
      tc[0] = home % ntx;
      tc[1] = (home / ntx) % nty;
      tc[2] = home / (ntx * nty);
      return home;
    }
    const int32_t cell = B.cell[p];
    if (cell < 0) return -1;
    i = cell & kMaxDim;
    j = (cell >> kCellBits) & kMaxDim;
    k = cell >> (2 * kCellBits);
  } else {
    const T x = ((const T *)B.pos[0])[p];
    if (x < T(0)) return -1;
    i = (int)floorT(x);
    j = (int)floorT(((const T *)B.pos[1])[p]);
    k = (int)floorT(((const T *)B.pos[2])[p]);
  }
  tc[0] = i >> kTileShift;
  tc[1] = j >> kTileShift;
  tc[2] = k >> kTileShift;
  return tc[0] + ntx * (tc[1] + nty * tc[2]);
}

__device__ __forceinline__ int neighbour_rel(const int tc[3], int tx, int ty, int tz) {
  const int dx = tc[0] - tx, dy = tc[1] - ty, dz = tc[2] - tz;
  if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return -1;
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

__device__ __forceinline__ int neighbour_tile(int rel, int tx, int ty, int tz, int ntx, int nty) {
  const int dx = rel % 3 - 1, dy = (rel / 3) % 3 - 1, dz = rel / 9 - 1;
  return (tx + dx) + ntx * ((ty + dy) + nty * (tz + dz));
}

// The source entries of workgroup wg for species s: a chunk of an unsorted
// range, or a tile's region (wg < ntiles; home tile wg) / a chunk of the
// overflow list (wg >= ntiles: chunk wg - ntiles, so that a long list is
// spread over many workgroups). o.any is false if the workgroup has no
// source.
struct SortSrc {
  Src r;
  int home;  // home tile, or -1
  bool any;
};

__device__ __forceinline__ SortSrc sort_src(const SortParams &P, int s, int wg, int64_t chunk) {
  SortSrc o;
  o.home = -1;
  o.any = false;
  if ((P.unsorted >> s) & 1) {
    const int64_t a = (int64_t)wg * chunk;
    if (a >= P.n_src[s]) return o;
    const int64_t b = a + chunk < P.n_src[s] ? a + chunk : P.n_src[s];
    o.r.base = a;
    o.r.n1 = (int32_t)(b - a);
    o.r.na = 0;
    o.r.gap = 0;
  } else if (wg < P.ntiles) {
    o.r = src_of(P.bins, P.cur, s, wg, P.ntiles);
    o.home = wg;
  } else {
    const Src all = src_of(P.bins, P.cur, s, P.ntiles, P.ntiles);
    const int64_t a = (int64_t)(wg - P.ntiles) * chunk;
    if (a >= all.n1) return o;
    o.r.base = all.base + a;
    o.r.n1 = (int32_t)(all.n1 - a < chunk ? all.n1 - a : chunk);
    o.r.na = 0;
    o.r.gap = 0;
  }
  o.any = true;
  return o;
}

template <int R>
__global__ __launch_bounds__(kBlock) void sort_count_kernel(SortParams P, int64_t chunk) {
  __shared__ int32_t sH[kNeighbours];
  const int s = blockIdx.y;
  if (!((P.sel >> s) & 1)) return;  // uniform
  const int nt = P.ntiles;
  const SortSrc so = sort_src(P, s, blockIdx.x, chunk);
  if (!so.any) return;  // uniform
  const int t = so.home;
  int tx = 0, ty = 0, tz = 0;
  if (t >= 0) {
    tx = t % P.ntx;
    ty = (t / P.ntx) % P.nty;
    tz = t / (P.ntx * P.nty);
  }
  if (threadIdx.x < kNeighbours) sH[threadIdx.x] = 0;
  __syncthreads();
  const PBuf B = P.src[s];
  const int32_t np = so.r.n1 + so.r.na;
  for (int32_t k = threadIdx.x; k < np; k += kBlock) {
    int tc[3];
    const int ct = tile_at<R>(B, so.r.base + src_off(so.r, k), P.ntx, P.nty, t, tc);
    if (ct < 0) continue;
    const int rel = t >= 0 ? neighbour_rel(tc, tx, ty, tz) : -1;
    if (rel >= 0) agg_add(sH, rel);
    else atomicAdd(&P.count[s * nt + ct], 1);
  }
  __syncthreads();
  if (t >= 0 && threadIdx.x < kNeighbours) {
    const int h = sH[threadIdx.x];
    P.hist[((int64_t)s * nt + t) * kNeighbours + threadIdx.x] = h;
    if (h) atomicAdd(&P.count[s * nt + neighbour_tile(threadIdx.x, tx, ty, tz, P.ntx, P.nty)], h);
  }
}

// Plans the new layout from the tile counts (stay zone + arrival zone per
// tile, exclusive scan of the capacities); clears the counters for the
// scatter pass. One workgroup per species.
__global__ __launch_bounds__(1024) void sort_scan_kernel(SortParams P) {
  __shared__ long long sS[1024];
  const int s = blockIdx.x;
  if (!((P.sel >> s) & 1)) return;  // uniform
  const int nt = P.ntiles;
  const int out = 1 - P.cur;
  const int per = (nt + 1023) / 1024;
  const int b = threadIdx.x * per;
  const int e = b + per < nt ? b + per : nt;
  const bool flat = (P.unsorted >> s) & 1;
  long long local = 0, extra = 0;
  for (int i = b; i < e; ++i) {
    const int64_t j = (int64_t)s * nt + i;
    const int32_t c = P.count[j];
    local += stay_zone(c) + arrival_zone(c);
    if (P.inflow) extra += inflow_room(P.inflow[j]);
    if (!flat) extra += demand_room(c, P.bins.arr[P.cur][j]);
  }
  // the allowances for growth only if the regions with them fit the buffer
  sS[threadIdx.x] = local + extra;
  __syncthreads();
  for (int o = 512; o >= 1; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sS[threadIdx.x] += sS[threadIdx.x + o];
    __syncthreads();
  }
  const bool use = sS[0] <= P.region_cap[s];
  __syncthreads();
  if (use) local += extra;
  sS[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long v = threadIdx.x >= (unsigned)o ? sS[threadIdx.x - o] : 0;
    __syncthreads();
    sS[threadIdx.x] += v;
    __syncthreads();
  }
  long long run = sS[threadIdx.x] - local;
  for (int i = b; i < e; ++i) {
    const int64_t j = (int64_t)s * nt + i;
    // a freshly loaded species has no valid counters in the source buffer
    // either (the scatter clears them for binned species after reading)
    const int32_t a = flat ? 0 : P.bins.arr[P.cur][j];  // arrivals wanted in the last step
    if (flat) P.bins.arr[P.cur][j] = 0;
    const int32_t c = P.count[j];
    const int32_t in = use && P.inflow ? P.inflow[j] : 0;
    const int32_t ga = use ? a : 0;
    const int32_t sz = stay_zone(c) + kInflowSteps * in + kDemandSteps * ga;
    const int32_t az = arrival_zone(c) > 2 * ga ? arrival_zone(c) : 2 * ga;
    const int32_t cap = sz + az + 2 * in;
    P.dst_lay.base[j] = run;
    P.dst_lay.cap[j] = cap;
    P.dst_lay.sz[j] = sz;
    P.bins.nst[out][j] = c;
    P.bins.arr[out][j] = 0;
    run += cap;
    P.count[j] = 0;
    P.cursor[j] = 0;
  }
  if (threadIdx.x == 1023) {
    if (sS[1023] > P.region_cap[s]) atomicOr(P.err, kErrCapacity);
    P.bins.ovf[out][s] = 0;
    if (flat) P.bins.ovf[P.cur][s] = 0;
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void sort_scatter_kernel(SortParams P, int64_t chunk) {
  __shared__ long long sBase[kNeighbours];
  __shared__ int32_t sCur[kNeighbours];
  const int s = blockIdx.y;
  if (!((P.sel >> s) & 1)) return;  // uniform
  const int nt = P.ntiles;
  const SortSrc so = sort_src(P, s, blockIdx.x, chunk);
  if (!so.any) return;  // uniform
  const int t = so.home;
  int tx = 0, ty = 0, tz = 0;
  if (t >= 0) {
    tx = t % P.ntx;
    ty = (t / P.ntx) % P.nty;
    tz = t / (P.ntx * P.nty);
    if (threadIdx.x < kNeighbours) {
      const int h = P.hist[((int64_t)s * nt + t) * kNeighbours + threadIdx.x];
      long long base = 0;
      if (h) {
        const int nb = neighbour_tile(threadIdx.x, tx, ty, tz, P.ntx, P.nty);
        base = P.dst_lay.base[(int64_t)s * nt + nb] + atomicAdd(&P.cursor[s * nt + nb], h);
      }
      sBase[threadIdx.x] = base;
      sCur[threadIdx.x] = 0;
    }
  }
  __syncthreads();
  const PBuf S = P.src[s], Dd = P.dst[s];
  const bool ids = (P.has_ids >> s) & 1;
  const int32_t np = so.r.n1 + so.r.na;
  for (int32_t k = threadIdx.x; k < np; k += kBlock) {
    const int64_t p = so.r.base + src_off(so.r, k);
    int tc[3];
    const int ct = tile_at<R>(S, p, P.ntx, P.nty, t, tc);
    if (ct < 0) continue;
    const int rel = t >= 0 ? neighbour_rel(tc, tx, ty, tz) : -1;
    long long q;
    if (rel >= 0) {
      q = sBase[rel] + agg_add(sCur, rel);
    } else {
      q = P.dst_lay.base[(int64_t)s * nt + ct] + atomicAdd(&P.cursor[s * nt + ct], 1);
    }
    using T = typename RealOf<R>::T;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ((T *)Dd.pos[d])[q] = ((const T *)S.pos[d])[p];
      ((T *)Dd.vel[d])[q] = ((const T *)S.vel[d])[p];
    }
    // (the destination is a region: the stored offsets carry the cell)
    if (ids) Dd.ids[q] = S.ids[p];
  }
  // the source counters are consumed (the source buffer is the next output;
  // the overflow count, which every overflow chunk reads, in the commit pass)
  if (t >= 0 && !((P.unsorted >> s) & 1)) {
    __syncthreads();
    if (threadIdx.x == 0) P.bins.arr[P.cur][(int64_t)s * nt + t] = 0;
  }
}

// After the scatter: the new layout and stay counts of every re-bucketed
// species become those of the source buffer index, whose particle storage the
// host swaps with the destination's, and its overflow list is empty. One
// thread per tile.
__global__ void sort_commit_kernel(SortParams P) {
  const int s = blockIdx.y;
  if (!((P.sel >> s) & 1)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.ntiles) return;
  if (i == 0) P.bins.ovf[P.cur][s] = 0;
  const int64_t j = (int64_t)s * P.ntiles + i;
  P.bins.lay.base[j] = P.dst_lay.base[j];
  P.bins.lay.cap[j] = P.dst_lay.cap[j];
  P.bins.lay.sz[j] = P.dst_lay.sz[j];
  P.bins.nst[P.cur][j] = P.bins.nst[1 - P.cur][j];
}

// Sampled read-back: for every particle whose id is in the sorted list, write
// its state (cell units, FP64) to the list slot. One workgroup per tile region
// (and one for the overflow list).
template <int R>
__global__ void find_ids_kernel(PBuf B, Bins bins, int32_t cur, int32_t s, int32_t nt, int32_t ntx,
                                int32_t nty,
                                const int64_t *ids, int64_t n_ids, int32_t *found, double *out,
                                PhysUnits phys) {
  using T = typename RealOf<R>::T;
  const Src r = src_of(bins, cur, s, blockIdx.x, nt);
  const int32_t np = r.n1 + r.na;
  for (int32_t k = threadIdx.x; k < np; k += blockDim.x) {
    const int64_t p = r.base + src_off(r, k);
    double g[3];
    if constexpr (R == PIC_REPR_FP32_CELL) {
      int ci[3];
      const float *X[3] = {(const float *)B.pos[0], (const float *)B.pos[1], (const float *)B.pos[2]};
      if ((int)blockIdx.x < nt) {  // a tile's region: the tile and the offsets' sub-cells
        const int t = blockIdx.x;
        ci[0] = ((t % ntx) << kTileShift) + off_sub(X[0][p]);
        ci[1] = (((t / ntx) % nty) << kTileShift) + off_sub(X[1][p]);
        ci[2] = ((t / (ntx * nty)) << kTileShift) + off_sub(X[2][p]);
      } else {
        const int32_t cell = B.cell[p];
        if (cell < 0) continue;
        ci[0] = cell & kMaxDim;
        ci[1] = (cell >> kCellBits) & kMaxDim;
        ci[2] = cell >> (2 * kCellBits);
      }
      for (int d = 0; d < 3; ++d) g[d] = (double)ci[d] + (double)off_value(X[d][p]);
    } else {
      const T x = ((const T *)B.pos[0])[p];
      if (x < T(0)) continue;
      for (int d = 0; d < 3; ++d) g[d] = (double)((const T *)B.pos[d])[p];
    }
    const int64_t id = B.ids[p];
    int64_t lo = 0, hi = n_ids;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ids[mid] < id) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= n_ids || ids[lo] != id) continue;
    found[lo] = 1;
    for (int d = 0; d < 3; ++d) {
      const double u = (double)((const T *)B.vel[d])[p];
      out[d * n_ids + lo] = phys.on ? phys.origin[d] + g[d] * phys.h : g[d];
      out[(3 + d) * n_ids + lo] = phys.on ? u * phys.h : u;
    }
  }
}

// ------------------------------------------------------------------ utility

// The common end of injection and photoemission for one lane's particle
// (has: the lane holds one; g, v in cell units, FP64): rounded to the
// representation, the box and object tests of a pushed particle (collected at
// once, or dropped if outside the box), appended to its tile's arrival zone
// in the output buffer, deposited, counted. Every lane of the wave calls it.
__device__ __forceinline__ int sp_slot() { return (int)(blockIdx.x & (kCountSlots - 1)); }

template <int R, int D>
__device__ __forceinline__ void emit_particle(const InjParams &P, bool has, int s, const double g[3],
                                              const double v[3]) {
  using T = typename RealOf<R>::T;
  using A = typename AccOf<D>::type;
  constexpr bool kCell = R == PIC_REPR_FP32_CELL;
  constexpr bool kFixed = D == PIC_DEP_FIXED64;
  const bool crater = P.geom.kind == PIC_OBJ_CRATER;
  const bool ids = (P.has_ids >> s) & 1;
  const int sx = P.nx + 1, sy = (P.nx + 1) * (P.ny + 1);
  const int lane = __lane_id();
  bool inside = false, keep = false;
  Particle<T> pt;
  int ci[3] = {0, 0, 0};
  T fo[3] = {T(0), T(0), T(0)};
  if (has) {
    // the representation of the injected particle, then the tests of a pushed one
    if constexpr (kCell) {
      for (int q = 0; q < 3; ++q) {
        ci[q] = (int)floor(g[q]);
        fo[q] = (T)(g[q] - (double)ci[q]);
        if (fo[q] == T(1)) {
          fo[q] = T(0);
          ci[q] += 1;
        }
      }
      inside = box_face(ci, P.nx, P.ny, P.nz, crater) < 0;
      pt.cell = pack_cell(ci[0], ci[1], ci[2]);
      for (int q = 0; q < 3; ++q) pt.x[q] = off_pack(fo[q], ci[q]);
    } else {
      for (int q = 0; q < 3; ++q) pt.x[q] = (T)g[q];
      inside = box_face_abs(pt.x, P.nx, P.ny, P.nz, crater) < 0;
      if (inside) {
        for (int q = 0; q < 3; ++q) {
          ci[q] = (int)floorT(pt.x[q]);
          fo[q] = pt.x[q] - (T)ci[q];
        }
      }
      pt.cell = 0;
    }
    for (int q = 0; q < 3; ++q) pt.u[q] = (T)v[q];
    pt.id = -1;
    if (inside) {
      const GeomT<T> G = geom_of<T>(P.geom);
      int bin;
      if constexpr (kCell) bin = hit_cell(G, P.nx, P.ny, ci, fo);
      else bin = hit_abs(G, P.nx, P.ny, pt.x);
      if (bin >= 0) atomicAdd((unsigned long long *)&P.tally[(int64_t)bin * P.ns + s], 1ull);
      keep = bin < 0;
    }
  }

  // append to the arrival zone of the particle's tile (one reservation per
  // tile and species in the wave)
  if (keep) {
    const int key = s * P.ntiles + tile_of_cell(ci, P.ntx, P.nty);
    const int32_t kk = agg_add(P.bins.arr[P.out_idx], key);
    const int32_t cap = P.bins.lay.cap[key], room = cap - P.bins.lay.sz[key];
    int64_t slot = -1;
    if (kk < room) {
      slot = P.bins.lay.base[key] + cap - 1 - kk;
    } else {
      const int32_t o = atomicAdd(&P.bins.ovf[P.out_idx][s], 1);
      if (o < P.bins.ovf_cap[s]) slot = P.bins.ovf_base[s] + o;
      else atomicOr(P.err, kErrCapacity);
    }
    if (slot >= 0) store_particle<R>(P.out[s], slot, pt, ids, P.bins.ovf_base[s]);
  }

  // deposit: the contributions of the lanes that landed in the same cell are
  // summed across the wave first (integer sums: exact), one atomic per corner
  A C[8];
  {
    T W[8];
    weights(fo, W);
    const T chg = (T)P.chg[s];
    if constexpr (kFixed) {
      const bool neg = chg < T(0);
      const T amag = absT(chg) * two32<T>();
      const unsigned long long fmag =
          (unsigned long long)(P.chg_fixed[s] < 0 ? -P.chg_fixed[s] : P.chg_fixed[s]);
      unsigned long long sum = 0;
      for (int q = 0; q < 7; ++q) {
        const unsigned long long m = fix_mag<T>(amag * W[q]);
        sum += m;
        C[q] = neg ? 0ull - m : m;
      }
      C[7] = neg ? 0ull - (fmag - sum) : fmag - sum;
    } else {
      for (int q = 0; q < 8; ++q) C[q] = (A)(chg * W[q]);
    }
  }
  const int b0 = keep ? ci[0] + sx * ci[1] + sy * ci[2] : -1;
  A *__restrict__ gRho = (A *)P.rho;
  const int off[8] = {0, 1, sx, sx + 1, sy, sy + 1, sy + sx, sy + sx + 1};
  unsigned long long pending = __ballot(keep);
  while (pending) {  // wave-uniform
    const int leader = __ffsll(pending) - 1;
    const int bl = __shfl(b0, leader);
    const unsigned long long m = __ballot(keep && b0 == bl) & pending;
    const bool mine = (m >> lane) & 1ull;
    for (int q = 0; q < 8; ++q) {
      A vsum = mine ? C[q] : A(0);
      for (int o = 32; o >= 1; o >>= 1) vsum += __shfl_xor(vsum, o);
      if (lane == leader) {
        if constexpr (kFixed) atomicAdd(&gRho[bl + off[q]], vsum);
        else unsafeAtomicAdd(&gRho[bl + off[q]], vsum);
      }
    }
    pending &= ~m;
  }

  // the injected counts: one atomic per wave and species, on the workgroup's
  // count slot
  const int slot = sp_slot();
  for (int sp = 0; sp < P.ns; ++sp) {
    unsigned long long c = (inside && s == sp) ? 1ull : 0ull;
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
    if (c && lane == 0)
      atomicAdd((unsigned long long *)&P.injected[sp * kCountSlots + slot], c);
  }
}


// Injection: one thread per (species, face, face cell, ghost slot); a face
// cell has floor(mean) + 1 slots, of which the first floor(mean + U) hold a
// ghost. A ghost is drawn, moved dt and, if it ends inside the box, rounded to
// the representation, tested against the object (collected at once) or
// appended to its tile's arrival zone in the output buffer and deposited.
template <int R, int D>
__global__ __launch_bounds__(256) void inject_kernel(InjParams P) {
  using T = typename RealOf<R>::T;
  constexpr bool kCell = R == PIC_REPR_FP32_CELL;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nsf = P.ns * 6;
  const bool active = tid < P.first[nsf];
  int sf = 0;
  while (active && P.first[sf + 1] <= tid) ++sf;
  const int s = sf / 6, f = sf % 6;
  const int64_t slot_id = tid - P.first[sf];
  const int64_t gmax = P.gmax[s][f];
  const int64_t cell = active ? slot_id / gmax : 0;
  const int64_t j = active ? slot_id - cell * gmax + 1 : 0;  // ghost 1..gmax of the face cell
  const int n[3] = {P.nx, P.ny, P.nz};
  const int axis = f / 2;
  const bool max_side = (f & 1) != 0;
  const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
  const int64_t a = cell % n[t1], b = cell / n[t1];
  const uint64_t ckey = inj_cell_key(P.seed, P.step, s, f, cell);
  const int64_t k = active ? (int64_t)floor(P.mean[s][f] + inj_uniform(sm_mix(ckey ^ 0ull), 0)) : 0;
  const bool crater = P.geom.kind == PIC_OBJ_CRATER;

  // the ghost of this slot, if the face cell has one there
  bool enters = false;
  double g[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
  uint64_t key = 0, d = 3;
  int attempts = 0;
  double z1 = 0.0;
  if (active && j <= k) {
    // the normal component first: most ghosts do not reach the face, and
    // the test of the normal axis alone (in the representation, as the box
    // test makes it) rejects them before the tangential draws
    key = sm_mix(ckey ^ (uint64_t)j);
    const double depth = P.L[s][f] * (1.0 - inj_uniform(key, 2));
    double z0;
    normal_pair(key, &d, &attempts, &z0, &z1);
    v[axis] = P.u[s][axis] + P.vth[s] * z0;
    g[axis] = fma(v[axis], P.dt, max_side ? (double)n[axis] + depth : -depth);
    if constexpr (kCell) {
      int i = (int)floor(g[axis]);
      const T o = (T)(g[axis] - (double)i);
      if (o == T(1)) i += 1;
      enters = i < n[axis] && (i >= 0 || (crater && axis == 2));
    } else {
      const T x = (T)g[axis];
      enters = x < (T)n[axis] && (x >= T(0) || (crater && axis == 2));
    }
  }
  if (enters) {
    double z2, z3;
    normal_pair(key, &d, &attempts, &z2, &z3);
    (void)z3;
    v[t1] = P.u[s][t1] + P.vth[s] * z1;
    v[t2] = P.u[s][t2] + P.vth[s] * z2;
    g[t1] = fma(v[t1], P.dt, (double)a + inj_uniform(key, 0));
    g[t2] = fma(v[t2], P.dt, (double)b + inj_uniform(key, 1));
  }
  emit_particle<R, D>(P, enters, s, g, v);
}

// Photoemission from the sunlit terrain: one thread per (surface column,
// slot); a lit column has floor(mean) + 1 slots (the largest over the columns),
// of which the first floor(mean + U) hold a photoelectron. The terrain at the
// column centre gives the normal n, the sunlight index I = s.n and the
// shadow (a bowl column is lit if the ray to the Sun leaves the bowl sphere,
// a chord of 2 Rc I, at or above the flat ground); mean = rate I / n_z. A
// photoelectron starts at a uniform point of the column's footprint on the
// ground with vth (|z0| n + z1 t1 + z2 t2), t1 = (n_z, 0, -n_x) normalised,
// t2 = n x t1, and moves a uniform fraction of dt; then it is handled like an
// injected particle.
template <int R, int D>
__global__ __launch_bounds__(256) void photo_kernel(InjParams P) {
  const PhotoParams &E = P.pe;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncol = (int64_t)P.nx * P.ny;
  const bool active = tid < ncol * E.gmax;
  const int64_t col = active ? tid / E.gmax : 0;
  const int64_t j = active ? tid - col * E.gmax + 1 : 0;  // photoelectron 1..gmax of the column
  const int64_t ci = col % P.nx, cj = col / P.nx;
  const int s = E.s;
  // the terrain at the column centre
  const double dx = ((double)ci + 0.5) - E.cx, dy = ((double)cj + 0.5) - E.cy;
  const double r2 = dx * dx + dy * dy;
  const bool bowl = r2 < E.a2;
  double n[3], zg;
  if (bowl) {
    zg = E.zc - __builtin_sqrt(E.rc2 - r2);
    n[0] = -dx / E.rc;
    n[1] = -dy / E.rc;
    n[2] = (E.zc - zg) / E.rc;
  } else {
    zg = E.z_flat;
    n[0] = 0.0;
    n[1] = 0.0;
    n[2] = 1.0;
  }
  const double I = (E.sun[0] * n[0] + E.sun[1] * n[1]) + E.sun[2] * n[2];
  const bool lit = I > 0.0 && (!bowl || zg + (2.0 * E.rc * I) * E.sun[2] >= E.z_flat);
  const uint64_t ckey = inj_cell_key(E.seed, P.step, s, 6, col);
  int64_t k = 0;
  if (active && lit) k = (int64_t)floor((E.rate * I) / n[2] + inj_uniform(sm_mix(ckey ^ 0ull), 0));
  const bool has = active && j <= k;
  double g[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
  if (has) {
    const uint64_t key = sm_mix(ckey ^ (uint64_t)j);
    const double x = (double)ci + inj_uniform(key, 0), y = (double)cj + inj_uniform(key, 1);
    const double ex = x - E.cx, ey = y - E.cy;
    const double q2 = ex * ex + ey * ey;
    const double z0g = q2 < E.a2 ? E.zc - __builtin_sqrt(E.rc2 - q2) : E.z_flat;
    const double tau = P.dt * inj_uniform(key, 2);
    uint64_t d = 3;
    int attempts = 0;
    double z0, z1, z2, z3;
    normal_pair(key, &d, &attempts, &z0, &z1);
    normal_pair(key, &d, &attempts, &z2, &z3);
    (void)z3;
    const double l1 = __builtin_sqrt(n[2] * n[2] + n[0] * n[0]);
    const double t1[3] = {n[2] / l1, 0.0, -n[0] / l1};
    const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2],
                          n[0] * t1[1] - n[1] * t1[0]};
    const double a0 = __builtin_fabs(z0);
    for (int c = 0; c < 3; ++c) v[c] = E.vth * ((a0 * n[c] + z1 * t1[c]) + z2 * t2[c]);
    g[0] = fma(v[0], tau, x);
    g[1] = fma(v[1], tau, y);
    g[2] = fma(v[2], tau, z0g);
  }
  emit_particle<R, D>(P, has, s, g, v);
}

__global__ void fill_kernel(uint32_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <int R>
__global__ void load_f32_kernel(LoadParams L) {
  using T = typename RealOf<R>::T;
  const int32_t n3[3] = {L.nx, L.ny, L.nz};
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L.n;
       p += (int64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    int ci[3];
    float o[3];
    double g[3];
    for (int d = 0; d < 3; ++d) {
      g[d] = ((double)L.x[d][p] - L.origin[d]) / L.h;
      bad |= !(g[d] >= 0.0 && g[d] < (double)n3[d]);
      // an FP32 coordinate just below the upper face may round up onto it
      if constexpr (R == PIC_REPR_FP32_ABS) bad |= !((float)g[d] < (float)n3[d]);
      if constexpr (R == PIC_REPR_FP32_CELL) {
        int i = bad ? 0 : (int)__builtin_floor(g[d]);
        float oo = (float)(g[d] - (double)i);
        if (oo == 1.0f) {
          oo = 0.0f;
          i += 1;
        }
        ci[d] = i;
        o[d] = oo;
      }
    }
    if (bad) {
      atomicAdd(L.bad, 1);
      continue;
    }
    if constexpr (R == PIC_REPR_FP32_CELL) {
      // an offset rounded up into the next cell may leave the box
      if (ci[0] >= L.nx || ci[1] >= L.ny || ci[2] >= L.nz) {
        atomicAdd(L.bad, 1);
        continue;
      }
      L.out.cell[p] = pack_cell(ci[0], ci[1], ci[2]);
      for (int d = 0; d < 3; ++d) ((float *)L.out.pos[d])[p] = off_pack(o[d], ci[d]);
    } else {
      for (int d = 0; d < 3; ++d) ((T *)L.out.pos[d])[p] = (T)g[d];
    }
    for (int d = 0; d < 3; ++d) ((T *)L.out.vel[d])[p] = (T)((double)L.v[d][p] / L.h);
    if (L.ids) L.out.ids[p] = L.ids[p];
  }
}

template <class V4>
__global__ void node_E_kernel(const float *Ex, const float *Ey, const float *Ez, V4 *E,
                              int64_t nodes, int32_t *bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nodes;
       i += (int64_t)gridDim.x * blockDim.x) {
    V4 e;
    e.x = Ex[i];
    e.y = Ey[i];
    e.z = Ez[i];
    e.w = 0;
    if (!(__builtin_isfinite(Ex[i]) && __builtin_isfinite(Ey[i]) && __builtin_isfinite(Ez[i])))
      atomicAdd(bad, 1);
    E[i] = e;
  }
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <int R, int D>
hipError_t launch_step_rd(bool push, const StepParams &p, hipStream_t s) {
  if (p.ntiles <= 0) return hipSuccess;
  // one workgroup per tile plus ovf_groups for the overflow list
  const dim3 grid(p.ntiles + p.ovf_groups);
  if (push && p.reflect)
    hipLaunchKernelGGL((step_kernel<R, D, true, true>), grid, dim3(kBlock), 0, s, p);
  else if (push)
    hipLaunchKernelGGL((step_kernel<R, D, true, false>), grid, dim3(kBlock), 0, s, p);
  else
    hipLaunchKernelGGL((step_kernel<R, D, false, false>), grid, dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

template <int R>
hipError_t launch_step_r(int deposit, bool push, const StepParams &p, hipStream_t s) {
  switch (deposit) {
    case PIC_DEP_FIXED64: return launch_step_rd<R, PIC_DEP_FIXED64>(push, p, s);
    case PIC_DEP_ATOMIC_FP32: return launch_step_rd<R, PIC_DEP_ATOMIC_FP32>(push, p, s);
    case PIC_DEP_ATOMIC_FP64: return launch_step_rd<R, PIC_DEP_ATOMIC_FP64>(push, p, s);
  }
  return hipErrorInvalidValue;
}

constexpr int64_t kChunk = 4096;

// Workgroups per species: tiles + chunks of the overflow list (as many as its
// capacity takes) for binned species, chunks for unsorted ones (max_src: the
// largest unsorted range).
int64_t sort_blocks(const SortParams &p, int64_t max_src) {
  int64_t n = (max_src + kChunk - 1) / kChunk;
  for (int s = 0; s < p.ns; ++s) {
    if (!(((p.sel & ~p.unsorted) >> s) & 1)) continue;
    const int64_t b = (int64_t)p.ntiles + (p.bins.ovf_cap[s] + kChunk - 1) / kChunk;
    if (b > n) n = b;
  }
  return n;
}

}  // namespace

hipError_t launch_step(int repr, int deposit, bool push, const StepParams &p, hipStream_t s) {
  switch (repr) {
    case PIC_REPR_FP64: return launch_step_r<PIC_REPR_FP64>(deposit, push, p, s);
    case PIC_REPR_FP32_ABS: return launch_step_r<PIC_REPR_FP32_ABS>(deposit, push, p, s);
    case PIC_REPR_FP32_CELL: return launch_step_r<PIC_REPR_FP32_CELL>(deposit, push, p, s);
  }
  return hipErrorInvalidValue;
}

template <int R, int D>
hipError_t launch_batch_rd(bool refl, const BatchTable &t, int32_t grid, hipStream_t s) {
  const int64_t eb = D == PIC_DEP_ATOMIC_FP32 ? 4 : 8;
  hipLaunchKernelGGL(batch_clear_kernel, dim3(64, t.nslots), dim3(256), 0, s, t, eb);
  if (refl)
    hipLaunchKernelGGL((batch_step_kernel<R, D, true>), dim3(grid), dim3(kBlock), 0, s, t);
  else
    hipLaunchKernelGGL((batch_step_kernel<R, D, false>), dim3(grid), dim3(kBlock), 0, s, t);
  hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(256), 0, s, t);
  return hipGetLastError();
}

template <int R>
hipError_t launch_batch_r(int deposit, bool refl, const BatchTable &t, int32_t grid,
                          hipStream_t s) {
  switch (deposit) {
    case PIC_DEP_FIXED64: return launch_batch_rd<R, PIC_DEP_FIXED64>(refl, t, grid, s);
    case PIC_DEP_ATOMIC_FP32: return launch_batch_rd<R, PIC_DEP_ATOMIC_FP32>(refl, t, grid, s);
    case PIC_DEP_ATOMIC_FP64: return launch_batch_rd<R, PIC_DEP_ATOMIC_FP64>(refl, t, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_flags(const BatchTable &t, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(batch_flags_kernel, dim3(1), dim3(256), 0, s, t, out);
  return hipGetLastError();
}

hipError_t launch_batch_step(int repr, int deposit, bool refl, const BatchTable &t, int32_t grid,
                             hipStream_t s) {
  if (t.nslots <= 0 || grid <= 0) return hipSuccess;
  switch (repr) {
    case PIC_REPR_FP64: return launch_batch_r<PIC_REPR_FP64>(deposit, refl, t, grid, s);
    case PIC_REPR_FP32_ABS: return launch_batch_r<PIC_REPR_FP32_ABS>(deposit, refl, t, grid, s);
    case PIC_REPR_FP32_CELL: return launch_batch_r<PIC_REPR_FP32_CELL>(deposit, refl, t, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sort_count(int repr, const SortParams &p, int64_t max_src, hipStream_t s) {
  const int64_t nb = sort_blocks(p, max_src);
  if (nb <= 0 || nb > 0x7fffffff) return nb <= 0 ? hipSuccess : hipErrorInvalidValue;
  const dim3 grid((unsigned)nb, p.ns);
  switch (repr) {
    case PIC_REPR_FP64:
      hipLaunchKernelGGL(sort_count_kernel<PIC_REPR_FP64>, grid, dim3(kBlock), 0, s, p, kChunk);
      break;
    case PIC_REPR_FP32_ABS:
      hipLaunchKernelGGL(sort_count_kernel<PIC_REPR_FP32_ABS>, grid, dim3(kBlock), 0, s, p, kChunk);
      break;
    default:
      hipLaunchKernelGGL(sort_count_kernel<PIC_REPR_FP32_CELL>, grid, dim3(kBlock), 0, s, p, kChunk);
  }
  return hipGetLastError();
}

hipError_t launch_sort_scan(const SortParams &p, hipStream_t s) {
  hipLaunchKernelGGL(sort_scan_kernel, dim3(p.ns), dim3(1024), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_sort_commit(const SortParams &p, hipStream_t s) {
  if (p.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(sort_commit_kernel, dim3((p.ntiles + 255) / 256, p.ns), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_sort_scatter(int repr, const SortParams &p, int64_t max_src, hipStream_t s) {
  const int64_t nb = sort_blocks(p, max_src);
  if (nb <= 0 || nb > 0x7fffffff) return nb <= 0 ? hipSuccess : hipErrorInvalidValue;
  const dim3 grid((unsigned)nb, p.ns);
  switch (repr) {
    case PIC_REPR_FP64:
      hipLaunchKernelGGL(sort_scatter_kernel<PIC_REPR_FP64>, grid, dim3(kBlock), 0, s, p, kChunk);
      break;
    case PIC_REPR_FP32_ABS:
      hipLaunchKernelGGL(sort_scatter_kernel<PIC_REPR_FP32_ABS>, grid, dim3(kBlock), 0, s, p, kChunk);
      break;
    default:
      hipLaunchKernelGGL(sort_scatter_kernel<PIC_REPR_FP32_CELL>, grid, dim3(kBlock), 0, s, p, kChunk);
  }
  return hipGetLastError();
}

// rho and the output overflow counts of a step cleared in one launch
__global__ void step_clear_kernel(uint32_t *r, int64_t n, int32_t *ovf, int32_t ns) {
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)ns) ovf[threadIdx.x] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = 0u;
}

hipError_t launch_step_clear(void *rho, int64_t bytes, int32_t *ovf_out, int32_t ns,
                             hipStream_t s) {
  const int64_t n = bytes / 4;
  hipLaunchKernelGGL(step_clear_kernel, dim3(grid_for(n > 0 ? n : 1, 256)), dim3(256), 0, s,
                     (uint32_t *)rho, n, ovf_out, ns);
  return hipGetLastError();
}

hipError_t launch_fill(void *ptr, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 4;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, (uint32_t *)ptr, n);
  return hipGetLastError();
}

template <int R>
hipError_t launch_inject_r(int deposit, const InjParams &p, dim3 grid, hipStream_t s) {
  switch (deposit) {
    case PIC_DEP_FIXED64:
      hipLaunchKernelGGL((inject_kernel<R, PIC_DEP_FIXED64>), grid, dim3(256), 0, s, p);
      break;
    case PIC_DEP_ATOMIC_FP32:
      hipLaunchKernelGGL((inject_kernel<R, PIC_DEP_ATOMIC_FP32>), grid, dim3(256), 0, s, p);
      break;
    case PIC_DEP_ATOMIC_FP64:
      hipLaunchKernelGGL((inject_kernel<R, PIC_DEP_ATOMIC_FP64>), grid, dim3(256), 0, s, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R>
hipError_t launch_photo_r(int deposit, const InjParams &p, dim3 grid, hipStream_t s) {
  switch (deposit) {
    case PIC_DEP_FIXED64:
      hipLaunchKernelGGL((photo_kernel<R, PIC_DEP_FIXED64>), grid, dim3(256), 0, s, p);
      break;
    case PIC_DEP_ATOMIC_FP32:
      hipLaunchKernelGGL((photo_kernel<R, PIC_DEP_ATOMIC_FP32>), grid, dim3(256), 0, s, p);
      break;
    case PIC_DEP_ATOMIC_FP64:
      hipLaunchKernelGGL((photo_kernel<R, PIC_DEP_ATOMIC_FP64>), grid, dim3(256), 0, s, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_photo(int repr, int deposit, const InjParams &p, hipStream_t s) {
  const int64_t total = (int64_t)p.nx * p.ny * p.pe.gmax;
  if (total <= 0) return hipSuccess;
  const dim3 grid(grid_for(total, 256));
  switch (repr) {
    case PIC_REPR_FP64: return launch_photo_r<PIC_REPR_FP64>(deposit, p, grid, s);
    case PIC_REPR_FP32_ABS: return launch_photo_r<PIC_REPR_FP32_ABS>(deposit, p, grid, s);
    case PIC_REPR_FP32_CELL: return launch_photo_r<PIC_REPR_FP32_CELL>(deposit, p, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_inject(int repr, int deposit, const InjParams &p, hipStream_t s) {
  const int64_t total = p.first[p.ns * 6];
  if (total <= 0) return hipSuccess;
  const dim3 grid(grid_for(total, 256));
  switch (repr) {
    case PIC_REPR_FP64: return launch_inject_r<PIC_REPR_FP64>(deposit, p, grid, s);
    case PIC_REPR_FP32_ABS: return launch_inject_r<PIC_REPR_FP32_ABS>(deposit, p, grid, s);
    case PIC_REPR_FP32_CELL: return launch_inject_r<PIC_REPR_FP32_CELL>(deposit, p, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_load_f32(int repr, const LoadParams &p, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  const dim3 grid(grid_for(p.n, 256));
  switch (repr) {
    case PIC_REPR_FP64:
      hipLaunchKernelGGL(load_f32_kernel<PIC_REPR_FP64>, grid, dim3(256), 0, s, p);
      break;
    case PIC_REPR_FP32_ABS:
      hipLaunchKernelGGL(load_f32_kernel<PIC_REPR_FP32_ABS>, grid, dim3(256), 0, s, p);
      break;
    default:
      hipLaunchKernelGGL(load_f32_kernel<PIC_REPR_FP32_CELL>, grid, dim3(256), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_find_ids(int repr, const PBuf &buf, const Bins &bins, int32_t cur, int32_t s,
                           int32_t ntiles, int32_t ntx, int32_t nty, const int64_t *ids_sorted,
                           int64_t n_ids, int32_t *found, double *out6, const PhysUnits &phys,
                           hipStream_t st) {
  if (n_ids <= 0) return hipSuccess;
  const dim3 grid(ntiles + 1);
  switch (repr) {
    case PIC_REPR_FP64:
      hipLaunchKernelGGL(find_ids_kernel<PIC_REPR_FP64>, grid, dim3(256), 0, st, buf, bins, cur, s,
                         ntiles, ntx, nty, ids_sorted, n_ids, found, out6, phys);
      break;
    case PIC_REPR_FP32_ABS:
      hipLaunchKernelGGL(find_ids_kernel<PIC_REPR_FP32_ABS>, grid, dim3(256), 0, st, buf, bins, cur,
                         s, ntiles, ntx, nty, ids_sorted, n_ids, found, out6, phys);
      break;
    default:
      hipLaunchKernelGGL(find_ids_kernel<PIC_REPR_FP32_CELL>, grid, dim3(256), 0, st, buf, bins, cur,
                         s, ntiles, ntx, nty, ids_sorted, n_ids, found, out6, phys);
  }
  return hipGetLastError();
}

// The scratch of pic_get_particles_by_id_noalloc (each GPU holds its own copy
// until the process ends). In host code `scratch` names a host-side stand-in,
// not a device address: every use goes through the address that
// hipGetSymbolAddress gives per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(void **ptr) {
  constexpr int kDevices = 64;
  static std::mutex mu;
  static void *addr[kDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_node_E_f32(int repr, const float *Ex, const float *Ey, const float *Ez,
                             void *E, int64_t nodes, int32_t *bad, hipStream_t s) {
  const dim3 grid(grid_for(nodes, 256));
  if (repr == PIC_REPR_FP64)
    hipLaunchKernelGGL(node_E_kernel<D4>, grid, dim3(256), 0, s, Ex, Ey, Ez, (D4 *)E, nodes, bad);
  else
    hipLaunchKernelGGL(node_E_kernel<F4>, grid, dim3(256), 0, s, Ex, Ey, Ez, (F4 *)E, nodes, bad);
  return hipGetLastError();
}

}  // namespace pic
