// PIC particle-mesh oracle: a plain, slow CPU implementation of one explicit
// PIC step (gather -> push -> boundary/object -> deposit). It runs on one
// thread unless orc_config.threads asks for more (below).
//
// THIS FILE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark load it. The GPU library never links,
// includes or calls it, and it shares no code with the GPU library.
//
// What it follows:
//   * The PIC loop of §2.1: charge is weighted from particles to mesh nodes
//     ("scatter"), the field is interpolated at particle positions ("gather"),
//     and velocity and position are updated ("particle-push"). The field solve
//     of the loop is not computed here: the node electric field is an input.
//   * §3.1.3: particles hitting outer boundaries are absorbed and removed
//     (the open-box reading: all six faces remove, counted per face).
//   * §5.2.2 and the "other" phase of Table 1 (§3.3): particles hitting the
//     object or the lunar surface are collected and their charge accumulated
//     for surface charging (a per-bin count per species; charge = q*w*count).
//   * §5.2.1: the terrain is a height function z = z(x, y); here a flat plane
//     with a spherical-bowl crater.
//   * §3.1.1 / §5.2.1: lengths are normalised so that the PIC cell has size h
//     (unit cells in every workload).
// The paper names neither the weighting order nor the integrator. This oracle
// takes first-order (trilinear, cloud-in-cell) weighting with node-centred E
// and rho, and the leapfrog push with velocities stored at half steps.
//
// The step, per particle, in index order (internal coordinates are cell units
// g = (x - origin)/h, velocities u = v/h):
//   1. locate: i = floor(g), f = g - i           (cell-relative form: stored)
//   2. weights: w0 = 1 - f, w1 = f per axis; W[a+2b+4c] = (wx[a]*wy[b])*wz[c]
//   3. gather: acc = W[0]*E[node 0]; acc = fma(W[n], E[node n], acc), n = 1..7
//   4. kick:   u = fma(qmdt, E_p, u), qmdt = q/m*dt/h
//   5. drift:  g = fma(u, dt, g)   (cell form: o' = fma(u,dt,o), s = floor(o'),
//              o' -= s, if o' == 1 then o' = 0, s += 1; i += s)
//   6. box:    first axis (x, y, z) with g < 0 (face 2d) or g >= n (face 2d+1)
//              -> escaped. For the crater terrain, z < 0 is not an escape.
//   7. object: sphere |g - c|^2 <= R^2, or crater (z < 0) or (z <= z_flat and
//              |g - zc|^2 >= Rc^2) -> absorbed, counted in its bin: the
//              crater's surface column (i, j); the sphere's one bin, or with
//              m patches its surface patch (sphere_patch below).
//   8. deposit (after all particles moved): rho is zeroed, then every alive
//      particle adds its charge chg = q*w times W[n] at its new position.
//      Fixed-point mode: C[n] = llrint(chg*W[n] * 2^32) for n < 7 and
//      C[7] = llrint(chg * 2^32) - sum_{n<7} C[n], added to int64 rhoF;
//      output rho = rhoF * 2^-32 / h^3.
//
// Global boundaries (the particle setups of §3.1.3 and §5.2.2):
//   * reflection: a face in the `reflect` mask mirrors a particle that crossed
//     it (position about the face, normal velocity negated), right after the
//     drift and before the box / object tests, axes x, y, z in turn;
//   * injection: faces in `inj_faces` feed ambient particles of a drifting
//     Maxwellian (density n, thermal speed vth, drift u per species) each step,
//     after every loaded particle was pushed and before the deposit. The paper
//     gives no method; this oracle uses a ghost layer: per face cell, a slab of
//     thickness L = min(1, dt (max(0, u.n_in) + 6 vth)) outside the face holds
//     floor(n L + U) ghost particles uniform in the slab with velocities drawn
//     from the drifting Maxwellian (the first normal drawn is the component
//     along the face normal); each moves dt (g' = fma(v, dt, g)) and is
//     injected if it ends inside the box (the terrain's z < 0 counts as inside
//     and is then collected), rounded to the form's representation and tested
//     against the object like a pushed particle; it carries v as its half-step
//     velocity.
//   Random numbers: SplitMix64 (Steele, Lea and Flood, 2014) used as a
//   counter-based generator keyed by (seed, step, species, face, face cell,
//   ghost); uniforms (x >> 11) 2^-53; normals by Marsaglia's polar method with
//   ln computed by ln x = e ln 2 + 2 atanh((m - 1)/(m + 1)), m in [sqrt(1/2),
//   sqrt(2)), atanh by its Taylor series to s^23 -- only correctly rounded
//   operations, so that any implementation of the same steps gives the same bits.
//
// The arithmetic type T is double for the FP64 form and float for the two FP32
// mirrors (absolute positions; int32 cell + float offset). The same expression
// order is used in every form. Build with -ffp-contract=off so that no
// multiply-add is fused unless written as fma.
//
// Threads (orc_config.threads > 1, OpenMP): the particles' updates of one
// step are independent of each other (each reads the fixed node field and its
// own state), so steps 1-7 run for the particles in parallel, the removal
// counters being integer sums; the fixed-point deposit sums each thread's
// particles into its own int64 rho, and the threads' arrays are added in
// thread order. Integer addition is associative, so every result is the same
// bit for bit as on one thread. The injection and the FP32 / FP64 summing
// deposits (whose rounding depends on the order) stay on one thread.

#include <omp.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr double kFix = 4294967296.0;  // 2^32
constexpr int kMaxSpecies = 4;

enum { REPR_FP64 = 0, REPR_FP32_ABS = 1, REPR_FP32_CELL = 2 };
enum { DEP_FIXED64 = 0, DEP_FP32 = 1, DEP_FP64 = 2 };
enum { OBJ_NONE = 0, OBJ_SPHERE = 1, OBJ_CRATER = 2 };
enum { ORC_OK = 0, ORC_E_INVALID = -1, ORC_E_CAPACITY = -2, ORC_E_RANGE = -5 };

}  // namespace

extern "C" {

typedef struct {
  int32_t nx, ny, nz;
  double h;
  double origin[3];
  double dt;
  int32_t n_species;
  double q[kMaxSpecies], m[kMaxSpecies], w[kMaxSpecies];
  int32_t obj_kind;  // 0 none, 1 sphere, 2 crater
  double center[3];  // sphere centre; crater axis at (center[0], center[1])
  double radius;     // sphere radius
  double z_flat, rim_radius, depth;  // crater: flat ground height, bowl radius, depth
  int32_t repr;      // 0 FP64, 1 FP32 absolute, 2 FP32 cell-relative
  int32_t deposit;   // 0 fixed-point int64, 1 FP32 sum, 2 FP64 sum
  int32_t reflect;   // bit f: box face f (x-, x+, y-, y+, z-, z+) reflects
  int32_t inj_faces; // bit f: box face f injects ambient particles
  uint64_t inj_seed;
  double inj_density[kMaxSpecies];  // particles per unit volume
  double inj_vth[kMaxSpecies];      // thermal speed per component
  double inj_drift[kMaxSpecies][3];
  int32_t sphere_patches;  // sphere: 0 one bin; m > 0: 6 m^2 surface patches
  int32_t pe_species;      // crater: photoelectron species, -1 none
  uint64_t pe_seed;
  double pe_sun[3];        // direction towards the Sun (any length, z > 0)
  double pe_flux;          // emitted particles per unit area and time at normal incidence
  double pe_vth;           // thermal speed of the emitted half-Maxwellian
  int32_t first_step;      // index of the run's first step: the random draws of injection
                           // and photoemission are keyed by the step index, so a run
                           // continued from step k draws what one long run draws there
  int32_t threads;         // OpenMP threads for the particle updates and the
                           // fixed-point deposit (0 or 1: one thread)
} orc_config;

typedef struct {
  double *x, *y, *z, *vx, *vy, *vz;  // n: final state, physical units
  int32_t *fate;                     // n: 0 alive, 1 escaped, 2 absorbed
  int32_t *where;                    // n: face (escaped) or bin (absorbed), else -1
  int32_t *when;                     // n: step of removal (0-based), else -1
  double *rho;                       // nodes: charge density
  int64_t *rho_fixed;                // nodes: fixed-point rho (fixed mode), may be null
  int64_t *tally;                    // nbins * n_species: absorbed counts [bin][s]
  int64_t *escaped;                  // 6 * n_species: escaped counts [face][s]
  int64_t cap;                       // capacity of the per-particle arrays (>= n)
  int64_t n_out;                     // particles written: the n loaded, then the
                                     // injected ones in injection order
  int32_t *species;                  // cap: species of every written particle
  int64_t *injected;                 // n_species: particles injected (incl. collected)
} orc_out;

// The object as an interface of the field problem (orc_field_solve), in the
// field mesh's cell units with node 0 at the origin.
typedef struct {
  int32_t kind;                      // 0 none, 1 sphere, 2 crater terrain
  double center[3];                  // sphere centre; crater axis at (center[0], center[1])
  double radius;                     // sphere
  double z_flat, rim_radius, depth;  // crater
  double eps_in;                     // permittivity inside the object (> 0)
} orc_field_object;

}  // extern "C"

namespace {

inline float fma_t(float a, float b, float c) { return std::fmaf(a, b, c); }
inline double fma_t(double a, double b, double c) { return std::fma(a, b, c); }
inline float floor_t(float a) { return std::floor(a); }
inline double floor_t(double a) { return std::floor(a); }

// Trilinear (cloud-in-cell) weights of the 8 corners of a cell, corner
// n = a + 2b + 4c at offset (a, b, c).
template <class T>
void weights(const T f[3], T W[8]) {
  const T wx[2] = {T(1) - f[0], f[0]};
  const T wy[2] = {T(1) - f[1], f[1]};
  const T wz[2] = {T(1) - f[2], f[2]};
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) W[a + 2 * b + 4 * c] = (wx[a] * wy[b]) * wz[c];
}

struct Mesh {
  int32_t n[3];
  int64_t sx, sy;  // node strides: node(i,j,k) = i + sx*j + sy*k
  int64_t nodes() const { return sy * (n[2] + 1); }
  int64_t node(int64_t i, int64_t j, int64_t k) const { return i + sx * j + sy * k; }
};

Mesh make_mesh(const orc_config& c) {
  Mesh m;
  m.n[0] = c.nx; m.n[1] = c.ny; m.n[2] = c.nz;
  m.sx = c.nx + 1;
  m.sy = (int64_t)(c.nx + 1) * (c.ny + 1);
  return m;
}

// Node indices of the 8 corners of cell (i, j, k), same corner order as weights().
void corners(const Mesh& m, const int32_t i[3], int64_t idx[8]) {
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) idx[a + 2 * b + 4 * c] = m.node(i[0] + a, i[1] + b, i[2] + c);
}

template <class T>
void gather(const T* E[3], const int64_t idx[8], const T W[8], T out[3]) {
  for (int d = 0; d < 3; ++d) {
    T acc = W[0] * E[d][idx[0]];
    for (int n = 1; n < 8; ++n) acc = fma_t(W[n], E[d][idx[n]], acc);
    out[d] = acc;
  }
}

// Fixed-point contributions (scale 2^32) of one particle: round half to even,
// and the remainder of the rounded total charge goes to corner 7 so that the
// eight contributions sum exactly to llrint(chg * 2^32).
template <class T>
void fixed_contrib(T chg, const T W[8], int64_t C[8]) {
  int64_t sum = 0;
  for (int n = 0; n < 7; ++n) {
    const T cw = chg * W[n];
    C[n] = std::llrint((double)cw * kFix);
    sum += C[n];
  }
  C[7] = std::llrint((double)chg * kFix) - sum;
}

// Per-species constants in the arithmetic type of the form.
template <class T>
struct SpeciesConst {
  T qmdt;  // q/m * dt / h
  T chg;   // q * w
};

// Object geometry in cell units, rounded to the arithmetic type of the form.
template <class T>
struct Geometry {
  int kind;
  int patches;  // sphere surface patches per cube-face edge (0: one bin)
  T c[3];    // sphere centre / crater axis (x, y); c[2] = bowl sphere centre height
  T r2;      // sphere R^2 / crater bowl-sphere Rc^2
  T z_flat;  // crater flat ground
  // integer + fractional split for the cell-relative form
  int32_t ci[3];
  T cf[3];
  int32_t zfi;
  T zff;
};

template <class T>
Geometry<T> make_geometry(const orc_config& cfg) {
  Geometry<T> g{};
  g.kind = cfg.obj_kind;
  g.patches = cfg.obj_kind == OBJ_SPHERE ? cfg.sphere_patches : 0;
  double c[3] = {0, 0, 0}, r2 = 0, zf = 0;
  if (cfg.obj_kind == OBJ_SPHERE) {
    for (int d = 0; d < 3; ++d) c[d] = (cfg.center[d] - cfg.origin[d]) / cfg.h;
    const double R = cfg.radius / cfg.h;
    r2 = R * R;
  } else if (cfg.obj_kind == OBJ_CRATER) {
    // Spherical bowl of radius a (at the flat level) and depth d below the flat
    // ground z_flat: its sphere has radius Rc = (a^2 + d^2) / (2d) and centre
    // height zc = z_flat - d + Rc.
    const double a = cfg.rim_radius / cfg.h, dep = cfg.depth / cfg.h;
    zf = (cfg.z_flat - cfg.origin[2]) / cfg.h;
    const double Rc = (a * a + dep * dep) / (2.0 * dep);
    c[0] = (cfg.center[0] - cfg.origin[0]) / cfg.h;
    c[1] = (cfg.center[1] - cfg.origin[1]) / cfg.h;
    c[2] = zf - dep + Rc;
    r2 = Rc * Rc;
  }
  for (int d = 0; d < 3; ++d) {
    g.c[d] = (T)c[d];
    g.ci[d] = (int32_t)std::floor(c[d]);
    g.cf[d] = (T)(c[d] - g.ci[d]);
  }
  g.r2 = (T)r2;
  g.z_flat = (T)zf;
  g.zfi = (int32_t)std::floor(zf);
  g.zff = (T)(zf - g.zfi);
  return g;
}

// ---- object predicates ------------------------------------------------------

template <class T>
T dist2(const T d[3]) {
  return fma_t(d[2], d[2], fma_t(d[1], d[1], d[0] * d[0]));
}

// Surface patch of a collected particle on a sphere with m patches per
// cube-face edge (6 m^2 patches; the per-patch collected charge is the
// surface charge distribution behind the flux jump of eq. (2.5)). d is the
// particle's offset from the centre; its direction is projected on the cube
// around the sphere (gnomonic cube map): the face is that of the largest |d_a|
// (ties to the lower axis; face 2a for d_a < 0, 2a + 1 otherwise), and the
// two other components, in axis order and divided by |d_a|, lie in [-1, 1]
// and are cut into m equal intervals each. Only correctly rounded operations,
// in the form's type.
template <class T>
int32_t sphere_patch(const T d[3], int m) {
  const T a[3] = {std::fabs(d[0]), std::fabs(d[1]), std::fabs(d[2])};
  int ax = 0;
  if (a[1] > a[ax]) ax = 1;
  if (a[2] > a[ax]) ax = 2;
  const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
  const int face = 2 * ax + (d[ax] < T(0) ? 0 : 1);
  T su = T(0), sv = T(0);
  if (a[ax] > T(0)) {
    su = d[u] / a[ax];
    sv = d[v] / a[ax];
  }
  const T half = (T)(0.5 * m);
  auto cell = [&](T t) {
    const int k = (int)floor_t((t + T(1)) * half);
    return k < 0 ? 0 : (k > m - 1 ? m - 1 : k);
  };
  return (int32_t)((face * m + cell(sv)) * m + cell(su));
}

// Absolute-position forms. Returns the bin (>= 0) when absorbed, else -1.
template <class T>
int32_t object_hit_abs(const Geometry<T>& G, const Mesh& m, const T g[3]) {
  if (G.kind == OBJ_SPHERE) {
    const T d[3] = {g[0] - G.c[0], g[1] - G.c[1], g[2] - G.c[2]};
    if (!(dist2(d) <= G.r2)) return -1;
    return G.patches ? sphere_patch(d, G.patches) : 0;
  }
  if (G.kind == OBJ_CRATER) {
    bool hit = g[2] < T(0);
    if (!hit && g[2] <= G.z_flat) {
      const T d[3] = {g[0] - G.c[0], g[1] - G.c[1], g[2] - G.c[2]};
      hit = dist2(d) >= G.r2;
    }
    if (!hit) return -1;
    int64_t ix = (int64_t)floor_t(g[0]), iy = (int64_t)floor_t(g[1]);
    ix = ix < 0 ? 0 : (ix > m.n[0] - 1 ? m.n[0] - 1 : ix);
    iy = iy < 0 ? 0 : (iy > m.n[1] - 1 ? m.n[1] - 1 : iy);
    return (int32_t)(ix + (int64_t)m.n[0] * iy);
  }
  return -1;
}

// Cell-relative form: a coordinate minus a constant c = ci + cf is
// (float)(i - ci) + (o - cf).
int32_t object_hit_cell(const Geometry<float>& G, const Mesh& m, const int32_t i[3],
                        const float o[3]) {
  if (G.kind == OBJ_SPHERE) {
    float d[3];
    for (int k = 0; k < 3; ++k) d[k] = (float)(i[k] - G.ci[k]) + (o[k] - G.cf[k]);
    if (!(dist2(d) <= G.r2)) return -1;
    return G.patches ? sphere_patch(d, G.patches) : 0;
  }
  if (G.kind == OBJ_CRATER) {
    bool hit = i[2] < 0;
    if (!hit) {
      const float zrel = (float)(i[2] - G.zfi) + (o[2] - G.zff);
      if (zrel <= 0.0f) {
        float d[3];
        for (int k = 0; k < 3; ++k) d[k] = (float)(i[k] - G.ci[k]) + (o[k] - G.cf[k]);
        hit = dist2(d) >= G.r2;
      }
    }
    if (!hit) return -1;
    int64_t ix = i[0] < 0 ? 0 : (i[0] > m.n[0] - 1 ? m.n[0] - 1 : i[0]);
    int64_t iy = i[1] < 0 ? 0 : (i[1] > m.n[1] - 1 ? m.n[1] - 1 : i[1]);
    return (int32_t)(ix + (int64_t)m.n[0] * iy);
  }
  return -1;
}

// ---- box exit ----------------------------------------------------------------

// First offending axis in x, y, z order, lower face before upper face.
// For the crater terrain the z-lower face is not an exit (absorbed instead).
template <class T>
int box_face_abs(const Mesh& m, const T g[3], bool crater) {
  for (int d = 0; d < 3; ++d) {
    if (g[d] < T(0) && !(crater && d == 2)) return 2 * d;
    if (g[d] >= (T)m.n[d]) return 2 * d + 1;
  }
  return -1;
}

int box_face_cell(const Mesh& m, const int32_t i[3], bool crater) {
  for (int d = 0; d < 3; ++d) {
    if (i[d] < 0 && !(crater && d == 2)) return 2 * d;
    if (i[d] >= m.n[d]) return 2 * d + 1;
  }
  return -1;
}

// ---- global boundaries: random numbers -------------------------------------------

constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ULL;

// SplitMix64 output function (the generator's state increment is kGolden).
uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Key of one ghost particle (j >= 1) or of a face cell's count draw (j = 0).
uint64_t inj_key(uint64_t seed, int32_t step, int s, int f, int64_t cell, int64_t j) {
  uint64_t k = sm_mix(seed + kGolden);
  k = sm_mix(k ^ (uint64_t)(uint32_t)step);
  k = sm_mix(k ^ (uint64_t)(s * 8 + f));
  k = sm_mix(k ^ (uint64_t)cell);
  return sm_mix(k ^ (uint64_t)j);
}

// Draw d (0, 1, ...) of a key: uniform in [0, 1) on the 2^-53 grid.
double inj_uniform(uint64_t key, uint64_t d) {
  return (double)(sm_mix(key + (d + 1) * kGolden) >> 11) * 0x1.0p-53;
}

// Natural logarithm of x > 0 (finite): x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// ln x = e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.1716, atanh by its
// Taylor series s (1 + s^2/3 + s^4/5 + ... + s^22/23) in Horner form.
double ln_series(double x) {
  int e = 0;
  double m = std::frexp(x, &e);  // m in [0.5, 1)
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double t = s * s;
  double p = 1.0 / 23.0;
  for (int k = 21; k >= 1; k -= 2) p = p * t + 1.0 / (double)k;
  return (double)e * 0.69314718055994530942 + 2.0 * s * p;
}

// Three standard normals by Marsaglia's polar method; *d counts the draws used.
void normals3(uint64_t key, uint64_t* d, double z[3]) {
  int got = 0;
  for (int attempt = 0; attempt < 64 && got < 3; ++attempt) {
    const double a = 2.0 * inj_uniform(key, (*d)++) - 1.0;
    const double b = 2.0 * inj_uniform(key, (*d)++) - 1.0;
    const double r = a * a + b * b;
    if (!(r > 0.0 && r < 1.0)) continue;
    const double f = std::sqrt(-2.0 * ln_series(r) / r);
    z[got++] = a * f;
    if (got < 3) z[got++] = b * f;
  }
  while (got < 3) z[got++] = 0.0;  // 64 rejected pairs: probability 0.2146^64
}

// Injection geometry of one face in cell units.
struct InjFace {
  int f, axis, t1, t2;  // face, its normal axis, the two tangential axes
  bool max_side;        // face at n[axis] (else at 0)
  int64_t cells;        // n[t1] * n[t2]
};

InjFace inj_face(const int32_t n[3], int f) {
  InjFace F;
  F.f = f;
  F.axis = f / 2;
  F.max_side = (f & 1) != 0;
  F.t1 = F.axis == 0 ? 1 : 0;
  F.t2 = F.axis == 2 ? 1 : 2;
  F.cells = (int64_t)n[F.t1] * n[F.t2];
  return F;
}

// Per-species injection constants in cell units (from physical inputs).
struct InjSpecies {
  double ncell;   // particles per cell volume
  double vth;     // cell units per unit time
  double u[3];
};

InjSpecies inj_species(const orc_config& c, int s) {
  InjSpecies I;
  const double h3 = c.h * c.h * c.h;
  I.ncell = c.inj_density[s] * h3;
  I.vth = c.inj_vth[s] / c.h;
  for (int d = 0; d < 3; ++d) I.u[d] = c.inj_drift[s][d] / c.h;
  return I;
}

// Ghost-slab thickness of a face for a species.
double inj_thickness(const InjSpecies& I, const InjFace& F, double dt) {
  const double un = F.max_side ? -I.u[F.axis] : I.u[F.axis];
  double L = dt * ((un > 0.0 ? un : 0.0) + 6.0 * I.vth);
  if (L > 1.0) L = 1.0;
  return L;
}

// Visits every ghost particle of one step that ends inside the box, in the
// order species, face, face cell, ghost: emit(s, g[3], v[3]) in cell units.
template <class Emit>
void inject_ghosts(const orc_config& cfg, const int32_t n[3], int32_t step, Emit emit) {
  for (int s = 0; s < cfg.n_species; ++s) {
    const InjSpecies I = inj_species(cfg, s);
    if (!(I.ncell > 0.0)) continue;
    for (int f = 0; f < 6; ++f) {
      if (!((cfg.inj_faces >> f) & 1)) continue;
      const InjFace F = inj_face(n, f);
      const double L = inj_thickness(I, F, cfg.dt);
      const double mean = I.ncell * L;
      for (int64_t cell = 0; cell < F.cells; ++cell) {
        const int64_t a = cell % n[F.t1], b = cell / n[F.t1];
        const int64_t k = (int64_t)std::floor(mean + inj_uniform(inj_key(cfg.inj_seed, step, s, f, cell, 0), 0));
        for (int64_t j = 1; j <= k; ++j) {
          const uint64_t key = inj_key(cfg.inj_seed, step, s, f, cell, j);
          double g[3], v[3], z[3];
          g[F.t1] = (double)a + inj_uniform(key, 0);
          g[F.t2] = (double)b + inj_uniform(key, 1);
          const double depth = L * (1.0 - inj_uniform(key, 2));
          g[F.axis] = F.max_side ? (double)n[F.axis] + depth : -depth;
          uint64_t d = 3;
          normals3(key, &d, z);
          // the first normal goes to the face's normal axis, then t1, t2
          v[F.axis] = I.u[F.axis] + I.vth * z[0];
          v[F.t1] = I.u[F.t1] + I.vth * z[1];
          v[F.t2] = I.u[F.t2] + I.vth * z[2];
          for (int q = 0; q < 3; ++q) g[q] = std::fma(v[q], cfg.dt, g[q]);
          emit(s, g, v);
        }
      }
    }
  }
}

// ---- photoemission (the lunar setup of §5.2.2) -------------------------------
//
// Photoelectrons are generated at the sunlit terrain according to the local
// sunlight index, the inner product of the unit direction to the Sun s and
// the terrain's outward unit normal n, and not in shadow. The paper fixes no
// more; this oracle takes: per surface column (i, j) and step, the terrain at
// the column centre gives n, the ground height and I = s.n; the column is
// lit if I > 0 and, in the bowl, the ray from that ground point towards the
// Sun leaves the bowl sphere at or above the flat ground (a chord of length
// 2 Rc I; outside the bowl nothing rises above the ground, so it is lit).
// A lit column emits floor(mean + U) photoelectrons with
// mean = (flux / w) h^2 dt I / n_z (the flux at normal incidence times the
// cosine of incidence over the column's terrain area h^2 / n_z). Each starts
// at a uniform point of the column's footprint on the ground, with a
// half-Maxwellian velocity about n (vth (|z0| n + z1 t1 + z2 t2), t1 =
// (n_z, 0, -n_x) normalised, t2 = n x t1), and moves a uniform fraction of dt
// (g = fma(v, dt U, ground point)); then it is handled like an injected
// particle (the box and terrain tests, appended after the ambient injection).
// Random numbers: the injection's keys with face index 6 for the column:
// draw 0 of ghost 0 for the count; draws 0, 1 (footprint), 2 (fraction) and
// normals from draw 3 for ghost q >= 1.

struct PhotoSetup {
  bool on = false;
  int s = 0;
  uint64_t seed = 0;
  double sun[3] = {0, 0, 0};
  double rate = 0.0, vth = 0.0;  // rate = (flux / w) h^2 dt; vth in cell units
  double cx = 0, cy = 0, zc = 0, rc = 0, rc2 = 0, a2 = 0, z_flat = 0;  // terrain, cell units
};

PhotoSetup photo_setup(const orc_config& c) {
  PhotoSetup P;
  if (c.obj_kind != OBJ_CRATER || c.pe_species < 0) return P;
  P.on = true;
  P.s = c.pe_species;
  P.seed = c.pe_seed;
  const double len =
      std::sqrt(c.pe_sun[0] * c.pe_sun[0] + c.pe_sun[1] * c.pe_sun[1] + c.pe_sun[2] * c.pe_sun[2]);
  for (int d = 0; d < 3; ++d) P.sun[d] = c.pe_sun[d] / len;
  P.rate = (c.pe_flux / c.w[P.s]) * (c.h * c.h) * c.dt;
  P.vth = c.pe_vth / c.h;
  const double a = c.rim_radius / c.h, dep = c.depth / c.h;
  P.rc = (a * a + dep * dep) / (2.0 * dep);
  P.rc2 = P.rc * P.rc;
  P.a2 = a * a;
  P.z_flat = (c.z_flat - c.origin[2]) / c.h;
  P.zc = P.z_flat - dep + P.rc;
  P.cx = (c.center[0] - c.origin[0]) / c.h;
  P.cy = (c.center[1] - c.origin[1]) / c.h;
  return P;
}

double photo_ground(const PhotoSetup& P, double x, double y) {
  const double dx = x - P.cx, dy = y - P.cy;
  const double r2 = dx * dx + dy * dy;
  return r2 < P.a2 ? P.zc - std::sqrt(P.rc2 - r2) : P.z_flat;
}

// Terrain at the centre of column (i, j): outward normal, ground height,
// sunlight index and whether the column is lit.
void photo_column(const PhotoSetup& P, int64_t i, int64_t j, double n[3], double* zg, double* I,
                  bool* lit) {
  const double dx = ((double)i + 0.5) - P.cx, dy = ((double)j + 0.5) - P.cy;
  const double r2 = dx * dx + dy * dy;
  const bool bowl = r2 < P.a2;
  if (bowl) {
    *zg = P.zc - std::sqrt(P.rc2 - r2);
    n[0] = -dx / P.rc;
    n[1] = -dy / P.rc;
    n[2] = (P.zc - *zg) / P.rc;
  } else {
    *zg = P.z_flat;
    n[0] = 0.0;
    n[1] = 0.0;
    n[2] = 1.0;
  }
  *I = (P.sun[0] * n[0] + P.sun[1] * n[1]) + P.sun[2] * n[2];
  *lit = *I > 0.0 && (!bowl || *zg + (2.0 * P.rc * *I) * P.sun[2] >= P.z_flat);
}

// Visits every photoelectron of one step in column order: emit(s, g, v).
template <class Emit>
void photo_emit(const orc_config& cfg, const int32_t n[3], int32_t step, Emit emit) {
  const PhotoSetup P = photo_setup(cfg);
  if (!P.on) return;
  for (int64_t col = 0; col < (int64_t)n[0] * n[1]; ++col) {
    const int64_t i = col % n[0], j = col / n[0];
    double nr[3], zg, I;
    bool lit;
    photo_column(P, i, j, nr, &zg, &I, &lit);
    if (!lit) continue;
    const double mean = (P.rate * I) / nr[2];
    const int64_t k =
        (int64_t)std::floor(mean + inj_uniform(inj_key(P.seed, step, P.s, 6, col, 0), 0));
    const double l1 = std::sqrt(nr[2] * nr[2] + nr[0] * nr[0]);
    const double t1[3] = {nr[2] / l1, 0.0, -nr[0] / l1};
    const double t2[3] = {nr[1] * t1[2] - nr[2] * t1[1], nr[2] * t1[0] - nr[0] * t1[2],
                          nr[0] * t1[1] - nr[1] * t1[0]};
    for (int64_t q = 1; q <= k; ++q) {
      const uint64_t key = inj_key(P.seed, step, P.s, 6, col, q);
      const double x = (double)i + inj_uniform(key, 0), y = (double)j + inj_uniform(key, 1);
      const double z0 = photo_ground(P, x, y);
      const double tau = cfg.dt * inj_uniform(key, 2);
      uint64_t d = 3;
      double z[3];
      normals3(key, &d, z);
      const double a0 = std::fabs(z[0]);
      double v[3], g[3];
      for (int c = 0; c < 3; ++c) v[c] = P.vth * ((a0 * nr[c] + z[1] * t1[c]) + z[2] * t2[c]);
      g[0] = std::fma(v[0], tau, x);
      g[1] = std::fma(v[1], tau, y);
      g[2] = std::fma(v[2], tau, z0);
      emit(P.s, g, v);
    }
  }
}

// Mirror about a reflecting face; absolute positions (cell units).
template <class T>
void reflect_abs(const orc_config& cfg, const int32_t n[3], T g[3], T u[3]) {
  for (int d = 0; d < 3; ++d) {
    if (((cfg.reflect >> (2 * d)) & 1) && g[d] < T(0)) {
      g[d] = -g[d];
      u[d] = -u[d];
    }
    if (((cfg.reflect >> (2 * d + 1)) & 1) && g[d] >= (T)n[d]) {
      g[d] = (T)(2 * n[d]) - g[d];
      if (g[d] >= (T)n[d]) g[d] = std::nextafter((T)n[d], T(0));
      u[d] = -u[d];
    }
  }
}

// Mirror about a reflecting face; cell-relative form (cell i, offset o).
void reflect_cell(const orc_config& cfg, const int32_t n[3], int32_t i[3], float o[3], float u[3]) {
  for (int d = 0; d < 3; ++d) {
    const bool lo = ((cfg.reflect >> (2 * d)) & 1) && i[d] < 0;
    const bool hi = ((cfg.reflect >> (2 * d + 1)) & 1) && i[d] >= n[d];
    if (!lo && !hi) continue;
    const int32_t m = lo ? 0 : 2 * n[d];  // position -> m - position
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
    if (hi && i[d] >= n[d]) {  // exactly on the face: just inside
      i[d] = n[d] - 1;
      o[d] = std::nextafter(1.0f, 0.0f);
    }
    u[d] = -u[d];
  }
}

// ---- deposit -----------------------------------------------------------------

struct RhoAcc {
  int mode;
  std::vector<int64_t> fixed;
  std::vector<float> f32;
  std::vector<double> f64;
  void reset(int64_t nodes) {
    if (mode == DEP_FIXED64) fixed.assign(nodes, 0);
    if (mode == DEP_FP32) f32.assign(nodes, 0.0f);
    if (mode == DEP_FP64) f64.assign(nodes, 0.0);
  }
  template <class T>
  void add(const int64_t idx[8], const T W[8], T chg) {
    if (mode == DEP_FIXED64) {
      add_fixed(fixed.data(), idx, W, chg);
    } else if (mode == DEP_FP32) {
      for (int n = 0; n < 8; ++n) f32[idx[n]] += (float)(chg * W[n]);
    } else {
      for (int n = 0; n < 8; ++n) f64[idx[n]] += (double)(chg * W[n]);
    }
  }
  template <class T>
  static void add_fixed(int64_t* r, const int64_t idx[8], const T W[8], T chg) {
    int64_t C[8];
    fixed_contrib(chg, W, C);
    for (int n = 0; n < 8; ++n) r[idx[n]] += C[n];
  }
};

// Number of threads a run uses.
int run_threads(const orc_config& cfg) { return cfg.threads > 1 ? cfg.threads : 1; }

// The deposit of every alive particle (alive(p), contribution by
// at(p, idx, W, chg)): in index order on one thread; with several threads
// and the fixed-point mode, each thread's particles into its own int64 array
// (part), the arrays added in thread order.
template <class T, class Alive, class At>
void deposit_particles(RhoAcc& rho, std::vector<std::vector<int64_t>>& part, int nthr,
                       int64_t np, int64_t nodes, Alive alive, At at) {
  rho.reset(nodes);
  if (nthr <= 1 || rho.mode != DEP_FIXED64) {
    for (int64_t p = 0; p < np; ++p) {
      if (!alive(p)) continue;
      int64_t idx[8];
      T W[8], chg;
      at(p, idx, W, &chg);
      rho.add(idx, W, chg);
    }
    return;
  }
  part.resize(nthr);
#pragma omp parallel num_threads(nthr)
  {
    std::vector<int64_t>& r = part[omp_get_thread_num()];
    r.assign(nodes, 0);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
      if (!alive(p)) continue;
      int64_t idx[8];
      T W[8], chg;
      at(p, idx, W, &chg);
      RhoAcc::add_fixed(r.data(), idx, W, chg);
    }
  }
#pragma omp parallel for schedule(static) num_threads(nthr)
  for (int64_t k = 0; k < nodes; ++k) {
    int64_t a = 0;
    for (int t = 0; t < nthr; ++t) a += part[t][k];
    rho.fixed[k] = a;
  }
}

// ---- particle state of each form -----------------------------------------------

template <class T>
struct AbsState {  // FP64 or FP32 absolute positions in cell units
  std::vector<T> g[3], u[3];
};

struct CellState {  // int32 cell + FP32 offset in [0, 1)
  std::vector<int32_t> i[3];
  std::vector<float> o[3], u[3];
};

bool finite3(const double* a) {
  return std::isfinite(a[0]) && std::isfinite(a[1]) && std::isfinite(a[2]);
}

// Shared driver bookkeeping: fates and counters.
struct Book {
  std::vector<int32_t> fate, where, when;
  std::vector<int64_t> tally, escaped;
};

template <class T>
int run_abs(const orc_config& cfg, int64_t n, const int32_t* sp, const double* const xin[3],
            const double* const vin[3], const double* const Ein[3], int32_t nsteps,
            orc_out* out) {
  const Mesh M = make_mesh(cfg);
  const int64_t nodes = M.nodes();
  const int ns = cfg.n_species;
  const bool crater = cfg.obj_kind == OBJ_CRATER;
  const Geometry<T> G = make_geometry<T>(cfg);
  const int64_t nbins =
      crater ? (int64_t)cfg.nx * cfg.ny
             : (cfg.obj_kind != OBJ_SPHERE
                    ? 0
                    : (cfg.sphere_patches > 0 ? 6 * (int64_t)cfg.sphere_patches * cfg.sphere_patches
                                              : 1));
  std::vector<T> E[3];
  for (int d = 0; d < 3; ++d) {
    E[d].resize(nodes);
    for (int64_t k = 0; k < nodes; ++k) E[d][k] = (T)Ein[d][k];
  }
  const T* Ep[3] = {E[0].data(), E[1].data(), E[2].data()};
  SpeciesConst<T> S[kMaxSpecies];
  for (int s = 0; s < ns; ++s) {
    S[s].qmdt = (T)(cfg.q[s] / cfg.m[s] * cfg.dt / cfg.h);
    S[s].chg = (T)(cfg.q[s] * cfg.w[s]);
  }
  const T dt = (T)cfg.dt;

  AbsState<T> P;
  for (int d = 0; d < 3; ++d) {
    P.g[d].resize(n);
    P.u[d].resize(n);
    for (int64_t p = 0; p < n; ++p) {
      P.g[d][p] = (T)((xin[d][p] - cfg.origin[d]) / cfg.h);
      P.u[d][p] = (T)(vin[d][p] / cfg.h);
    }
  }
  std::vector<int32_t> spv(sp, sp + n);
  Book B;
  B.fate.assign(n, 0);
  B.where.assign(n, -1);
  B.when.assign(n, -1);
  B.tally.assign(nbins * ns, 0);
  B.escaped.assign(6 * ns, 0);
  std::vector<int64_t> injected(ns, 0);
  RhoAcc rho;
  rho.mode = cfg.deposit;

  // an injected particle (cell units, FP64) in this form's arithmetic
  auto inject = [&](int32_t step) {
    const auto add = [&](int s, const double gd[3], const double vd[3]) {
      const T g[3] = {(T)gd[0], (T)gd[1], (T)gd[2]};
      if (box_face_abs(M, g, crater) >= 0) return;  // did not enter the box
      injected[s] += 1;
      for (int d = 0; d < 3; ++d) {
        P.g[d].push_back(g[d]);
        P.u[d].push_back((T)vd[d]);
      }
      spv.push_back(s);
      const int32_t bin = object_hit_abs(G, M, g);
      B.fate.push_back(bin >= 0 ? 2 : 0);
      B.where.push_back(bin);
      B.when.push_back(bin >= 0 ? step : -1);
      if (bin >= 0) B.tally[(int64_t)bin * ns + s] += 1;
    };
    inject_ghosts(cfg, M.n, cfg.first_step + step, add);
    photo_emit(cfg, M.n, cfg.first_step + step, add);
  };

  const int nthr = run_threads(cfg);
  std::vector<std::vector<int64_t>> part;
  auto deposit_all = [&]() {
    deposit_particles<T>(
        rho, part, nthr, (int64_t)spv.size(), nodes, [&](int64_t p) { return B.fate[p] == 0; },
        [&](int64_t p, int64_t* idx, T* W, T* chg) {
          T g[3] = {P.g[0][p], P.g[1][p], P.g[2][p]};
          int32_t i[3];
          T f[3];
          for (int d = 0; d < 3; ++d) {
            i[d] = (int32_t)floor_t(g[d]);
            f[d] = g[d] - (T)i[d];
          }
          weights(f, W);
          corners(M, i, idx);
          *chg = S[spv[p]].chg;
        });
  };

  for (int32_t step = 0; step < nsteps; ++step) {
    const int64_t np = (int64_t)spv.size();
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(nthr) if (nthr > 1)
    for (int64_t p = 0; p < np; ++p) {
      if (B.fate[p] != 0) continue;
      const int s = spv[p];
      T g[3] = {P.g[0][p], P.g[1][p], P.g[2][p]};
      T u[3] = {P.u[0][p], P.u[1][p], P.u[2][p]};
      int32_t i[3];
      T f[3];
      for (int d = 0; d < 3; ++d) {
        i[d] = (int32_t)floor_t(g[d]);
        f[d] = g[d] - (T)i[d];
      }
      T W[8];
      weights(f, W);
      int64_t idx[8];
      corners(M, i, idx);
      T Epart[3];
      gather(Ep, idx, W, Epart);
      for (int d = 0; d < 3; ++d) u[d] = fma_t(S[s].qmdt, Epart[d], u[d]);
      for (int d = 0; d < 3; ++d) g[d] = fma_t(u[d], dt, g[d]);
      const double gd[3] = {(double)g[0], (double)g[1], (double)g[2]};
      if (!finite3(gd)) {
#pragma omp atomic write
        bad = 1;
        continue;
      }
      if (cfg.reflect) reflect_abs(cfg, M.n, g, u);
      for (int d = 0; d < 3; ++d) {
        P.g[d][p] = g[d];
        P.u[d][p] = u[d];
      }
      const int face = box_face_abs(M, g, crater);
      if (face >= 0) {
        B.fate[p] = 1;
        B.where[p] = face;
        B.when[p] = step;
#pragma omp atomic
        B.escaped[face * ns + s] += 1;
        continue;
      }
      const int32_t bin = object_hit_abs(G, M, g);
      if (bin >= 0) {
        B.fate[p] = 2;
        B.where[p] = bin;
        B.when[p] = step;
#pragma omp atomic
        B.tally[(int64_t)bin * ns + s] += 1;
      }
    }
    if (bad) return ORC_E_RANGE;
    if (cfg.inj_faces || (crater && cfg.pe_species >= 0)) inject(step);
    deposit_all();
  }
  if (nsteps == 0) deposit_all();

  // outputs
  const int64_t nout = (int64_t)spv.size();
  if (nout > out->cap) return ORC_E_CAPACITY;
  out->n_out = nout;
  for (int s = 0; s < ns; ++s)
    if (out->injected) out->injected[s] = injected[s];
  for (int64_t p = 0; p < nout; ++p) {
    if (out->species) out->species[p] = spv[p];
    out->x[p] = cfg.origin[0] + (double)P.g[0][p] * cfg.h;
    out->y[p] = cfg.origin[1] + (double)P.g[1][p] * cfg.h;
    out->z[p] = cfg.origin[2] + (double)P.g[2][p] * cfg.h;
    out->vx[p] = (double)P.u[0][p] * cfg.h;
    out->vy[p] = (double)P.u[1][p] * cfg.h;
    out->vz[p] = (double)P.u[2][p] * cfg.h;
    out->fate[p] = B.fate[p];
    out->where[p] = B.where[p];
    out->when[p] = B.when[p];
  }
  const double h3 = cfg.h * cfg.h * cfg.h;
  for (int64_t k = 0; k < nodes; ++k) {
    if (cfg.deposit == DEP_FIXED64) {
      out->rho[k] = ((double)rho.fixed[k] * (1.0 / kFix)) / h3;
      if (out->rho_fixed) out->rho_fixed[k] = rho.fixed[k];
    } else if (cfg.deposit == DEP_FP32) {
      out->rho[k] = (double)rho.f32[k] / h3;
    } else {
      out->rho[k] = rho.f64[k] / h3;
    }
  }
  if (!B.tally.empty()) std::memcpy(out->tally, B.tally.data(), sizeof(int64_t) * B.tally.size());
  std::memcpy(out->escaped, B.escaped.data(), sizeof(int64_t) * B.escaped.size());
  return ORC_OK;
}

int run_cell(const orc_config& cfg, int64_t n, const int32_t* sp, const double* const xin[3],
             const double* const vin[3], const double* const Ein[3], int32_t nsteps,
             orc_out* out) {
  typedef float T;
  const Mesh M = make_mesh(cfg);
  const int64_t nodes = M.nodes();
  const int ns = cfg.n_species;
  const bool crater = cfg.obj_kind == OBJ_CRATER;
  const Geometry<T> G = make_geometry<T>(cfg);
  const int64_t nbins =
      crater ? (int64_t)cfg.nx * cfg.ny
             : (cfg.obj_kind != OBJ_SPHERE
                    ? 0
                    : (cfg.sphere_patches > 0 ? 6 * (int64_t)cfg.sphere_patches * cfg.sphere_patches
                                              : 1));
  std::vector<T> E[3];
  for (int d = 0; d < 3; ++d) {
    E[d].resize(nodes);
    for (int64_t k = 0; k < nodes; ++k) E[d][k] = (T)Ein[d][k];
  }
  const T* Ep[3] = {E[0].data(), E[1].data(), E[2].data()};
  SpeciesConst<T> S[kMaxSpecies];
  for (int s = 0; s < ns; ++s) {
    S[s].qmdt = (T)(cfg.q[s] / cfg.m[s] * cfg.dt / cfg.h);
    S[s].chg = (T)(cfg.q[s] * cfg.w[s]);
  }
  const T dt = (T)cfg.dt;

  CellState P;
  for (int d = 0; d < 3; ++d) {
    P.i[d].resize(n);
    P.o[d].resize(n);
    P.u[d].resize(n);
    for (int64_t p = 0; p < n; ++p) {
      const double gd = (xin[d][p] - cfg.origin[d]) / cfg.h;
      int32_t i = (int32_t)std::floor(gd);
      float o = (float)(gd - (double)i);
      if (o == 1.0f) {  // offset rounded up to the next cell
        o = 0.0f;
        i += 1;
      }
      P.i[d][p] = i;
      P.o[d][p] = o;
      P.u[d][p] = (T)(vin[d][p] / cfg.h);
    }
  }
  std::vector<int32_t> spv(sp, sp + n);
  Book B;
  B.fate.assign(n, 0);
  B.where.assign(n, -1);
  B.when.assign(n, -1);
  B.tally.assign(nbins * ns, 0);
  B.escaped.assign(6 * ns, 0);
  std::vector<int64_t> injected(ns, 0);
  RhoAcc rho;
  rho.mode = cfg.deposit;

  // an injected particle (cell units, FP64) in the cell-relative form
  auto inject = [&](int32_t step) {
    const auto add = [&](int s, const double gd[3], const double vd[3]) {
      int32_t i[3];
      T o[3];
      for (int d = 0; d < 3; ++d) {
        i[d] = (int32_t)std::floor(gd[d]);
        o[d] = (T)(gd[d] - (double)i[d]);
        if (o[d] == 1.0f) {
          o[d] = 0.0f;
          i[d] += 1;
        }
      }
      if (box_face_cell(M, i, crater) >= 0) return;  // did not enter the box
      injected[s] += 1;
      for (int d = 0; d < 3; ++d) {
        P.i[d].push_back(i[d]);
        P.o[d].push_back(o[d]);
        P.u[d].push_back((T)vd[d]);
      }
      spv.push_back(s);
      const int32_t bin = object_hit_cell(G, M, i, o);
      B.fate.push_back(bin >= 0 ? 2 : 0);
      B.where.push_back(bin);
      B.when.push_back(bin >= 0 ? step : -1);
      if (bin >= 0) B.tally[(int64_t)bin * ns + s] += 1;
    };
    inject_ghosts(cfg, M.n, cfg.first_step + step, add);
    photo_emit(cfg, M.n, cfg.first_step + step, add);
  };

  const int nthr = run_threads(cfg);
  std::vector<std::vector<int64_t>> part;
  auto deposit_all = [&]() {
    deposit_particles<T>(
        rho, part, nthr, (int64_t)spv.size(), nodes, [&](int64_t p) { return B.fate[p] == 0; },
        [&](int64_t p, int64_t* idx, T* W, T* chg) {
          const int32_t i[3] = {P.i[0][p], P.i[1][p], P.i[2][p]};
          const T f[3] = {P.o[0][p], P.o[1][p], P.o[2][p]};
          weights(f, W);
          corners(M, i, idx);
          *chg = S[spv[p]].chg;
        });
  };

  for (int32_t step = 0; step < nsteps; ++step) {
    const int64_t np = (int64_t)spv.size();
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(nthr) if (nthr > 1)
    for (int64_t p = 0; p < np; ++p) {
      if (B.fate[p] != 0) continue;
      const int s = spv[p];
      int32_t i[3] = {P.i[0][p], P.i[1][p], P.i[2][p]};
      T o[3] = {P.o[0][p], P.o[1][p], P.o[2][p]};
      T u[3] = {P.u[0][p], P.u[1][p], P.u[2][p]};
      T W[8];
      weights(o, W);
      int64_t idx[8];
      corners(M, i, idx);
      T Epart[3];
      gather(Ep, idx, W, Epart);
      for (int d = 0; d < 3; ++d) u[d] = fma_t(S[s].qmdt, Epart[d], u[d]);
      bool runaway = false;
      for (int d = 0; d < 3 && !runaway; ++d) {
        T op = fma_t(u[d], dt, o[d]);
        T sh = floor_t(op);
        op = op - sh;
        if (op == 1.0f) {  // a tiny negative offset rounded up to 1 after the shift
          op = 0.0f;
          sh = sh + 1.0f;
        }
        // non-finite, or more than 2^20 cells in one step
        runaway = !std::isfinite(op) || !(std::fabs(sh) <= 1048576.0f);
        o[d] = op;
        i[d] += runaway ? 0 : (int32_t)sh;
      }
      if (runaway) {
#pragma omp atomic write
        bad = 1;
        continue;
      }
      if (cfg.reflect) reflect_cell(cfg, M.n, i, o, u);
      for (int d = 0; d < 3; ++d) {
        P.i[d][p] = i[d];
        P.o[d][p] = o[d];
        P.u[d][p] = u[d];
      }
      const int face = box_face_cell(M, i, crater);
      if (face >= 0) {
        B.fate[p] = 1;
        B.where[p] = face;
        B.when[p] = step;
#pragma omp atomic
        B.escaped[face * ns + s] += 1;
        continue;
      }
      const int32_t bin = object_hit_cell(G, M, i, o);
      if (bin >= 0) {
        B.fate[p] = 2;
        B.where[p] = bin;
        B.when[p] = step;
#pragma omp atomic
        B.tally[(int64_t)bin * ns + s] += 1;
      }
    }
    if (bad) return ORC_E_RANGE;
    if (cfg.inj_faces || (crater && cfg.pe_species >= 0)) inject(step);
    deposit_all();
  }
  if (nsteps == 0) deposit_all();

  const int64_t nout = (int64_t)spv.size();
  if (nout > out->cap) return ORC_E_CAPACITY;
  out->n_out = nout;
  for (int s = 0; s < ns; ++s)
    if (out->injected) out->injected[s] = injected[s];
  for (int64_t p = 0; p < nout; ++p) {
    if (out->species) out->species[p] = spv[p];
    out->x[p] = cfg.origin[0] + ((double)P.i[0][p] + (double)P.o[0][p]) * cfg.h;
    out->y[p] = cfg.origin[1] + ((double)P.i[1][p] + (double)P.o[1][p]) * cfg.h;
    out->z[p] = cfg.origin[2] + ((double)P.i[2][p] + (double)P.o[2][p]) * cfg.h;
    out->vx[p] = (double)P.u[0][p] * cfg.h;
    out->vy[p] = (double)P.u[1][p] * cfg.h;
    out->vz[p] = (double)P.u[2][p] * cfg.h;
    out->fate[p] = B.fate[p];
    out->where[p] = B.where[p];
    out->when[p] = B.when[p];
  }
  const double h3 = cfg.h * cfg.h * cfg.h;
  for (int64_t k = 0; k < nodes; ++k) {
    if (cfg.deposit == DEP_FIXED64) {
      out->rho[k] = ((double)rho.fixed[k] * (1.0 / kFix)) / h3;
      if (out->rho_fixed) out->rho_fixed[k] = rho.fixed[k];
    } else if (cfg.deposit == DEP_FP32) {
      out->rho[k] = (double)rho.f32[k] / h3;
    } else {
      out->rho[k] = rho.f64[k] / h3;
    }
  }
  if (!B.tally.empty()) std::memcpy(out->tally, B.tally.data(), sizeof(int64_t) * B.tally.size());
  std::memcpy(out->escaped, B.escaped.data(), sizeof(int64_t) * B.escaped.size());
  return ORC_OK;
}

bool valid(const orc_config& c, int64_t n, const int32_t* sp, const double* const x[3]) {
  if (c.nx < 1 || c.ny < 1 || c.nz < 1 || !(c.h > 0) || !(c.dt > 0)) return false;
  if (c.n_species < 1 || c.n_species > kMaxSpecies) return false;
  if (c.repr < 0 || c.repr > 2 || c.deposit < 0 || c.deposit > 2) return false;
  if (c.obj_kind < 0 || c.obj_kind > 2) return false;
  if (c.obj_kind == OBJ_CRATER && !(c.depth > 0)) return false;
  for (int s = 0; s < c.n_species; ++s)
    if (!(c.m[s] > 0)) return false;
  if ((c.reflect | c.inj_faces) & ~63) return false;
  if (c.reflect & c.inj_faces) return false;             // a face reflects or injects
  if (c.obj_kind == OBJ_CRATER && ((c.reflect | c.inj_faces) & 16)) return false;  // terrain
  if (c.sphere_patches < 0 || c.sphere_patches > 64) return false;
  if (c.pe_species < -1 || c.pe_species >= c.n_species) return false;
  if (c.pe_species >= 0) {
    if (c.obj_kind != OBJ_CRATER) return false;  // photoemission from the terrain
    if (!(c.pe_flux >= 0) || !std::isfinite(c.pe_flux) || !(c.pe_vth >= 0) ||
        !std::isfinite(c.pe_vth) || !(c.w[c.pe_species] > 0))
      return false;
    if (!std::isfinite(c.pe_sun[0]) || !std::isfinite(c.pe_sun[1]) || !(c.pe_sun[2] > 0) ||
        !std::isfinite(c.pe_sun[2]))
      return false;
  }
  if (c.sphere_patches && c.obj_kind != OBJ_SPHERE) return false;
  for (int s = 0; s < c.n_species && c.inj_faces; ++s)
    if (!(c.inj_density[s] >= 0) || !(c.inj_vth[s] >= 0) || !std::isfinite(c.inj_drift[s][0]) ||
        !std::isfinite(c.inj_drift[s][1]) || !std::isfinite(c.inj_drift[s][2]))
      return false;
  const int32_t nn[3] = {c.nx, c.ny, c.nz};
  for (int64_t p = 0; p < n; ++p) {
    if (sp[p] < 0 || sp[p] >= c.n_species) return false;
    for (int d = 0; d < 3; ++d) {
      const double g = (x[d][p] - c.origin[d]) / c.h;
      if (!(g >= 0.0 && g < (double)nn[d])) return false;
    }
  }
  return true;
}

}  // namespace

extern "C" {

// Runs nsteps PIC steps on n particles (species index sp[p]); nsteps == 0 only
// deposits the loaded positions. Velocities are those at t - dt/2. Node fields
// are (nx+1)(ny+1)(nz+1) values, x fastest. Returns 0, -1 (invalid input), -2
// (more particles than out->cap after injection) or -5 (a non-finite or
// runaway position).
int orc_run(const orc_config* cfg, int64_t n, const int32_t* sp, const double* x,
            const double* y, const double* z, const double* vx, const double* vy,
            const double* vz, const double* Ex, const double* Ey, const double* Ez,
            int32_t nsteps, orc_out* out) {
  const double* xin[3] = {x, y, z};
  const double* vin[3] = {vx, vy, vz};
  const double* Ein[3] = {Ex, Ey, Ez};
  if (!cfg || !out || nsteps < 0 || n < 0 || out->cap < n || !valid(*cfg, n, sp, xin))
    return ORC_E_INVALID;
  if (cfg->repr == REPR_FP64) return run_abs<double>(*cfg, n, sp, xin, vin, Ein, nsteps, out);
  if (cfg->repr == REPR_FP32_ABS) return run_abs<float>(*cfg, n, sp, xin, vin, Ein, nsteps, out);
  return run_cell(*cfg, n, sp, xin, vin, Ein, nsteps, out);
}

// Pieces of the step, exposed so that tests can pin them one by one.
void orc_weights_f64(const double f[3], double W[8]) { weights(f, W); }
void orc_weights_f32(const float f[3], float W[8]) { weights(f, W); }

void orc_gather_f64(int32_t nx, int32_t ny, int32_t nz, const double* Ex, const double* Ey,
                    const double* Ez, const int32_t i[3], const double f[3], double out[3]) {
  orc_config c{};
  c.nx = nx; c.ny = ny; c.nz = nz;
  const Mesh M = make_mesh(c);
  double W[8];
  weights(f, W);
  int64_t idx[8];
  corners(M, i, idx);
  const double* E[3] = {Ex, Ey, Ez};
  gather(E, idx, W, out);
}

void orc_fixed_contrib_f64(double chg, const double W[8], int64_t C[8]) { fixed_contrib(chg, W, C); }
void orc_fixed_contrib_f32(float chg, const float W[8], int64_t C[8]) { fixed_contrib(chg, W, C); }

}  // extern "C"

namespace {

// ---- field solve on the PIC mesh ------------------------------------------------
//
// The boundary value problem of §2.1, -div(eps grad phi) = rho in the box,
// phi = g on the Dirichlet faces, d phi / dn = 0 on the others (the
// zero-Neumann symmetry planes of §3.1.3 and the open faces of §5.2.2).
// Node-centred finite volumes on the PIC nodes: a node's control volume is
// its dual cell clipped to the box, so on a Neumann face the zero flux is
// natural; the flux through the dual face of the link p-q is
// eps_pq w (phi_p - phi_q) h, w = product of the two tangential half-width
// factors c = 1/2 at a boundary index, else 1; the charge in the control
// volume is rho_p h^3 with rho_p the deposited nodal density (which at a
// boundary node already counts only the inside part of the cloud). So
//   (A phi)_p = 1 / h^2 sum_links eps_pq w (phi_p - phi_q) = rho_p,
// symmetric positive definite once one face is Dirichlet.
//
// The object as an interface (eq. (2.2)-(2.5); the paper discretises it with
// immersed finite elements on the same Cartesian mesh): the object region
// (sphere interior, or below the terrain) has eps_in, the plasma eps. A level
// set psi (< 0 inside: |x - c| - R for the sphere, z - h(x, y) for the
// terrain) is evaluated at the nodes; a link whose ends have psi of the same
// sign has that side's eps; a link that crosses has the inside fraction f from
// linear interpolation of psi (crossing at t = psi_a / (psi_a - psi_b) from
// the lower-index end a) and the series (harmonic) permittivity
// 1 / (f / eps_in + (1 - f) / eps), exact for a layered medium. The flux-jump
// source q(X) of eq. (2.5) is the collected surface charge, which enters the
// right-hand side as charge at the surface points of its tally bins (see
// orc_surface_rho). With no object, eps_pq = eps everywhere. Solved by
// preconditioned conjugate gradients (the PCG of §2.4) from the initial guess
// in phi, until ||r||_2 <= tol ||b||_2 (b: rho plus the Dirichlet terms) or
// max_iter iterations. The paper leaves the preconditioner open; two are
// here: Jacobi (z = r / diag A), and one geometric multigrid V-cycle (below).
// E = -grad phi at the nodes: central differences inside; on a Neumann face
// the normal component is 0; on a Dirichlet face the second-order one-sided
// difference.

// The object in the field problem (fine-mesh cell units, origin at node 0).
struct FieldObject {
  int kind;          // 1 sphere, 2 crater terrain
  double c[3], r;    // sphere centre, radius; crater: axis (c[0], c[1])
  double z_flat, a2, zc, rc2;  // crater: flat ground, rim radius^2, bowl sphere centre, radius^2
  double eps_in;
};

// Level set at a point (fine cells): < 0 inside the object.
double object_psi(const FieldObject& o, double x, double y, double z) {
  if (o.kind == OBJ_SPHERE) {
    const double dx = x - o.c[0], dy = y - o.c[1], dz = z - o.c[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz) - o.r;
  }
  const double dx = x - o.c[0], dy = y - o.c[1];
  const double r2 = dx * dx + dy * dy;
  const double ground = r2 < o.a2 ? o.zc - std::sqrt(o.rc2 - r2) : o.z_flat;
  return z - ground;
}

bool field_object(const orc_field_object& in, FieldObject& o) {
  if (!(in.eps_in > 0) || !std::isfinite(in.eps_in)) return false;
  o = FieldObject{};
  o.kind = in.kind;
  o.eps_in = in.eps_in;
  for (int d = 0; d < 3; ++d) o.c[d] = in.center[d];
  if (in.kind == OBJ_SPHERE) {
    if (!(in.radius > 0)) return false;
    o.r = in.radius;
    return true;
  }
  if (in.kind == OBJ_CRATER) {
    if (!(in.depth > 0) || !(in.rim_radius > 0)) return false;
    const double a = in.rim_radius, dep = in.depth;
    const double Rc = (a * a + dep * dep) / (2.0 * dep);
    o.z_flat = in.z_flat;
    o.a2 = a * a;
    o.zc = in.z_flat - dep + Rc;
    o.rc2 = Rc * Rc;
    return true;
  }
  return false;
}

// Series permittivity of a link whose lower-index end has psi a, the other b.
double link_eps(double a, double b, double ein, double eout) {
  const bool ia = a < 0.0, ib = b < 0.0;
  if (ia == ib) return ia ? ein : eout;
  const double t = a / (a - b);
  const double f = ia ? t : 1.0 - t;
  return (ein * eout) / (f * eout + (1.0 - f) * ein);
}

struct FieldGrid {
  int32_t n[3];
  int64_t sx, sy, nodes;
  double h, eps;
  int32_t mask;
  double g[6];
  double scale = 1.0;               // fine cells per cell of this grid
  const FieldObject* obj = nullptr;  // null: uniform eps
  // immersed finite elements (level 0 only): link coefficients c_pq of the
  // assembled operator, kIfeLinks per node (null: finite volumes)
  const std::vector<double>* ife = nullptr;
  double psi(int i, int j, int k) const {
    return object_psi(*obj, scale * i, scale * j, scale * k);
  }
  // coefficient of the link (i, j, k) - (i2, j2, k2) with tangential weight w
  double coef(int i, int j, int k, int i2, int j2, int k2, double w) const {
    if (!obj) return eps / (h * h) * w;
    const bool lower = id(i, j, k) < id(i2, j2, k2);
    const double a = lower ? psi(i, j, k) : psi(i2, j2, k2);
    const double b = lower ? psi(i2, j2, k2) : psi(i, j, k);
    return link_eps(a, b, obj->eps_in, eps) * w / (h * h);
  }
  bool dir(int i, int j, int k) const {
    return ((mask & 1) && i == 0) || ((mask & 2) && i == n[0]) || ((mask & 4) && j == 0) ||
           ((mask & 8) && j == n[1]) || ((mask & 16) && k == 0) || ((mask & 32) && k == n[2]);
  }
  // Dirichlet value of a node (the first Dirichlet face it lies on, faces in order)
  double gval(int i, int j, int k) const {
    if ((mask & 1) && i == 0) return g[0];
    if ((mask & 2) && i == n[0]) return g[1];
    if ((mask & 4) && j == 0) return g[2];
    if ((mask & 8) && j == n[1]) return g[3];
    if ((mask & 16) && k == 0) return g[4];
    return g[5];
  }
  double c(int d, int i) const { return (i == 0 || i == n[d]) ? 0.5 : 1.0; }
  int64_t id(int i, int j, int k) const { return i + sx * j + sy * k; }
};

// Visits the links of node (i, j, k): f(q, c) for each neighbour q in the box,
// c the link's coefficient in A (eps_pq w / h^2).
// Neighbours of a node in the five-tetrahedra mesh: the 6 axis neighbours,
// then the 12 face diagonals (every edge of the mesh is one of these).
constexpr int kIfeLinks = 18;
constexpr int kIfeOff[kIfeLinks][3] = {
    {-1, 0, 0},  {1, 0, 0},  {0, -1, 0}, {0, 1, 0},  {0, 0, -1}, {0, 0, 1},
    {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 1, 0},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1},  {1, 0, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}, {0, 1, 1}};

template <class F>
void field_links(const FieldGrid& G, int i, int j, int k, F f) {
  const int64_t p = G.id(i, j, k);
  if (G.ife) {
    for (int l = 0; l < kIfeLinks; ++l) {
      const int a = i + kIfeOff[l][0], b = j + kIfeOff[l][1], c = k + kIfeOff[l][2];
      if (a < 0 || b < 0 || c < 0 || a > G.n[0] || b > G.n[1] || c > G.n[2]) continue;
      const double cl = (*G.ife)[p * kIfeLinks + l];
      if (cl != 0.0) f(G.id(a, b, c), cl);
    }
    return;
  }
  const double wx = G.c(1, j) * G.c(2, k), wy = G.c(0, i) * G.c(2, k), wz = G.c(0, i) * G.c(1, j);
  if (i > 0) f(p - 1, G.coef(i, j, k, i - 1, j, k, wx));
  if (i < G.n[0]) f(p + 1, G.coef(i, j, k, i + 1, j, k, wx));
  if (j > 0) f(p - G.sx, G.coef(i, j, k, i, j - 1, k, wy));
  if (j < G.n[1]) f(p + G.sx, G.coef(i, j, k, i, j + 1, k, wy));
  if (k > 0) f(p - G.sy, G.coef(i, j, k, i, j, k - 1, wz));
  if (k < G.n[2]) f(p + G.sy, G.coef(i, j, k, i, j, k + 1, wz));
}

FieldGrid field_grid(int32_t nx, int32_t ny, int32_t nz, double h, double eps, int32_t mask,
                     const double g[6]);

// ---- immersed finite elements ------------------------------------------------
//
// The paper's discretisation of the interface (§2.3; §3.1.1: each cubic PIC
// cell is cut into five tetrahedra, and the IFE mesh is the PIC mesh). Away
// from the interface the IFE space is the standard linear finite element
// space on the tetrahedra; in a tetrahedron that the interface cuts, the basis
// functions are linear on each side, continuous across the interface (eq.
// (2.4)) and have a continuous flux eps d phi / dn across it (eq. (2.5) with
// q = 0: the charge on the surface enters the right-hand side). The paper
// gives the construction by reference only; this oracle takes:
//   * tetrahedra: cube (i, j, k) of parity p = (i + j + k) mod 2 has the
//     central tetrahedron on its four corners (a, b, c) with a + b + c = p
//     mod 2 and one corner tetrahedron per other corner (that corner and its
//     three axis neighbours), so that the face diagonals of neighbouring cubes
//     coincide;
//   * the interface in a tetrahedron: the zero set of the linear interpolant
//     psi_h of the level set's values at its vertices (a plane); T- = {psi_h
//     < 0} lies in the object (eps_in), T+ (psi_h >= 0) in the plasma (eps); a
//     tetrahedron is cut when its vertices have psi < 0 and psi >= 0;
//   * in a cut tetrahedron the basis function with vertex values v is
//     phi- = sum_j c_j lambda_j (lambda: barycentric coordinates) on T- and
//     phi+ = phi- + t psi_h on T+ (so phi+ = phi- on the interface), with t
//     such that eps_in grad phi- . g = eps grad phi+ . g, g = grad psi_h:
//     t = kappa (a . g), a = grad phi-, kappa = (eps_in - eps) / (eps |g|^2).
//     The vertex values are v = c + d t, d_i = psi_i at the vertices outside
//     and 0 inside; with w_j = grad lambda_j . g this is v = (I + kappa d w^T) c,
//     so c = v - kappa d (w . v) / (1 + kappa w . d);
//   * element matrix K_ij = eps_in |T-| a_i . a_j + eps |T+| b_i . b_j,
//     b = a + t g, computed for i <= j and mirrored;
//   * the operator is the assembled matrix over h^3 (the right-hand side is
//     the nodal charge density, the deposit's charge per node over h^3, as
//     for the finite volumes), applied in link form
//     (A phi)_p = sum_q c_pq (phi_p - phi_q), c_pq = -A_pq, over the 18
//     neighbours of the five-tetrahedra mesh (its rows sum to zero: the
//     constant function is in every element's space).

// Gradients of the barycentric coordinates of a tetrahedron and its volume.
void tet_gradients(const double X[4][3], double G[4][3], double* vol) {
  double e[3][3];
  for (int r = 0; r < 3; ++r)
    for (int d = 0; d < 3; ++d) e[r][d] = X[r + 1][d] - X[0][d];
  const auto cross = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  double c23[3], c31[3], c12[3];
  cross(e[1], e[2], c23);
  cross(e[2], e[0], c31);
  cross(e[0], e[1], c12);
  const double det = e[0][0] * c23[0] + e[0][1] * c23[1] + e[0][2] * c23[2];
  for (int d = 0; d < 3; ++d) {
    G[1][d] = c23[d] / det;
    G[2][d] = c31[d] / det;
    G[3][d] = c12[d] / det;
    G[0][d] = -(G[1][d] + G[2][d] + G[3][d]);
  }
  *vol = std::fabs(det) / 6.0;
}

double tet_volume(const double* A, const double* B, const double* C, const double* D) {
  double e[3][3];
  for (int d = 0; d < 3; ++d) {
    e[0][d] = B[d] - A[d];
    e[1][d] = C[d] - A[d];
    e[2][d] = D[d] - A[d];
  }
  const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                     e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                     e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
  return std::fabs(det) / 6.0;
}

// Volume of {psi_h < 0} in the tetrahedron (vertex values psi).
double tet_inside_volume(const double X[4][3], const double psi[4], double vol) {
  int neg[4], pos[4], nn = 0, np = 0;
  for (int i = 0; i < 4; ++i) {
    if (psi[i] < 0.0) neg[nn++] = i;
    else pos[np++] = i;
  }
  if (np == 0) return vol;
  if (nn == 0) return 0.0;
  // crossing point on the edge from vertex a to vertex b
  const auto at = [&](int a, int b, double* P) {
    const double t = psi[a] / (psi[a] - psi[b]);
    for (int d = 0; d < 3; ++d) P[d] = X[a][d] + t * (X[b][d] - X[a][d]);
  };
  if (nn == 1 || np == 1) {  // a small tetrahedron at the lone vertex
    const int lone = nn == 1 ? neg[0] : pos[0];
    const int* other = nn == 1 ? pos : neg;
    double P[3][3];
    for (int r = 0; r < 3; ++r) at(lone, other[r], P[r]);
    const double small = tet_volume(X[lone], P[0], P[1], P[2]);
    return nn == 1 ? small : vol - small;
  }
  // two and two: the inside part is a prism with ends (a, Pac, Pad) and
  // (b, Pbc, Pbd) and lateral edges a-b, Pac-Pbc, Pad-Pbd; three tetrahedra
  const int a = neg[0], b = neg[1], c = pos[0], d = pos[1];
  double Pac[3], Pad[3], Pbc[3], Pbd[3];
  at(a, c, Pac);
  at(a, d, Pad);
  at(b, c, Pbc);
  at(b, d, Pbd);
  return tet_volume(X[a], Pac, Pad, X[b]) + tet_volume(Pac, Pad, X[b], Pbd) +
         tet_volume(Pac, X[b], Pbc, Pbd);
}

// The IFE basis of one tetrahedron: grad phi- of basis function i (a[i]),
// its interface coefficient t[i], the vertex coefficients c[i][j] of phi-,
// g = grad psi_h and the volume of T-. For an uncut tetrahedron a = grad
// lambda, t = 0, c = identity, and the inside volume is all or nothing.
struct IfeBasis {
  double a[4][3], t[4], c[4][4], g[3], vol, vin;
  bool cut;
};

IfeBasis ife_basis(const double X[4][3], const double psi[4], double ein, double eout) {
  IfeBasis B{};
  double G[4][3];
  tet_gradients(X, G, &B.vol);
  bool any_in = false, any_out = false;
  for (int i = 0; i < 4; ++i) (psi[i] < 0.0 ? any_in : any_out) = true;
  B.cut = any_in && any_out;
  B.vin = tet_inside_volume(X, psi, B.vol);
  for (int d = 0; d < 3; ++d) {
    B.g[d] = 0.0;
    for (int i = 0; i < 4; ++i) B.g[d] += psi[i] * G[i][d];
  }
  double kappa = 0.0, w[4] = {0, 0, 0, 0}, dv[4] = {0, 0, 0, 0}, wd = 0.0;
  if (B.cut) {
    const double g2 = B.g[0] * B.g[0] + B.g[1] * B.g[1] + B.g[2] * B.g[2];
    kappa = (ein - eout) / (eout * g2);
    for (int j = 0; j < 4; ++j) {
      w[j] = G[j][0] * B.g[0] + G[j][1] * B.g[1] + G[j][2] * B.g[2];
      dv[j] = psi[j] < 0.0 ? 0.0 : psi[j];
      wd += w[j] * dv[j];
    }
  }
  const double den = 1.0 + kappa * wd;
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) B.c[i][j] = (i == j ? 1.0 : 0.0) - kappa * dv[j] * w[i] / den;
    for (int d = 0; d < 3; ++d) {
      B.a[i][d] = 0.0;
      for (int j = 0; j < 4; ++j) B.a[i][d] += B.c[i][j] * G[j][d];
    }
    B.t[i] = kappa * (B.a[i][0] * B.g[0] + B.a[i][1] * B.g[1] + B.a[i][2] * B.g[2]);
  }
  return B;
}

// Element matrix of the IFE basis (uncut: eps of its side times the linear
// finite element matrix).
void ife_element(const double X[4][3], const double psi[4], double ein, double eout,
                 double K[4][4]) {
  const IfeBasis B = ife_basis(X, psi, ein, eout);
  const double vout = B.vol - B.vin;
  for (int i = 0; i < 4; ++i)
    for (int j = i; j < 4; ++j) {
      double aa = 0.0, bb = 0.0;
      for (int d = 0; d < 3; ++d) {
        aa += B.a[i][d] * B.a[j][d];
        bb += (B.a[i][d] + B.t[i] * B.g[d]) * (B.a[j][d] + B.t[j] * B.g[d]);
      }
      K[i][j] = ein * B.vin * aa + eout * vout * bb;
      K[j][i] = K[i][j];
    }
}

// The five tetrahedra of cube (i, j, k) as corner offsets (a, b, c).
void cube_tets(int i, int j, int k, int T[5][4][3]) {
  const int p = (i + j + k) & 1;
  int even[4][3], odd[4][3], ne = 0, no = 0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int* dst = ((a + b + c) & 1) == p ? even[ne++] : odd[no++];
        dst[0] = a;
        dst[1] = b;
        dst[2] = c;
      }
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) T[0][v][d] = even[v][d];
  for (int o = 0; o < 4; ++o) {  // the odd corner and its three axis neighbours
    for (int d = 0; d < 3; ++d) T[1 + o][0][d] = odd[o][d];
    int m = 1;
    for (int e = 0; e < 4; ++e) {
      const int dist = std::abs(even[e][0] - odd[o][0]) + std::abs(even[e][1] - odd[o][1]) +
                       std::abs(even[e][2] - odd[o][2]);
      if (dist != 1) continue;
      for (int d = 0; d < 3; ++d) T[1 + o][m][d] = even[e][d];
      ++m;
    }
  }
}

int ife_link(int di, int dj, int dk) {
  for (int l = 0; l < kIfeLinks; ++l)
    if (kIfeOff[l][0] == di && kIfeOff[l][1] == dj && kIfeOff[l][2] == dk) return l;
  return -1;
}

// Assembles the link coefficients of the IFE operator on grid G (the object
// in G.obj with eps_in inside, G.eps outside; no object: uniform G.eps).
void ife_assemble(const FieldGrid& G, std::vector<double>& c) {
  c.assign(G.nodes * kIfeLinks, 0.0);
  const double ein = G.obj ? G.obj->eps_in : G.eps;
  const double h3 = G.h * G.h * G.h;
  for (int k = 0; k < G.n[2]; ++k)
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        int T[5][4][3];
        cube_tets(i, j, k, T);
        for (int t = 0; t < 5; ++t) {
          double X[4][3], psi[4];
          int idx[4][3];
          for (int v = 0; v < 4; ++v) {
            idx[v][0] = i + T[t][v][0];
            idx[v][1] = j + T[t][v][1];
            idx[v][2] = k + T[t][v][2];
            for (int d = 0; d < 3; ++d) X[v][d] = G.h * idx[v][d];
            psi[v] = G.obj ? G.psi(idx[v][0], idx[v][1], idx[v][2]) : 1.0;
          }
          double K[4][4];
          ife_element(X, psi, ein, G.eps, K);
          for (int r = 0; r < 4; ++r)
            for (int q = 0; q < 4; ++q) {
              if (r == q) continue;
              const int l = ife_link(idx[q][0] - idx[r][0], idx[q][1] - idx[r][1],
                                     idx[q][2] - idx[r][2]);
              c[G.id(idx[r][0], idx[r][1], idx[r][2]) * kIfeLinks + l] -= K[r][q] / h3;
            }
        }
      }
}

// ---- multigrid V-cycle preconditioner ----------------------------------------
//
// Textbook geometric multigrid on nested node grids. Level l + 1 takes every
// other node of level l (all cell counts even), spacing 2h, the same faces and
// the same finite-volume operator (rediscretised, homogeneous Dirichlet values:
// the V-cycle acts on corrections). Grids are coarsened while a level has more
// than kMgCoarseNodes nodes, at most kMgLevels levels; the coarsest level is
// solved exactly (Cholesky). A grid that cannot reach kMgCoarseNodes so, or is
// already that small, keeps the Jacobi preconditioner.
//   prolongation P: trilinear interpolation of the coarse corrections;
//   restriction R = P^T / 8 (the coarse density of the fine residual charge:
//     a residual is a density, charge over h^3, and h_c^3 = 8 h^3);
//   smoother: kMgSweeps damped-Jacobi sweeps e += w (b - A e) / diag A before
//     the coarse correction and as many after it.
// With the same smoother before and after, R proportional to P^T and an exact
// (symmetric) coarsest solve, one V-cycle from a zero guess is a symmetric
// positive definite linear map of the residual (w * eigenvalues of
// diag^-1 A < 2), so CG stays CG.

constexpr int kMgLevels = 8;
constexpr int64_t kMgCoarseNodes = 1024;
constexpr int kMgSweeps = 2;
constexpr double kMgOmega = 6.0 / 7.0;

struct Multigrid {
  std::vector<FieldGrid> lv;        // level 0: the PIC mesh
  std::vector<int64_t> unk;         // coarsest level: node of each unknown
  std::vector<double> chol;         // coarsest level: Cholesky factor (row-major, lower)
};

bool dirichlet_node(const FieldGrid& G, int64_t q) {
  const int i = (int)(q % G.sx), j = (int)((q / G.sx) % (G.n[1] + 1)), k = (int)(q / G.sy);
  return G.dir(i, j, k);
}

// Levels and the coarsest factor; false when the grid does not coarsen so.
bool mg_setup(const FieldGrid& G0, Multigrid& M) {
  M.lv.assign(1, G0);
  while (M.lv.back().nodes > kMgCoarseNodes && (int)M.lv.size() < kMgLevels) {
    const FieldGrid& f = M.lv.back();
    if (f.n[0] % 2 || f.n[1] % 2 || f.n[2] % 2) break;
    FieldGrid c = field_grid(f.n[0] / 2, f.n[1] / 2, f.n[2] / 2, 2.0 * f.h, f.eps, f.mask, f.g);
    c.scale = 2.0 * f.scale;
    c.obj = f.obj;
    M.lv.push_back(c);
  }
  if (M.lv.size() < 2 || M.lv.back().nodes > kMgCoarseNodes) return false;
  const FieldGrid& C = M.lv.back();
  std::vector<int64_t> pos(C.nodes, -1);
  for (int64_t q = 0; q < C.nodes; ++q)
    if (!dirichlet_node(C, q)) {
      pos[q] = (int64_t)M.unk.size();
      M.unk.push_back(q);
    }
  const int64_t m = (int64_t)M.unk.size();
  std::vector<double> A(m * m, 0.0);
  for (int64_t u = 0; u < m; ++u) {
    const int64_t q0 = M.unk[u];
    const int i = (int)(q0 % C.sx), j = (int)((q0 / C.sx) % (C.n[1] + 1)), k = (int)(q0 / C.sy);
    field_links(C, i, j, k, [&](int64_t q, double c) {
      A[u * m + u] += c;
      if (pos[q] >= 0) A[u * m + pos[q]] -= c;
    });
  }
  // A = L L^T
  M.chol.assign(m * m, 0.0);
  for (int64_t r = 0; r < m; ++r)
    for (int64_t c = 0; c <= r; ++c) {
      double v = A[r * m + c];
      for (int64_t t = 0; t < c; ++t) v -= M.chol[r * m + t] * M.chol[c * m + t];
      M.chol[r * m + c] = r == c ? std::sqrt(v) : v / M.chol[c * m + c];
    }
  return true;
}

// (A e)_p at an unknown node of a level, e = 0 on the Dirichlet nodes.
double mg_apply(const FieldGrid& G, const std::vector<double>& e, int i, int j, int k) {
  const int64_t p = G.id(i, j, k);
  double a = 0.0;
  field_links(G, i, j, k, [&](int64_t q, double c) { a += c * (e[p] - e[q]); });
  return a;
}

double mg_diag(const FieldGrid& G, int i, int j, int k) {
  double d = 0.0;
  field_links(G, i, j, k, [&](int64_t, double c) { d += c; });
  return d;
}

void mg_jacobi(const FieldGrid& G, const std::vector<double>& b, std::vector<double>& e) {
  std::vector<double> out(G.nodes, 0.0);
  for (int k = 0; k <= G.n[2]; ++k)
    for (int j = 0; j <= G.n[1]; ++j)
      for (int i = 0; i <= G.n[0]; ++i) {
        if (G.dir(i, j, k)) continue;
        const int64_t p = G.id(i, j, k);
        out[p] = e[p] + kMgOmega * (b[p] - mg_apply(G, e, i, j, k)) / mg_diag(G, i, j, k);
      }
  e.swap(out);
}

// coarse index and weight of the 1 or 2 coarse nodes a fine index interpolates from
int mg_parents(int a, int c[2], double w[2]) {
  if (a % 2 == 0) {
    c[0] = a / 2; w[0] = 1.0;
    return 1;
  }
  c[0] = (a - 1) / 2; c[1] = (a + 1) / 2; w[0] = w[1] = 0.5;
  return 2;
}

// Visits the coarse parents of fine node (i, j, k): f(coarse node, weight).
template <class F>
void mg_each_parent(const FieldGrid& C, int i, int j, int k, F f) {
  int ci[2], cj[2], ck[2];
  double wi[2], wj[2], wk[2];
  const int ni = mg_parents(i, ci, wi), nj = mg_parents(j, cj, wj), nk = mg_parents(k, ck, wk);
  for (int c = 0; c < nk; ++c)
    for (int b = 0; b < nj; ++b)
      for (int a = 0; a < ni; ++a) f(C.id(ci[a], cj[b], ck[c]), wi[a] * wj[b] * wk[c]);
}

void mg_vcycle(const Multigrid& M, size_t l, const std::vector<double>& b, std::vector<double>& e) {
  const FieldGrid& G = M.lv[l];
  e.assign(G.nodes, 0.0);
  if (l + 1 == M.lv.size()) {  // exact solve: L y = b, L^T e = y
    const int64_t m = (int64_t)M.unk.size();
    std::vector<double> y(m);
    for (int64_t r = 0; r < m; ++r) {
      double v = b[M.unk[r]];
      for (int64_t t = 0; t < r; ++t) v -= M.chol[r * m + t] * y[t];
      y[r] = v / M.chol[r * m + r];
    }
    for (int64_t r = m - 1; r >= 0; --r) {
      double v = y[r];
      for (int64_t t = r + 1; t < m; ++t) v -= M.chol[t * m + r] * e[M.unk[t]];
      e[M.unk[r]] = v / M.chol[r * m + r];
    }
    return;
  }
  for (int t = 0; t < kMgSweeps; ++t) mg_jacobi(G, b, e);
  const FieldGrid& C = M.lv[l + 1];
  std::vector<double> bc(C.nodes, 0.0), ec;
  for (int k = 0; k <= G.n[2]; ++k)  // bc = P^T (b - A e) / 8
    for (int j = 0; j <= G.n[1]; ++j)
      for (int i = 0; i <= G.n[0]; ++i) {
        if (G.dir(i, j, k)) continue;
        const double res = b[G.id(i, j, k)] - mg_apply(G, e, i, j, k);
        mg_each_parent(C, i, j, k, [&](int64_t Q, double w) { bc[Q] += w * res / 8.0; });
      }
  for (int64_t Q = 0; Q < C.nodes; ++Q)
    if (dirichlet_node(C, Q)) bc[Q] = 0.0;
  mg_vcycle(M, l + 1, bc, ec);
  for (int k = 0; k <= G.n[2]; ++k)  // e += P ec
    for (int j = 0; j <= G.n[1]; ++j)
      for (int i = 0; i <= G.n[0]; ++i) {
        if (G.dir(i, j, k)) continue;
        double v = 0.0;
        mg_each_parent(C, i, j, k, [&](int64_t Q, double w) { v += w * ec[Q]; });
        e[G.id(i, j, k)] += v;
      }
  for (int t = 0; t < kMgSweeps; ++t) mg_jacobi(G, b, e);
}

int field_solve(const FieldGrid& G, const double* rho, double* x, double tol, int32_t max_iter,
                int32_t precond, int32_t* iters, double* relres, int32_t* levels) {
  Multigrid M;
  const bool mg = precond == 0 && mg_setup(G, M);
  if (levels) *levels = mg ? (int32_t)M.lv.size() : 0;
  std::vector<double> rv, zv;
  // z = B r
  auto precondition = [&](const std::vector<double>& r, std::vector<double>& z,
                          const std::vector<double>& D, const std::vector<char>& unk) {
    if (mg) {
      mg_vcycle(M, 0, r, zv);
      for (int64_t q = 0; q < G.nodes; ++q) z[q] = unk[q] ? zv[q] : 0.0;
    } else {
      for (int64_t q = 0; q < G.nodes; ++q) z[q] = unk[q] ? r[q] / D[q] : 0.0;
    }
  };
  const int64_t N = G.nodes;
  std::vector<double> r(N, 0.0), z(N, 0.0), p(N, 0.0), Ap(N, 0.0), D(N, 0.0);
  std::vector<char> unk(N, 0);
  double bb = 0.0, rz = 0.0, rr = 0.0;
  for (int k = 0; k <= G.n[2]; ++k)
    for (int j = 0; j <= G.n[1]; ++j)
      for (int i = 0; i <= G.n[0]; ++i) {
        const int64_t q0 = G.id(i, j, k);
        if (G.dir(i, j, k)) {
          x[q0] = G.gval(i, j, k);
          continue;
        }
        unk[q0] = 1;
      }
  for (int k = 0; k <= G.n[2]; ++k)
    for (int j = 0; j <= G.n[1]; ++j)
      for (int i = 0; i <= G.n[0]; ++i) {
        const int64_t q0 = G.id(i, j, k);
        if (!unk[q0]) continue;
        double ax = 0.0, b = rho[q0], d = 0.0;
        field_links(G, i, j, k, [&](int64_t q, double c) {
          ax += c * (x[q0] - x[q]);
          d += c;
          if (!unk[q]) b += c * x[q];
        });
        r[q0] = rho[q0] - ax;
        D[q0] = d;
        bb += b * b;
        rr += r[q0] * r[q0];
      }
  const double bn = std::sqrt(bb);
  int32_t it = 0;
  if (!(std::sqrt(rr) <= tol * bn)) {
    precondition(r, z, D, unk);
    for (int64_t q = 0; q < N; ++q) {
      p[q] = z[q];
      rz += r[q] * z[q];
    }
    for (it = 1; it <= max_iter; ++it) {
      double pap = 0.0;
      for (int k = 0; k <= G.n[2]; ++k)
        for (int j = 0; j <= G.n[1]; ++j)
          for (int i = 0; i <= G.n[0]; ++i) {
            const int64_t q0 = G.id(i, j, k);
            if (!unk[q0]) continue;
            double a = 0.0;
            field_links(G, i, j, k, [&](int64_t q, double c) { a += c * (p[q0] - p[q]); });
            Ap[q0] = a;
            pap += p[q0] * Ap[q0];
          }
      const double alpha = rz / pap;
      rr = 0.0;
      for (int64_t q = 0; q < N; ++q) {
        if (!unk[q]) continue;
        x[q] = x[q] + alpha * p[q];
        r[q] = r[q] - alpha * Ap[q];
        rr += r[q] * r[q];
      }
      if (std::sqrt(rr) <= tol * bn) break;
      precondition(r, z, D, unk);
      double rz1 = 0.0;
      for (int64_t q = 0; q < N; ++q) rz1 += r[q] * z[q];
      const double beta = rz1 / rz;
      rz = rz1;
      for (int64_t q = 0; q < N; ++q)
        if (unk[q]) p[q] = z[q] + beta * p[q];
    }
    if (it > max_iter) it = max_iter;
  }
  if (iters) *iters = it;
  if (relres) *relres = bn > 0.0 ? std::sqrt(rr) / bn : 0.0;
  return ORC_OK;
}

// E = -grad phi at the nodes.
void field_E(const FieldGrid& G, const double* phi, double* E[3]) {
  for (int k = 0; k <= G.n[2]; ++k)
    for (int j = 0; j <= G.n[1]; ++j)
      for (int i = 0; i <= G.n[0]; ++i) {
        const int idx[3] = {i, j, k};
        const int64_t q0 = G.id(i, j, k);
        const int64_t st[3] = {1, G.sx, G.sy};
        for (int d = 0; d < 3; ++d) {
          const int a = idx[d], n = G.n[d];
          double e;
          if (a > 0 && a < n) {
            e = -(phi[q0 + st[d]] - phi[q0 - st[d]]) / (2.0 * G.h);
          } else if (!((G.mask >> (2 * d + (a == 0 ? 0 : 1))) & 1)) {
            e = 0.0;  // zero-Neumann face
          } else if (n == 1) {
            e = a == 0 ? -(phi[q0 + st[d]] - phi[q0]) / G.h : -(phi[q0] - phi[q0 - st[d]]) / G.h;
          } else if (a == 0) {
            e = -(-3.0 * phi[q0] + 4.0 * phi[q0 + st[d]] - phi[q0 + 2 * st[d]]) / (2.0 * G.h);
          } else {
            e = -(3.0 * phi[q0] - 4.0 * phi[q0 - st[d]] + phi[q0 - 2 * st[d]]) / (2.0 * G.h);
          }
          E[d][q0] = e;
        }
      }
}

FieldGrid field_grid(int32_t nx, int32_t ny, int32_t nz, double h, double eps, int32_t mask,
                     const double g[6]) {
  FieldGrid G{};
  G.n[0] = nx; G.n[1] = ny; G.n[2] = nz;
  G.sx = nx + 1;
  G.sy = (int64_t)(nx + 1) * (ny + 1);
  G.nodes = G.sy * (nz + 1);
  G.h = h;
  G.eps = eps;
  G.mask = mask;
  for (int f = 0; f < 6; ++f) G.g[f] = g ? g[f] : 0.0;
  return G;
}

}  // namespace

extern "C" {

// Pieces of the boundary source, exposed for the pins.
uint64_t orc_splitmix_draw(uint64_t key, uint64_t d) { return sm_mix(key + (d + 1) * kGolden); }
double orc_inj_uniform(uint64_t seed, int32_t step, int32_t s, int32_t f, int64_t cell, int64_t j,
                       uint64_t d) {
  return inj_uniform(inj_key(seed, step, s, f, cell, j), d);
}
double orc_ln(double x) { return ln_series(x); }
void orc_normals3(uint64_t key, double z[3]) {
  uint64_t d = 0;
  normals3(key, &d, z);
}

// Field solve (see above). phi: in the initial guess, out the solution (nodes
// values). precond: 0 multigrid V-cycle where the grid coarsens (else Jacobi),
// 1 Jacobi; *levels gets the multigrid level count used (0: Jacobi). Returns
// 0, or -1 for invalid arguments (no Dirichlet face, h or eps not > 0, tol not
// > 0, max_iter < 0, precond not 0 or 1).
// obj (nullable, or kind 0): the object as an interface with permittivity
// eps_in inside (see above).
// op: 0 node-centred finite volumes, 1 immersed finite elements (the
// multigrid preconditioner then smooths its finest level with the IFE
// operator and corrects with the finite-volume operators of the coarser
// levels).
int orc_field_solve(int32_t nx, int32_t ny, int32_t nz, double h, double eps, int32_t dirichlet,
                    const double* g, const double* rho, double* phi, double tol, int32_t max_iter,
                    int32_t precond, const orc_field_object* obj, int32_t op, int32_t* iters,
                    double* relres, int32_t* levels) {
  if (nx < 1 || ny < 1 || nz < 1 || !(h > 0) || !(eps > 0) || !(tol > 0) || max_iter < 0 ||
      (dirichlet & 63) == 0 || (dirichlet & ~63) || !rho || !phi || precond < 0 || precond > 1 ||
      op < 0 || op > 1)
    return ORC_E_INVALID;
  FieldObject fo{};
  FieldGrid G = field_grid(nx, ny, nz, h, eps, dirichlet, g);
  if (obj && obj->kind != 0) {
    if (!field_object(*obj, fo)) return ORC_E_INVALID;
    G.obj = &fo;
  }
  std::vector<double> links;
  if (op == 1) {
    ife_assemble(G, links);
    G.ife = &links;
  }
  return field_solve(G, rho, phi, tol, max_iter, precond, iters, relres, levels);
}

// One multigrid V-cycle z = B r on the grid (homogeneous Dirichlet faces in
// the mask), for the pins of the preconditioner. Returns the level count, or
// 0 when the grid does not coarsen (z untouched), -1 for invalid arguments.
int orc_field_vcycle(int32_t nx, int32_t ny, int32_t nz, double h, double eps, int32_t dirichlet,
                     const orc_field_object* obj, int32_t op, const double* r, double* z) {
  if (nx < 1 || ny < 1 || nz < 1 || !(h > 0) || !(eps > 0) || (dirichlet & 63) == 0 ||
      (dirichlet & ~63) || !r || !z || op < 0 || op > 1)
    return ORC_E_INVALID;
  FieldObject fo{};
  FieldGrid G = field_grid(nx, ny, nz, h, eps, dirichlet, nullptr);
  if (obj && obj->kind != 0) {
    if (!field_object(*obj, fo)) return ORC_E_INVALID;
    G.obj = &fo;
  }
  std::vector<double> links;
  if (op == 1) {
    ife_assemble(G, links);
    G.ife = &links;
  }
  Multigrid M;
  if (!mg_setup(G, M)) return 0;
  std::vector<double> b(r, r + G.nodes), e;
  for (int64_t q = 0; q < G.nodes; ++q)
    if (dirichlet_node(G, q)) b[q] = 0.0;
  mg_vcycle(M, 0, b, e);
  for (int64_t q = 0; q < G.nodes; ++q) z[q] = e[q];
  return (int)M.lv.size();
}

void orc_field_E(int32_t nx, int32_t ny, int32_t nz, double h, int32_t dirichlet, const double* phi,
                 double* Ex, double* Ey, double* Ez) {
  double* E[3] = {Ex, Ey, Ez};
  field_E(field_grid(nx, ny, nz, h, 1.0, dirichlet, nullptr), phi, E);
}

// Pieces of the immersed finite elements, for the pins. X: the 4 vertices
// (x, y, z each), psi: the level set there.
// out (38 values): a[4][3] (grad phi- of each basis function), t[4], c[4][4]
// (phi- = sum_j c[i][j] lambda_j), g[3] (grad psi_h), volume, inside volume,
// cut (1 or 0).
void orc_ife_basis(const double* X, const double* psi, double ein, double eout, double* out) {
  double Xv[4][3];
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) Xv[v][d] = X[3 * v + d];
  const IfeBasis B = ife_basis(Xv, psi, ein, eout);
  int o = 0;
  for (int i = 0; i < 4; ++i)
    for (int d = 0; d < 3; ++d) out[o++] = B.a[i][d];
  for (int i = 0; i < 4; ++i) out[o++] = B.t[i];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[o++] = B.c[i][j];
  for (int d = 0; d < 3; ++d) out[o++] = B.g[d];
  out[o++] = B.vol;
  out[o++] = B.vin;
  out[o++] = B.cut ? 1.0 : 0.0;
}

void orc_ife_element(const double* X, const double* psi, double ein, double eout, double* K) {
  double Xv[4][3], Kv[4][4];
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) Xv[v][d] = X[3 * v + d];
  ife_element(Xv, psi, ein, eout, Kv);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) K[4 * i + j] = Kv[i][j];
}

// The five tetrahedra of cube (i, j, k): T[t][v] = corner offsets (60 ints).
void orc_cube_tets(int32_t i, int32_t j, int32_t k, int32_t* out) {
  int T[5][4][3];
  cube_tets(i, j, k, T);
  for (int t = 0; t < 5; ++t)
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) out[12 * t + 3 * v + d] = T[t][v][d];
}

// The assembled IFE link coefficients c[node][18] (neighbour order of the
// oracle source) on a grid; obj nullable (uniform eps).
int orc_ife_links(int32_t nx, int32_t ny, int32_t nz, double h, double eps,
                  const orc_field_object* obj, double* c) {
  if (nx < 1 || ny < 1 || nz < 1 || !(h > 0) || !(eps > 0) || !c) return ORC_E_INVALID;
  FieldObject fo{};
  FieldGrid G = field_grid(nx, ny, nz, h, eps, 1, nullptr);
  if (obj && obj->kind != 0) {
    if (!field_object(*obj, fo)) return ORC_E_INVALID;
    G.obj = &fo;
  }
  std::vector<double> links;
  ife_assemble(G, links);
  std::memcpy(c, links.data(), sizeof(double) * links.size());
  return ORC_OK;
}

// Level set of the object at points (cell units), for the pins.
double orc_object_psi(const orc_field_object* obj, double x, double y, double z) {
  FieldObject fo{};
  if (!obj || !field_object(*obj, fo)) return 0.0;
  return object_psi(fo, x, y, z);
}

// The collected surface charge as a source of the field problem (the flux
// jump q(X) of eq. (2.5)): the charge of each tally bin, sum over species of
// (q_s w_s) count[bin][s] in FP64, is placed at the bin's surface point and
// deposited to the mesh nodes like a particle's charge (trilinear weights,
// int64 fixed point at 2^32 with the remainder rule of the deposit), added to
// rho_fixed (nodes). The surface point of a crater column (i, j) is the
// terrain above its centre, (i + 1/2, j + 1/2, ground height); of a sphere
// patch the sphere point in the direction of the patch centre (the centre of
// its (iu, iv) square on its cube face). A sphere without patches has one bin
// for the whole sphere and no surface point: returns -1 then, and for invalid
// arguments; 0 otherwise.
int orc_surface_rho(const orc_config* cfg, const int64_t* tally, int64_t* rho_fixed) {
  if (!cfg || !tally || !rho_fixed) return ORC_E_INVALID;
  if (cfg->obj_kind == OBJ_NONE) return ORC_OK;
  if (cfg->obj_kind == OBJ_SPHERE && cfg->sphere_patches < 1) return ORC_E_INVALID;
  const Mesh M = make_mesh(*cfg);
  const Geometry<double> G = make_geometry<double>(*cfg);
  const int ns = cfg->n_species;
  const int m = cfg->sphere_patches;
  const int64_t nbins =
      cfg->obj_kind == OBJ_CRATER ? (int64_t)cfg->nx * cfg->ny : 6 * (int64_t)m * m;
  for (int64_t b = 0; b < nbins; ++b) {
    double Q = 0.0;
    for (int s = 0; s < ns; ++s) Q += (cfg->q[s] * cfg->w[s]) * (double)tally[b * ns + s];
    if (Q == 0.0) continue;
    double g[3];
    if (cfg->obj_kind == OBJ_CRATER) {
      g[0] = (double)(b % cfg->nx) + 0.5;
      g[1] = (double)(b / cfg->nx) + 0.5;
      const double dx = g[0] - G.c[0], dy = g[1] - G.c[1];
      const double a = cfg->rim_radius / cfg->h;
      const double r2 = dx * dx + dy * dy;
      g[2] = r2 < a * a ? G.c[2] - std::sqrt(G.r2 - r2) : G.z_flat;
    } else {
      const int face = (int)(b / ((int64_t)m * m)), iv = (int)((b / m) % m), iu = (int)(b % m);
      const int ax = face / 2;
      const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
      double d[3];
      d[ax] = face % 2 ? 1.0 : -1.0;
      d[u] = -1.0 + (2.0 * iu + 1.0) / m;
      d[v] = -1.0 + (2.0 * iv + 1.0) / m;
      const double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double R = std::sqrt(G.r2);
      for (int k = 0; k < 3; ++k) g[k] = G.c[k] + R * (d[k] / len);
    }
    int32_t i[3];
    double f[3];
    for (int k = 0; k < 3; ++k) {
      double fl = std::floor(g[k]);
      if (fl < 0.0) fl = 0.0;
      if (fl > (double)(M.n[k] - 1)) fl = (double)(M.n[k] - 1);
      i[k] = (int32_t)fl;
      double o = g[k] - fl;
      o = o < 0.0 ? 0.0 : (o > 1.0 ? 1.0 : o);
      f[k] = o;
    }
    double W[8];
    weights(f, W);
    int64_t C[8], idx[8];
    fixed_contrib(Q, W, C);
    corners(M, i, idx);
    for (int n = 0; n < 8; ++n) rho_fixed[idx[n]] += C[n];
  }
  return ORC_OK;
}

// Photoemission pieces for the pins: the terrain of column (i, j) as the
// emission sees it: out = {n_x, n_y, n_z, ground, sunlight index, lit (1/0),
// mean count per step}. Returns -1 without photoemission.
int orc_photo_column(const orc_config* cfg, int64_t i, int64_t j, double out[7]) {
  if (!cfg || !out) return ORC_E_INVALID;
  const PhotoSetup P = photo_setup(*cfg);
  if (!P.on) return ORC_E_INVALID;
  double n[3], zg, I;
  bool lit;
  photo_column(P, i, j, n, &zg, &I, &lit);
  for (int d = 0; d < 3; ++d) out[d] = n[d];
  out[3] = zg;
  out[4] = I;
  out[5] = lit ? 1.0 : 0.0;
  out[6] = lit ? (P.rate * I) / n[2] : 0.0;
  return ORC_OK;
}

// Most photoelectrons one step can emit (each lit column: floor(mean) + 1).
int64_t orc_photo_max_per_step(const orc_config* cfg) {
  if (!cfg) return 0;
  const PhotoSetup P = photo_setup(*cfg);
  if (!P.on) return 0;
  int64_t t = 0;
  for (int64_t col = 0; col < (int64_t)cfg->nx * cfg->ny; ++col) {
    double n[3], zg, I;
    bool lit;
    photo_column(P, col % cfg->nx, col / cfg->nx, n, &zg, &I, &lit);
    if (lit) t += (int64_t)std::floor((P.rate * I) / n[2]) + 1;
  }
  return t;
}

// Object predicate at one point (physical units), in the arithmetic of `repr`.
// Returns the bin when the point is absorbed, else -1.
int32_t orc_object_hit(const orc_config* cfg, double x, double y, double z) {
  const Mesh M = make_mesh(*cfg);
  const double gd[3] = {(x - cfg->origin[0]) / cfg->h, (y - cfg->origin[1]) / cfg->h,
                        (z - cfg->origin[2]) / cfg->h};
  if (cfg->repr == REPR_FP64) {
    const Geometry<double> G = make_geometry<double>(*cfg);
    return object_hit_abs(G, M, gd);
  }
  const Geometry<float> G = make_geometry<float>(*cfg);
  if (cfg->repr == REPR_FP32_ABS) {
    const float g[3] = {(float)gd[0], (float)gd[1], (float)gd[2]};
    return object_hit_abs(G, M, g);
  }
  int32_t i[3];
  float o[3];
  for (int d = 0; d < 3; ++d) {
    i[d] = (int32_t)std::floor(gd[d]);
    o[d] = (float)(gd[d] - i[d]);
    if (o[d] == 1.0f) {
      o[d] = 0.0f;
      i[d] += 1;
    }
  }
  return object_hit_cell(G, M, i, o);
}

}  // extern "C"
