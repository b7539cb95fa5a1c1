/* Seeded synthetic inputs for the particle-mesh workloads.
 *
 * This module draws inputs only: initial particle positions and half-step
 * velocities, and node electric fields. It holds none of the PIC step's
 * arithmetic; both the GPU library's tests/benchmark and the CPU oracle take
 * their inputs from here.
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): the value for
 * (seed, stream, index, draw) is the SplitMix64 output function applied to a
 * key derived from (seed, stream, index) advanced by (draw + 1) golden-gamma
 * increments. Normals come from the Box-Muller transform on the host.
 *
 * Quantisation: positions are multiples of 2^-16 (exact in float for
 * coordinates below 256); velocities and node fields are rounded to float, so
 * FP64 and FP32 consumers start from identical values.
 */
#include <math.h>
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t sm_key(uint64_t seed, uint64_t stream, uint64_t index) {
  uint64_t k = sm_mix(seed + GAMMA);
  k = sm_mix((k ^ stream) + GAMMA);
  return sm_mix((k ^ index) + GAMMA);
}

static inline uint64_t sm_draw(uint64_t key, uint64_t draw) { return sm_mix(key + (draw + 1) * GAMMA); }

/* uniform in [0, 1) with 53 random bits */
static inline double u01(uint64_t key, uint64_t draw) {
  return (double)(sm_draw(key, draw) >> 11) * (1.0 / 9007199254740992.0);
}

/* uniform in (0, 1] */
static inline double u01_open0(uint64_t key, uint64_t draw) {
  return ((double)(sm_draw(key, draw) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

uint64_t synth_draw_u64(uint64_t seed, uint64_t stream, uint64_t index, uint64_t draw) {
  return sm_draw(sm_key(seed, stream, index), draw);
}

typedef struct {
  uint64_t seed;
  uint64_t stream;      /* species index */
  int32_t nx, ny, nz;   /* box [0,nx) x [0,ny) x [0,nz) in cell units */
  int32_t obj_kind;     /* 0 none, 1 sphere (excluded region), 2 crater terrain */
  double center[3];     /* sphere centre; crater axis (center[0], center[1]) */
  double radius;        /* sphere radius */
  double z_flat, rim_radius, depth;  /* crater flat ground, bowl radius, bowl depth */
  double vth;           /* per-component thermal speed */
  double drift[3];      /* mean velocity */
} synth_species;

/* Region excluded from loading: inside the sphere, or below the terrain. */
static int excluded(const synth_species *s, double x, double y, double z) {
  if (s->obj_kind == 1) {
    double dx = x - s->center[0], dy = y - s->center[1], dz = z - s->center[2];
    return dx * dx + dy * dy + dz * dz <= s->radius * s->radius;
  }
  if (s->obj_kind == 2) {
    double a = s->rim_radius, d = s->depth;
    double Rc = (a * a + d * d) / (2.0 * d);
    double zc = s->z_flat - d + Rc;
    if (z > s->z_flat) return 0;
    double dx = x - s->center[0], dy = y - s->center[1], dz = z - zc;
    return dx * dx + dy * dy + dz * dz >= Rc * Rc;
  }
  return 0;
}

static void one_particle(const synth_species *s, int64_t p, float *x, float *y, float *z,
                         float *vx, float *vy, float *vz) {
  const uint64_t key = sm_key(s->seed, s->stream, (uint64_t)p);
  const double n3[3] = {(double)s->nx, (double)s->ny, (double)s->nz};
  double g[3] = {0, 0, 0};
  for (int attempt = 0; attempt < 256; ++attempt) {
    for (int d = 0; d < 3; ++d) {
      double u = u01(key, (uint64_t)(3 * attempt + d));
      g[d] = floor(u * n3[d] * 65536.0) / 65536.0;
    }
    if (!excluded(s, g[0], g[1], g[2])) break;
  }
  double nrm[4];
  for (int pair = 0; pair < 2; ++pair) {
    double u1 = u01_open0(key, (uint64_t)(1000 + 2 * pair));
    double u2 = u01(key, (uint64_t)(1001 + 2 * pair));
    double r = sqrt(-2.0 * log(u1));
    nrm[2 * pair] = r * cos(6.283185307179586 * u2);
    nrm[2 * pair + 1] = r * sin(6.283185307179586 * u2);
  }
  x[0] = (float)g[0];
  y[0] = (float)g[1];
  z[0] = (float)g[2];
  vx[0] = (float)(s->drift[0] + s->vth * nrm[0]);
  vy[0] = (float)(s->drift[1] + s->vth * nrm[1]);
  vz[0] = (float)(s->drift[2] + s->vth * nrm[2]);
}

/* Particles start .. start+count-1 of one species (idx == NULL), or the listed
 * particle indices idx[0..count-1]. Outputs are count floats each. */
void synth_particles(const synth_species *s, int64_t start, int64_t count, const int64_t *idx,
                     float *x, float *y, float *z, float *vx, float *vy, float *vz) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    const int64_t p = idx ? idx[k] : start + k;
    one_particle(s, p, x + k, y + k, z + k, vx + k, vy + k, vz + k);
  }
}

static inline float noise(uint64_t seed, uint64_t comp, int64_t node, double amp) {
  if (amp == 0.0) return 0.0f;
  const uint64_t key = sm_key(seed, 100 + comp, (uint64_t)node);
  return (float)(amp * (2.0 * u01(key, 0) - 1.0));
}

/* Field of a uniformly charged ball of charge Q and radius R centred at c, in
 * units where div E = rho (no 4*pi*eps0 factor beyond 4*pi): E = Q r / (4 pi s^3),
 * s = max(|r|, R) (linear inside the ball), plus uniform noise in [-amp, amp)
 * per component; rounded to float. Nodes x fastest. */
void synth_node_E_coulomb(int32_t nx, int32_t ny, int32_t nz, const double c[3], double R,
                          double Q, double amp, uint64_t seed, float *Ex, float *Ey, float *Ez) {
  const int64_t sx = nx + 1, sy = (int64_t)(nx + 1) * (ny + 1);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k <= nz; ++k)
    for (int64_t j = 0; j <= ny; ++j)
      for (int64_t i = 0; i <= nx; ++i) {
        const int64_t node = i + sx * j + sy * k;
        double r[3] = {(double)i - c[0], (double)j - c[1], (double)k - c[2]};
        double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double s = rr > R ? rr : R;
        double f = Q / (4.0 * 3.141592653589793 * s * s * s);
        Ex[node] = (float)(f * r[0] + (double)noise(seed, 0, node, amp));
        Ey[node] = (float)(f * r[1] + (double)noise(seed, 1, node, amp));
        Ez[node] = (float)(f * r[2] + (double)noise(seed, 2, node, amp));
      }
}

/* Sheath-like field above a surface at height z0: Ez = -E0 exp(-max(z - z0, 0)/L),
 * Ex = Ey = 0, plus uniform noise in [-amp, amp) per component; rounded to float. */
void synth_node_E_sheath(int32_t nx, int32_t ny, int32_t nz, double z0, double E0, double L,
                         double amp, uint64_t seed, float *Ex, float *Ey, float *Ez) {
  const int64_t sx = nx + 1, sy = (int64_t)(nx + 1) * (ny + 1);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k <= nz; ++k) {
    double zz = (double)k - z0;
    double ez = -E0 * exp(-(zz > 0 ? zz : 0.0) / L);
    for (int64_t j = 0; j <= ny; ++j)
      for (int64_t i = 0; i <= nx; ++i) {
        const int64_t node = i + sx * j + sy * k;
        Ex[node] = noise(seed, 0, node, amp);
        Ey[node] = noise(seed, 1, node, amp);
        Ez[node] = (float)(ez + (double)noise(seed, 2, node, amp));
      }
  }
}
