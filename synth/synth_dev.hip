// Device twin of the seeded particle generator of synth.c (input generation
// only; no arithmetic of the PIC step): the same counter-based SplitMix64
// draws, rejection of the excluded region and Box-Muller normals, written
// straight into device arrays. Its values can differ from the host
// generator's in the last bits of the velocities (device log / sin / cos), so
// it serves workloads that are compared GPU against GPU (serving), not
// against the oracle.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm_key(uint64_t seed, uint64_t stream, uint64_t index) {
  uint64_t k = sm_mix(seed + GAMMA);
  k = sm_mix((k ^ stream) + GAMMA);
  return sm_mix((k ^ index) + GAMMA);
}
__device__ __forceinline__ uint64_t sm_draw(uint64_t key, uint64_t draw) {
  return sm_mix(key + (draw + 1) * GAMMA);
}
__device__ __forceinline__ double u01(uint64_t key, uint64_t draw) {
  return (double)(sm_draw(key, draw) >> 11) * (1.0 / 9007199254740992.0);
}
__device__ __forceinline__ double u01_open0(uint64_t key, uint64_t draw) {
  return ((double)(sm_draw(key, draw) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

struct SynthSpecies {  // same layout as synth_species in synth.c
  uint64_t seed, stream;
  int32_t nx, ny, nz, obj_kind;
  double center[3], radius, z_flat, rim_radius, depth, vth, drift[3];
};

__device__ bool excluded(const SynthSpecies &s, double x, double y, double z) {
  if (s.obj_kind == 1) {
    double dx = x - s.center[0], dy = y - s.center[1], dz = z - s.center[2];
    return dx * dx + dy * dy + dz * dz <= s.radius * s.radius;
  }
  if (s.obj_kind == 2) {
    double a = s.rim_radius, d = s.depth;
    double Rc = (a * a + d * d) / (2.0 * d);
    double zc = s.z_flat - d + Rc;
    if (z > s.z_flat) return false;
    double dx = x - s.center[0], dy = y - s.center[1], dz = z - zc;
    return dx * dx + dy * dy + dz * dz >= Rc * Rc;
  }
  return false;
}

__global__ void particles_kernel(SynthSpecies s, int64_t start, int64_t count, float *x, float *y,
                                 float *z, float *vx, float *vy, float *vz) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = sm_key(s.seed, s.stream, (uint64_t)(start + k));
    const double n3[3] = {(double)s.nx, (double)s.ny, (double)s.nz};
    double g[3] = {0, 0, 0};
    for (int attempt = 0; attempt < 256; ++attempt) {
      for (int d = 0; d < 3; ++d) g[d] = floor(u01(key, (uint64_t)(3 * attempt + d)) * n3[d] * 65536.0) / 65536.0;
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
    x[k] = (float)g[0];
    y[k] = (float)g[1];
    z[k] = (float)g[2];
    vx[k] = (float)(s.drift[0] + s.vth * nrm[0]);
    vy[k] = (float)(s.drift[1] + s.vth * nrm[1]);
    vz[k] = (float)(s.drift[2] + s.vth * nrm[2]);
  }
}

extern "C" int synth_particles_dev(const SynthSpecies *s, int64_t start, int64_t count, float *x,
                                   float *y, float *z, float *vx, float *vy, float *vz,
                                   void *stream) {
  if (count <= 0) return 0;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(particles_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     *s, start, count, x, y, z, vx, vy, vz);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
