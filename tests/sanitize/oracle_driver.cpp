// Drives every entry of the oracle once on small inputs, for a build under
// AddressSanitizer and UndefinedBehaviorSanitizer: the three representations
// with a sphere (one bin and surface patches) and a crater, reflection,
// injection and photoemission, the field solve with both preconditioners,
// with and without the object as an interface, and the surface source; runs on
// one and on three threads.
#include "../../oracle/pic_oracle.cpp"

#include <cstdio>
#include <random>

namespace {

orc_config base(int obj) {
  orc_config c{};
  c.nx = 12;
  c.ny = 10;
  c.nz = 12;
  c.h = 1.0;
  c.dt = 0.05;
  c.n_species = 3;
  const double q[3] = {-1.0, 1.0, -1.0}, m[3] = {1.0, 100.0, 1.0};
  for (int s = 0; s < 3; ++s) {
    c.q[s] = q[s];
    c.m[s] = m[s];
    c.w[s] = 1.0;
  }
  c.obj_kind = obj;
  c.pe_species = -1;
  if (obj == 1) {
    c.center[0] = 6.0; c.center[1] = 5.0; c.center[2] = 6.0;
    c.radius = 2.5;
  } else if (obj == 2) {
    c.center[0] = 6.0; c.center[1] = 5.0;
    c.z_flat = 4.0; c.rim_radius = 3.0; c.depth = 1.5;
  }
  return c;
}

int run(const orc_config& c, int64_t n, int nsteps, uint64_t seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::normal_distribution<double> N(0.0, 0.7);
  std::vector<int32_t> sp(n);
  std::vector<double> x(n), y(n), z(n), vx(n), vy(n), vz(n);
  for (int64_t p = 0; p < n; ++p) {
    sp[p] = (int32_t)(p % 2);
    x[p] = U(g) * c.nx; y[p] = U(g) * c.ny; z[p] = (c.obj_kind == 2 ? 0.5 : 0.0) + U(g) * (c.nz - 1);
    vx[p] = N(g); vy[p] = N(g); vz[p] = N(g);
  }
  const int64_t nodes = (int64_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
  std::vector<double> E[3];
  for (auto& e : E) {
    e.resize(nodes);
    for (auto& v : e) v = 0.2 * (U(g) - 0.5);
  }
  const int64_t cap = n + 200000;
  std::vector<double> o[6];
  for (auto& a : o) a.resize(cap);
  std::vector<int32_t> fate(cap), where(cap), when(cap), spo(cap);
  std::vector<double> rho(nodes);
  std::vector<int64_t> rhof(nodes), tally(((int64_t)c.nx * c.ny + 6 * 64 * 64) * 3), esc(18), inj(3);
  orc_out out{};
  out.x = o[0].data(); out.y = o[1].data(); out.z = o[2].data();
  out.vx = o[3].data(); out.vy = o[4].data(); out.vz = o[5].data();
  out.fate = fate.data(); out.where = where.data(); out.when = when.data();
  out.rho = rho.data(); out.rho_fixed = rhof.data(); out.tally = tally.data();
  out.escaped = esc.data(); out.cap = cap; out.species = spo.data(); out.injected = inj.data();
  const int rc = orc_run(&c, n, sp.data(), x.data(), y.data(), z.data(), vx.data(), vy.data(),
                         vz.data(), E[0].data(), E[1].data(), E[2].data(), nsteps, &out);
  if (rc == 0 && c.obj_kind != 0 && (c.obj_kind == 2 || c.sphere_patches > 0)) {
    std::vector<int64_t> surf(nodes, 0);
    if (orc_surface_rho(&c, tally.data(), surf.data()) != 0) return 10;
  }
  return rc;
}

}  // namespace

int main() {
  int bad = 0;
  for (int repr = 0; repr < 3; ++repr)
    for (int obj = 0; obj < 3; ++obj) {
      orc_config c = base(obj);
      c.repr = repr;
      if (obj == 1) c.sphere_patches = repr + 1;
      c.reflect = obj == 2 ? 4 : 1 | 4;
      c.inj_faces = obj == 2 ? 2 | 32 : 2 | 8;
      c.inj_seed = 7;
      for (int s = 0; s < 2; ++s) {
        c.inj_density[s] = 4.0;
        c.inj_vth[s] = s ? 0.1 : 1.0;
      }
      if (obj == 2) {
        c.pe_species = 2; c.pe_seed = 3; c.pe_flux = 30.0; c.pe_vth = 0.4;
        c.pe_sun[0] = 0.98; c.pe_sun[2] = 0.17;
      }
      c.threads = (repr + obj) % 2 ? 3 : 1;  // the threaded updates and deposit too
      const int rc = run(c, 3000, 6, 11 + repr * 3 + obj);
      if (rc != 0) {
        std::printf("orc_run repr %d obj %d: %d\n", repr, obj, rc);
        ++bad;
      }
    }
  // field solves
  const int nx = 16, ny = 12, nz = 8;
  const int64_t nodes = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  std::vector<double> rho(nodes), phi(nodes), r(nodes), zz(nodes), Ex(nodes), Ey(nodes), Ez(nodes);
  std::mt19937_64 g(5);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (auto& v : rho) v = U(g);
  for (auto& v : r) v = U(g);
  const double vals[6] = {1.0, 0.0, 0, 0, 0, 0};
  orc_field_object objs[3] = {};
  objs[1].kind = 1; objs[1].center[0] = 8; objs[1].center[1] = 6; objs[1].center[2] = 4;
  objs[1].radius = 3; objs[1].eps_in = 4;
  objs[2].kind = 2; objs[2].center[0] = 8; objs[2].center[1] = 6; objs[2].z_flat = 3;
  objs[2].rim_radius = 4; objs[2].depth = 2; objs[2].eps_in = 10;
  for (int op = 0; op < 2; ++op)
  for (int k = 0; k < 3; ++k)
    for (int pc = 0; pc < 2; ++pc)
      for (int mask : {32, 63, 1 | 2}) {
        std::fill(phi.begin(), phi.end(), 0.0);
        int32_t it = 0, lv = 0;
        double rr = 0;
        if (orc_field_solve(nx, ny, nz, 1.0, 1.0, mask, vals, rho.data(), phi.data(), 1e-10, 500, pc,
                            k ? &objs[k] : nullptr, op, &it, &rr, &lv) != 0) {
          std::printf("field solve op %d obj %d precond %d mask %d failed\n", op, k, pc, mask);
          ++bad;
        }
        orc_field_E(nx, ny, nz, 1.0, mask, phi.data(), Ex.data(), Ey.data(), Ez.data());
        if (orc_field_vcycle(nx, ny, nz, 1.0, 1.0, mask, k ? &objs[k] : nullptr, op, r.data(),
                             zz.data()) < 0)
          ++bad;
      }
  {  // the IFE pieces on their own
    std::vector<double> links(nodes * 18), out(38), K(16);
    for (int k = 0; k < 3; ++k)
      if (orc_ife_links(nx, ny, nz, 1.0, 1.0, k ? &objs[k] : nullptr, links.data()) != 0) ++bad;
    const double X[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
    const double ps[4] = {-0.3, 0.2, 0.0, 0.7};
    orc_ife_basis(X, ps, 4.0, 1.0, out.data());
    orc_ife_element(X, ps, 4.0, 1.0, K.data());
    int32_t T[60];
    orc_cube_tets(1, 2, 3, T);
  }
  std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
