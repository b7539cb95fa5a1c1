// C-ABI of the particle-mesh hot path: context, validation, device memory,
// orchestration of the kernels (pic_kernels.hip) and read-back.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "pic_internal.h"
#include "pic_ife.h"

using namespace pic;

namespace {

constexpr double kTwo32 = 4294967296.0;
constexpr int kDefaultSort = 0;  // re-bucket with fresh capacities only on demand
constexpr int64_t kMaxCapacity = 0x7fffffffLL - 1024;

thread_local std::string g_create_error = "no error";

// A roctx range over a scope: the library's calls show up by name on the host
// timeline of a profiler (rocprofv3 --marker-trace), around the kernels they
// enqueue; without a profiler each range costs two library calls.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

int64_t particle_bytes(int repr) {
  return repr == PIC_REPR_FP64 ? 48 : (repr == PIC_REPR_FP32_ABS ? 24 : 28);
}
int64_t elem_bytes(int repr) { return repr == PIC_REPR_FP64 ? 8 : 4; }
int64_t rho_elem(int dep) { return dep == PIC_DEP_ATOMIC_FP32 ? 4 : 8; }
int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

struct Dims {
  int ns, nx, ny, nz, ntx, nty, ntz, ntiles;
  int64_t nodes, nbins;
};

Dims dims_of(const pic_config &c) {
  Dims L;
  L.ns = c.n_species;
  L.nx = c.nx;
  L.ny = c.ny;
  L.nz = c.nz;
  L.ntx = (c.nx + kTile - 1) / kTile;
  L.nty = (c.ny + kTile - 1) / kTile;
  L.ntz = (c.nz + kTile - 1) / kTile;
  L.ntiles = L.ntx * L.nty * L.ntz;
  L.nodes = (int64_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
  L.nbins = c.object.kind == PIC_OBJ_CRATER
                ? (int64_t)c.nx * c.ny
                : (c.object.kind == PIC_OBJ_SPHERE
                       ? (c.object.patches > 0 ? 6 * (int64_t)c.object.patches * c.object.patches
                                               : 1)
                       : 0);
  return L;
}

// Slots of one particle buffer of a species: the tile regions (with spare
// room) followed by the overflow list.
int64_t buffer_slots(int64_t cap, int64_t ntiles) {
  return region_slots(cap, ntiles) + overflow_slots(cap);
}

// Device bytes of one species buffer (all arrays, 256-B aligned each).
int64_t species_buffer_bytes(int repr, int64_t slots) {
  const int64_t e = elem_bytes(repr);
  int64_t b = 6 * align256(slots * e);
  if (repr == PIC_REPR_FP32_CELL) b += align256(slots * 4);
  return b;
}

int64_t mesh_bytes(const pic_config &c, const Dims &L) {
  const int64_t e4 = c.repr == PIC_REPR_FP64 ? 32 : 16;
  int64_t b = 2 * align256(L.nodes * e4);                      // node E + staging
  b += align256(L.nodes * rho_elem(c.deposit));                 // rho
  b += align256(L.nbins * L.ns * 8) + align256(6 * L.ns * 8);  // tallies
  b += 2 * align256((int64_t)L.ns * L.ntiles * 16);              // two tile layouts
  b += 6 * align256((int64_t)L.ns * L.ntiles * 4);              // stayed / arrived counts
  b += 2 * align256((int64_t)L.ns * L.ntiles * 4);              // counts, cursors
  b += align256((int64_t)L.ns * L.ntiles * kNeighbours * 4);    // per-tile histograms
  b += 4096;                                                    // stats, counters
  return b;
}

bool is_finite(double v) { return std::isfinite(v); }

const char *validate_config(const pic_config *c) {
  if (!c) return "config is NULL";
  if (c->nx < 1 || c->ny < 1 || c->nz < 1 || c->nx > kMaxDim || c->ny > kMaxDim ||
      c->nz > kMaxDim)
    return "nx, ny, nz must be in 1..1023";
  if (!(c->h > 0) || !is_finite(c->h)) return "h must be finite and > 0";
  if (!(c->dt > 0) || !is_finite(c->dt)) return "dt must be finite and > 0";
  for (int d = 0; d < 3; ++d)
    if (!is_finite(c->origin[d])) return "origin must be finite";
  if (c->n_species < 1 || c->n_species > PIC_MAX_SPECIES) return "n_species must be in 1..4";
  for (int s = 0; s < c->n_species; ++s) {
    const pic_species &sp = c->species[s];
    if (!(sp.m > 0) || !is_finite(sp.m)) return "species mass must be finite and > 0";
    if (!is_finite(sp.q) || !is_finite(sp.weight)) return "species charge and weight must be finite";
    if (!(std::fabs(sp.q * sp.weight) <= 1048576.0)) return "|q*weight| must be <= 2^20";
    if (c->capacity[s] < 0 || c->capacity[s] > kMaxCapacity)
      return "capacity must be in 0..2^31-1025";
  }
  if (!c->alloc != !c->dealloc) return "alloc and dealloc must be given together";
  if (c->repr < 0 || c->repr > 2) return "repr must be a pic_repr";
  if (c->deposit < 0 || c->deposit > 2) return "deposit must be a pic_deposit";
  if (c->sort_interval < 0 || c->sort_interval > 1000000) return "sort_interval must be 0..1e6";
  if (c->reflect & ~63) return "reflect: only bits 0..5 (the six box faces)";
  if (c->object.kind == PIC_OBJ_CRATER && (c->reflect & 16))
    return "reflect: the crater's z- face is the terrain";
  const pic_object &o = c->object;
  if (o.kind < 0 || o.kind > 2) return "object.kind must be a pic_object_kind";
  if (o.patches < 0 || o.patches > 64) return "object.patches must be 0..64";
  if (o.patches && o.kind != PIC_OBJ_SPHERE) return "object.patches: spheres only";
  if (o.kind == PIC_OBJ_SPHERE) {
    for (int d = 0; d < 3; ++d)
      if (!is_finite(o.center[d])) return "sphere centre must be finite";
    if (!(o.radius > 0) || !is_finite(o.radius)) return "sphere radius must be finite and > 0";
  }
  if (o.kind == PIC_OBJ_CRATER) {
    if (!is_finite(o.center[0]) || !is_finite(o.center[1]) || !is_finite(o.z_flat))
      return "crater centre and z_flat must be finite";
    if (!(o.rim_radius > 0) || !is_finite(o.rim_radius)) return "crater rim_radius must be > 0";
    if (!(o.depth > 0) || !is_finite(o.depth)) return "crater depth must be > 0";
  }
  return nullptr;
}

Geom geometry_of(const pic_config &c) {
  Geom g{};
  g.kind = c.object.kind;
  g.patches = c.object.kind == PIC_OBJ_SPHERE ? c.object.patches : 0;
  double cc[3] = {0, 0, 0}, r2 = 0, zf = 0;
  if (c.object.kind == PIC_OBJ_SPHERE) {
    for (int d = 0; d < 3; ++d) cc[d] = (c.object.center[d] - c.origin[d]) / c.h;
    const double R = c.object.radius / c.h;
    r2 = R * R;
  } else if (c.object.kind == PIC_OBJ_CRATER) {
    // bowl sphere: radius Rc = (a^2 + d^2) / (2d), centre height z_flat - d + Rc
    const double a = c.object.rim_radius / c.h, dep = c.object.depth / c.h;
    zf = (c.object.z_flat - c.origin[2]) / c.h;
    const double Rc = (a * a + dep * dep) / (2.0 * dep);
    cc[0] = (c.object.center[0] - c.origin[0]) / c.h;
    cc[1] = (c.object.center[1] - c.origin[1]) / c.h;
    cc[2] = zf - dep + Rc;
    r2 = Rc * Rc;
  }
  for (int d = 0; d < 3; ++d) {
    g.c[d] = cc[d];
    g.ci[d] = (int32_t)std::floor(cc[d]);
    g.cf[d] = cc[d] - (double)g.ci[d];
  }
  g.r2 = r2;
  g.z_flat = zf;
  g.zfi = (int32_t)std::floor(zf);
  g.zff = zf - (double)g.zfi;
  return g;
}

int64_t footprint(const pic_config &c) {
  const Dims L = dims_of(c);
  int64_t b = mesh_bytes(c, L);
  for (int s = 0; s < c.n_species; ++s)
    b += 2 * species_buffer_bytes(c.repr, buffer_slots(c.capacity[s], L.ntiles));
  return b;
}

struct Ev {
  int kind;  // 0 step, 1 sort, 2 clear, 3 injection, 4 field solve
  hipEvent_t a, b;
};

}  // namespace

struct pic_ctx {
  pic_config cfg;
  Dims L;
  Geom geom;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::vector<void *> allocs;
  void *E = nullptr, *E_spare = nullptr, *rho = nullptr;
  int64_t *tally = nullptr, *escaped = nullptr, *stats = nullptr;
  int32_t *err = nullptr, *bad = nullptr;
  pic::Layout lay[2] = {};  // tile layouts (the one in use: lay[li])
  int32_t *nst[2] = {nullptr, nullptr}, *arr[2] = {nullptr, nullptr}, *ovf[2] = {nullptr, nullptr};
  // pinned copy of the overflow counts of the current buffer, refreshed after
  // each step: species with a nonzero count want their regions re-planned
  volatile int32_t *ovf_host = nullptr;
  int32_t *count = nullptr, *cursor = nullptr, *hist = nullptr;
  struct Species {
    int64_t cap = 0;
    int64_t slots = 0;     // per buffer
    int64_t ovf_base = 0;  // start of the overflow list (= tile region slots)
    int32_t ovf_cap = 0;
    int64_t n_buf = 0;  // entries of a freshly loaded (unsorted) species
    bool unsorted = true;
    int64_t loaded = 0;
    bool ids = false;
    void *mem[2] = {nullptr, nullptr};
    int64_t *ids_mem[2] = {nullptr, nullptr};
    PBuf buf[2];
  } sp[PIC_MAX_SPECIES];
  int cur = 0;  // buffer holding the current state
  int li = 0;   // layout in use
  bool sorted = false;  // every species is binned
  bool E_set = false;
  int since_sort = 0;
  int K = kDefaultSort;
  std::string msg = "no error";
  bool prof = false;
  std::vector<Ev> events;
  std::vector<hipEvent_t> event_pool;
  pic_profile acc{};
  pic_batch *batch = nullptr;  // attached to a batch
  bool inj_on = false;          // ambient particles are injected each step
  bool pe_on = false;           // photoemission from the terrain each step
  PhotoParams pe{};
  int32_t *inflow = nullptr;    // device [ns][ntiles]: photoemission room per re-bucketing
  pic_injection inj{};
  int64_t step_index = 0;       // pic_step steps since creation (injection key)
  int64_t *injected = nullptr;  // device [ns][kCountSlots]: particles injected
  bool deposited = false;       // rho holds a deposit
  // field solve (allocated at the first solve)
  double *fx = nullptr, *fr = nullptr, *fz = nullptr, *fp = nullptr, *fAp = nullptr,
         *fpart = nullptr;
  FieldCtrl *fctrl = nullptr, *fctrl_host = nullptr;
  bool solved = false;
  // multigrid preconditioner (planned and allocated at the first multigrid solve)
  int32_t mg_levels = -1;       // -1 not planned; 0 the grid does not coarsen
  MgLevel mg[kMaxLevels] = {};
  double *mg_ainv = nullptr;    // coarsest inverse (m x m)
  int32_t *mg_umap = nullptr;   // coarsest unknowns' nodes
  int32_t mg_m = 0;
  int32_t mg_mask = -1;         // faces and permittivities the inverse was computed for
  double mg_eps = 0.0, mg_eps_obj = 0.0;
  bool mg_bufs = false;         // multigrid level buffers allocated
  int32_t field_levels = 0;     // of the last solve
  // object as an interface: level sets (once) and diagonals (per permittivities)
  int32_t if_psi_levels = 0;    // levels whose psi is computed
  int32_t if_diag_levels = 0;   // levels whose diag matches if_eps_*
  double if_eps_in = 0.0, if_eps_out = 0.0;
  int64_t *rho_surf = nullptr;  // surface source (fixed point)
  // immersed finite elements: row index per node, the rows (capacity in
  // rows), the fine level's diagonal, a counter; the rows hold for
  // ife_key_* (object as an interface, eps inside, eps outside)
  int32_t *ife_srow = nullptr, *ife_count = nullptr;
  double *ife_rows = nullptr, *ife_diag = nullptr;
  int64_t ife_rows_cap = 0;
  bool ife_ready = false;
  int32_t ife_key_iface = -1;
  double ife_key_in = 0.0, ife_key_out = 0.0;
  void *scratch = nullptr;      // the device's scratch of the no-allocation id lookup
};

namespace {

pic_status fail(pic_ctx *c, pic_status st, const std::string &m) {
  if (c) c->msg = m;
  else g_create_error = m;
  return st;
}

pic_status hip_fail(pic_ctx *c, hipError_t e, const char *where) {
  return fail(c, PIC_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define PIC_HIP(ctx, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);  \
  } while (0)

void carve(PBuf &b, void *mem, int repr, int64_t cap) {
  char *p = (char *)mem;
  const int64_t a = align256(cap * elem_bytes(repr));
  for (int d = 0; d < 3; ++d) {
    b.pos[d] = p;
    p += a;
  }
  for (int d = 0; d < 3; ++d) {
    b.vel[d] = p;
    p += a;
  }
  b.cell = repr == PIC_REPR_FP32_CELL ? (int32_t *)p : nullptr;
  b.ids = nullptr;
}

// Device memory of a context: from the caller's allocator when pic_config
// gives one, else hipMalloc; returned the same way.
void *dev_alloc(const pic_config &cf, int64_t bytes) {
  if (cf.alloc) return cf.alloc((size_t)bytes, cf.alloc_user);
  void *p = nullptr;
  return hipMalloc(&p, (size_t)bytes) == hipSuccess ? p : nullptr;
}

void dev_free(const pic_config &cf, void *p) {
  if (!p) return;
  if (cf.dealloc) cf.dealloc(p, cf.alloc_user);
  else (void)hipFree(p);
}

void free_all(pic_ctx *c) {
  for (void *p : c->allocs) dev_free(c->cfg, p);
  c->allocs.clear();
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  c->event_pool.clear();
  for (Ev &e : c->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->events.clear();
  if (c->ovf_host) (void)hipHostFree((void *)c->ovf_host);
  c->ovf_host = nullptr;
  if (c->fctrl_host) (void)hipHostFree(c->fctrl_host);
  c->fctrl_host = nullptr;
}

// Allocation owned by the context until pic_destroy.
hipError_t dmalloc(pic_ctx *c, void **p, int64_t bytes) {
  if (bytes <= 0) bytes = 256;
  *p = dev_alloc(c->cfg, bytes);
  if (!*p) return hipErrorOutOfMemory;
  c->allocs.push_back(*p);
  return hipSuccess;
}

// Allocates n buffers (owned by the context) or none: if one fails, those
// made are given back and no *out is set.
bool dmalloc_all(pic_ctx *c, int n, void **const *out, const int64_t *bytes) {
  const size_t mark = c->allocs.size();
  std::vector<void *> got((size_t)n, nullptr);
  for (int i = 0; i < n; ++i) {
    if (dmalloc(c, &got[(size_t)i], bytes[i]) != hipSuccess) {
      while (c->allocs.size() > mark) {
        dev_free(c->cfg, c->allocs.back());
        c->allocs.pop_back();
      }
      return false;
    }
  }
  for (int i = 0; i < n; ++i) *out[i] = got[(size_t)i];
  return true;
}

hipEvent_t take_event(pic_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records a start event when profiling; returns its index or -1.
int prof_begin(pic_ctx *c, int kind) {
  if (!c->prof) return -1;
  Ev ev{kind, take_event(c), take_event(c)};
  if (!ev.a || !ev.b) return -1;
  (void)hipEventRecord(ev.a, c->stream);
  c->events.push_back(ev);
  return (int)c->events.size() - 1;
}

void prof_end(pic_ctx *c, int idx) {
  if (idx >= 0) (void)hipEventRecord(c->events[idx].b, c->stream);
}

// Folds recorded events into the totals (stream must be idle).
void prof_collect(pic_ctx *c) {
  for (Ev &e : c->events) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      if (e.kind == 0) {
        c->acc.step_launches++;
        c->acc.step_ms += ms;
      } else if (e.kind == 1) {
        c->acc.sort_launches++;
        c->acc.sort_ms += ms;
      } else if (e.kind == 3) {
        c->acc.inject_launches++;
        c->acc.inject_ms += ms;
      } else if (e.kind == 4) {
        c->acc.field_solves++;
        c->acc.field_ms += ms;
      } else if (e.kind == 5) {
        c->acc.photo_launches++;
        c->acc.photo_ms += ms;
      } else {
        c->acc.clear_launches++;
        c->acc.clear_ms += ms;
      }
    }
    c->event_pool.push_back(e.a);
    c->event_pool.push_back(e.b);
  }
  c->events.clear();
}

pic_status check_ctx(pic_ctx *c) {
  if (!c) return PIC_E_INVALID;
  if (c->batch) return fail(c, PIC_E_STATE, "the context is attached to a batch");
  return PIC_OK;
}

// Synchronises, folds profiling events and reports device-side errors.
pic_status sync_and_check(pic_ctx *c) {
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  if (c->prof) prof_collect(c);
  int32_t err = 0;
  PIC_HIP(c, hipMemcpy(&err, c->err, sizeof(err), hipMemcpyDeviceToHost));
  if (err) {
    const int32_t zero = 0;
    PIC_HIP(c, hipMemcpy(c->err, &zero, sizeof(zero), hipMemcpyHostToDevice));
    if (err & kErrCapacity)
      return fail(c, PIC_E_NOMEM, "particles were lost: the tile regions and overflow list are full");
    if (err == kErrSurface)
      return fail(c, PIC_E_RANGE, "a tally bin's collected charge reached 2^30 (surface source)");
    return fail(c, PIC_E_RANGE, "a particle position became non-finite or moved > 2^20 cells");
  }
  return PIC_OK;
}

Bins bins_of(pic_ctx *c) {
  Bins B{};
  B.lay = c->lay[c->li];
  for (int b = 0; b < 2; ++b) {
    B.nst[b] = c->nst[b];
    B.arr[b] = c->arr[b];
    B.ovf[b] = c->ovf[b];
  }
  for (int s = 0; s < c->L.ns; ++s) {
    B.ovf_base[s] = c->sp[s].ovf_base;
    B.ovf_cap[s] = c->sp[s].ovf_cap;
  }
  return B;
}

int32_t ids_mask(pic_ctx *c) {
  int32_t m = 0;
  for (int s = 0; s < c->L.ns; ++s)
    if (c->sp[s].ids) m |= 1 << s;
  return m;
}

StepParams step_params(pic_ctx *c) {
  StepParams P{};
  const Dims &L = c->L;
  P.ovf_groups = ovf_groups_for(L.ntiles);
  for (int s = 0; s < L.ns; ++s) {
    P.buf[0][s] = c->sp[s].buf[0];
    P.buf[1][s] = c->sp[s].buf[1];
  }
  P.remaining = 1;
  P.bins = bins_of(c);
  P.cur = c->cur;
  P.ns = L.ns;
  P.nx = L.nx;
  P.ny = L.ny;
  P.nz = L.nz;
  P.ntx = L.ntx;
  P.nty = L.nty;
  P.ntz = L.ntz;
  P.ntiles = L.ntiles;
  P.has_ids = ids_mask(c);
  P.reflect = c->cfg.reflect;
  const bool f64 = c->cfg.repr == PIC_REPR_FP64;
  for (int s = 0; s < L.ns; ++s) {
    const pic_species &sp = c->cfg.species[s];
    P.qmdt[s] = sp.q / sp.m * c->cfg.dt / c->cfg.h;
    P.chg[s] = sp.q * sp.weight;
    const double chgT = f64 ? P.chg[s] : (double)(float)P.chg[s];
    P.chg_fixed[s] = std::llrint(chgT * kTwo32);
  }
  P.dt = c->cfg.dt;
  P.geom = c->geom;
  P.E = c->E;
  P.rho = c->rho;
  P.tally = c->tally;
  P.escaped = c->escaped;
  P.stats = c->stats;
  P.err = c->err;
  return P;
}

// Injection of one step into the output buffer `out` of that step. The slab
// thickness and the mean ghost count per face cell are evaluated in FP64 from
// the physical inputs exactly as stated with pic_injection.
InjParams inj_params(pic_ctx *c, int out) {
  InjParams I{};
  const Dims &L = c->L;
  const pic_config &cfg = c->cfg;
  for (int s = 0; s < L.ns; ++s) I.out[s] = c->sp[s].buf[out];
  I.bins = bins_of(c);
  I.out_idx = out;
  I.ns = L.ns;
  I.nx = L.nx;
  I.ny = L.ny;
  I.nz = L.nz;
  I.ntx = L.ntx;
  I.nty = L.nty;
  I.ntiles = L.ntiles;
  I.has_ids = ids_mask(c);
  I.step = (int32_t)c->step_index;
  I.seed = c->inj.seed;
  I.dt = cfg.dt;
  const int n[3] = {L.nx, L.ny, L.nz};
  const double h3 = cfg.h * cfg.h * cfg.h;
  const bool f64 = cfg.repr == PIC_REPR_FP64;
  int64_t total = 0;
  for (int s = 0; s < L.ns; ++s) {
    const double ncell = c->inj.density[s] * h3;
    I.vth[s] = c->inj.vth[s] / cfg.h;
    for (int d = 0; d < 3; ++d) I.u[s][d] = c->inj.drift[s][d] / cfg.h;
    for (int f = 0; f < 6; ++f) {
      I.first[s * 6 + f] = total;
      const int axis = f / 2;
      const double un = (f & 1) ? -I.u[s][axis] : I.u[s][axis];
      double th = cfg.dt * ((un > 0.0 ? un : 0.0) + 6.0 * I.vth[s]);
      if (th > 1.0) th = 1.0;
      I.L[s][f] = th;
      I.mean[s][f] = ncell * th;
      I.gmax[s][f] = (int64_t)std::floor(I.mean[s][f]) + 1;
      if (((c->inj.faces >> f) & 1) && ncell > 0.0)
        total += (int64_t)n[axis == 0 ? 1 : 0] * n[axis == 2 ? 1 : 2] * I.gmax[s][f];
    }
    const pic_species &sp = cfg.species[s];
    I.chg[s] = sp.q * sp.weight;
    const double chgT = f64 ? I.chg[s] : (double)(float)I.chg[s];
    I.chg_fixed[s] = std::llrint(chgT * kTwo32);
  }
  I.first[L.ns * 6] = total;
  I.geom = c->geom;
  I.rho = c->rho;
  I.tally = c->tally;
  I.injected = c->injected;
  I.err = c->err;
  return I;
}

// Re-bucketing with fresh tile capacities of the species in want and of every
// freshly loaded species: from the current buffer (tile regions + overflow
// list, or the flat range of a freshly loaded species) into the spare buffer
// under a new layout, which then becomes the species' current buffer (the
// buffer index stays; the two buffers of the species swap). The other species
// keep their particles and layout as they are.
pic_status do_sort(pic_ctx *c, int32_t want) {
  const Range range("pic_replan");
  const Dims &L = c->L;
  const int32_t all = (1 << L.ns) - 1;
  SortParams S{};
  S.sel = want & all;
  int64_t max_src = 0;
  for (int s = 0; s < L.ns; ++s) {
    const pic_ctx::Species &sp = c->sp[s];
    S.src[s] = sp.buf[c->cur];
    S.dst[s] = sp.buf[1 - c->cur];
    if (sp.unsorted) {
      S.unsorted |= 1 << s;
      S.n_src[s] = sp.n_buf;
      if (sp.n_buf > max_src) max_src = sp.n_buf;
    }
    S.region_cap[s] = sp.ovf_base;
  }
  S.sel |= S.unsorted;
  if (S.sel == 0) {
    c->sorted = true;
    return PIC_OK;
  }
  S.bins = bins_of(c);
  S.inflow = c->pe_on ? c->inflow : nullptr;
  S.dst_lay = c->lay[1 - c->li];
  S.cur = c->cur;
  S.count = c->count;
  S.cursor = c->cursor;
  S.hist = c->hist;
  S.ns = L.ns;
  S.nx = L.nx;
  S.ny = L.ny;
  S.nz = L.nz;
  S.ntx = L.ntx;
  S.nty = L.nty;
  S.ntz = L.ntz;
  S.ntiles = L.ntiles;
  S.has_ids = ids_mask(c);
  S.err = c->err;
  const int pe = prof_begin(c, 1);
  PIC_HIP(c, launch_sort_count(c->cfg.repr, S, max_src, c->stream));
  PIC_HIP(c, launch_sort_scan(S, c->stream));
  PIC_HIP(c, launch_sort_scatter(c->cfg.repr, S, max_src, c->stream));
  PIC_HIP(c, launch_sort_commit(S, c->stream));
  prof_end(c, pe);
  for (int s = 0; s < L.ns; ++s) {
    if (!((S.sel >> s) & 1)) continue;
    pic_ctx::Species &sp = c->sp[s];
    std::swap(sp.mem[0], sp.mem[1]);
    std::swap(sp.ids_mem[0], sp.ids_mem[1]);
    std::swap(sp.buf[0], sp.buf[1]);
    sp.unsorted = false;
  }
  c->sorted = true;
  if (S.sel == all) c->since_sort = 0;
  if (c->ovf_host)
    for (int s = 0; s < L.ns; ++s)
      if ((S.sel >> s) & 1) c->ovf_host[s] = 0;
  return PIC_OK;
}

// Before a step: rho, and the overflow counts of the buffer the step writes.
pic_status clear_rho(pic_ctx *c) {
  const int pe = prof_begin(c, 2);
  PIC_HIP(c, launch_step_clear(c->rho, c->L.nodes * rho_elem(c->cfg.deposit), c->ovf[1 - c->cur],
                               c->L.ns, c->stream));
  prof_end(c, pe);
  return PIC_OK;
}

// Particles injected per species: the sum of the species' count slots.
pic_status read_injected(pic_ctx *c, int64_t *out) {
  const int ns = c->L.ns;
  std::vector<int64_t> v((size_t)ns * kCountSlots);
  PIC_HIP(c, hipMemcpy(v.data(), c->injected, v.size() * 8, hipMemcpyDeviceToHost));
  for (int s = 0; s < ns; ++s) {
    int64_t a = 0;
    for (int k = 0; k < kCountSlots; ++k) a += v[(size_t)s * kCountSlots + k];
    out[s] = a;
  }
  return PIC_OK;
}

// Resets the collected counts, escape counters and injected count of one
// species.
pic_status reset_species_counters(pic_ctx *c, int s) {
  const Dims &L = c->L;
  std::vector<int64_t> t(L.nbins * L.ns), e(6 * L.ns);
  if (L.nbins) PIC_HIP(c, hipMemcpy(t.data(), c->tally, t.size() * 8, hipMemcpyDeviceToHost));
  PIC_HIP(c, hipMemcpy(e.data(), c->escaped, e.size() * 8, hipMemcpyDeviceToHost));
  for (int64_t b = 0; b < L.nbins; ++b) t[b * L.ns + s] = 0;
  for (int f = 0; f < 6; ++f) e[f * L.ns + s] = 0;
  if (L.nbins) PIC_HIP(c, hipMemcpy(c->tally, t.data(), t.size() * 8, hipMemcpyHostToDevice));
  PIC_HIP(c, hipMemcpy(c->escaped, e.data(), e.size() * 8, hipMemcpyHostToDevice));
  const std::vector<int64_t> z(kCountSlots, 0);
  PIC_HIP(c, hipMemcpy(c->injected + (size_t)s * kCountSlots, z.data(), kCountSlots * 8,
                       hipMemcpyHostToDevice));
  return PIC_OK;
}

// Makes the spare buffer of species s (just filled with n particles, unsorted)
// its current buffer; the other species keep theirs. The next step re-buckets.
pic_status commit_species(pic_ctx *c, int s, int64_t n, bool ids) {
  pic_ctx::Species &S = c->sp[s];
  std::swap(S.mem[0], S.mem[1]);
  std::swap(S.ids_mem[0], S.ids_mem[1]);
  std::swap(S.buf[0], S.buf[1]);
  S.n_buf = n;
  S.unsorted = true;
  S.loaded = n;
  S.ids = ids;
  c->sorted = false;
  return reset_species_counters(c, s);
}

// Ranges [offset, offset + count) of the current buffer that hold species s
// (tile regions and the overflow list). Re-buckets first if needed (the
// re-bucketing does not change any result). Synchronises.
// The live slot ranges (first, count) of species s in the current buffer
// (binned first if needed); tiles (nullable) gets each range's tile, -1 for
// the overflow list.
pic_status species_ranges(pic_ctx *c, int s, std::vector<std::pair<int64_t, int64_t>> &out,
                          std::vector<int32_t> *tiles = nullptr) {
  pic_status st;
  if (!c->sorted && (st = do_sort(c, 0)) != PIC_OK) return st;
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  const int nt = c->L.ntiles;
  std::vector<int64_t> base(nt);
  std::vector<int32_t> cap(nt), sz(nt), nst(nt), arr(nt);
  const int64_t o = (int64_t)s * nt;
  const pic::Layout &lay = c->lay[c->li];
  PIC_HIP(c, hipMemcpy(base.data(), lay.base + o, nt * 8, hipMemcpyDeviceToHost));
  PIC_HIP(c, hipMemcpy(cap.data(), lay.cap + o, nt * 4, hipMemcpyDeviceToHost));
  PIC_HIP(c, hipMemcpy(sz.data(), lay.sz + o, nt * 4, hipMemcpyDeviceToHost));
  PIC_HIP(c, hipMemcpy(nst.data(), c->nst[c->cur] + o, nt * 4, hipMemcpyDeviceToHost));
  PIC_HIP(c, hipMemcpy(arr.data(), c->arr[c->cur] + o, nt * 4, hipMemcpyDeviceToHost));
  int32_t novf = 0;
  PIC_HIP(c, hipMemcpy(&novf, c->ovf[c->cur] + s, 4, hipMemcpyDeviceToHost));
  out.clear();
  if (tiles) tiles->clear();
  for (int t = 0; t < nt; ++t) {
    const int64_t n1 = std::min(nst[t], sz[t]), na = std::min(arr[t], cap[t] - sz[t]);
    if (n1 > 0) out.emplace_back(base[t], n1);
    if (na > 0) out.emplace_back(base[t] + cap[t] - na, na);
    if (tiles) tiles->insert(tiles->end(), (n1 > 0) + (na > 0), t);
  }
  const int64_t no = std::min(novf, c->sp[s].ovf_cap);
  if (no > 0) {
    out.emplace_back(c->sp[s].ovf_base, no);
    if (tiles) tiles->push_back(-1);
  }
  return PIC_OK;
}

pic_status ensure_ids(pic_ctx *c, int s) {
  pic_ctx::Species &S = c->sp[s];
  if (S.ids_mem[0]) return PIC_OK;
  const int64_t b = align256(S.slots * 8);
  void **const outs[2] = {(void **)&S.ids_mem[0], (void **)&S.ids_mem[1]};
  const int64_t bytes[2] = {b, b};
  if (!dmalloc_all(c, 2, outs, bytes)) return fail(c, PIC_E_NOMEM, "no device memory for ids");
  S.buf[0].ids = S.ids_mem[0];
  S.buf[1].ids = S.ids_mem[1];
  return PIC_OK;
}

// Checks of an id lookup; then synchronises (reporting device-side errors)
// and makes sure the particles are binned. PIC_OK with nothing to do for n == 0.
pic_status by_id_prepare(pic_ctx *c, int32_t species, int64_t n, const int64_t *ids_sorted,
                         const int32_t *found, const double *x, const double *y, const double *z,
                         const double *vx, const double *vy, const double *vz) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (species < 0 || species >= c->L.ns) return fail(c, PIC_E_INVALID, "species out of range");
  if (n < 0) return fail(c, PIC_E_INVALID, "n must be >= 0");
  if (n > 0 && (!ids_sorted || !found || !x || !y || !z || !vx || !vy || !vz))
    return fail(c, PIC_E_INVALID, "arrays must not be NULL");
  for (int64_t k = 1; k < n; ++k)
    if (!(ids_sorted[k - 1] < ids_sorted[k]))
      return fail(c, PIC_E_INVALID, "ids must be distinct and ascending");
  if (!c->sp[species].ids) return fail(c, PIC_E_STATE, "no ids were loaded for this species");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK || n == 0) return st;
  if (!c->sorted && (st = do_sort(c, 0)) != PIC_OK) return st;
  return PIC_OK;
}

}  // namespace

extern "C" {

const char *pic_status_string(pic_status s) {
  switch (s) {
    case PIC_OK: return "PIC_OK";
    case PIC_E_INVALID: return "PIC_E_INVALID";
    case PIC_E_NOMEM: return "PIC_E_NOMEM";
    case PIC_E_DEVICE: return "PIC_E_DEVICE";
    case PIC_E_STATE: return "PIC_E_STATE";
    case PIC_E_RANGE: return "PIC_E_RANGE";
  }
  return "unknown pic_status";
}

const char *pic_last_error(const pic_ctx *ctx) {
  return ctx ? ctx->msg.c_str() : g_create_error.c_str();
}

pic_status pic_create(const pic_config *cfg, pic_ctx **out) {
  if (!out) return fail(nullptr, PIC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (const char *m = validate_config(cfg)) return fail(nullptr, PIC_E_INVALID, m);
  const int64_t need = footprint(*cfg);
  if (const char *b = std::getenv("PIC_HBM_BUDGET_BYTES")) {
    const long long budget = std::atoll(b);
    if (budget > 0 && need > budget)
      return fail(nullptr, PIC_E_NOMEM,
                  "footprint " + std::to_string(need) + " B exceeds PIC_HBM_BUDGET_BYTES");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, PIC_E_DEVICE, "no HIP device available");
  pic_ctx *c = new pic_ctx();
  c->cfg = *cfg;
  c->L = dims_of(*cfg);
  c->geom = geometry_of(*cfg);
  c->K = cfg->sort_interval > 0 ? cfg->sort_interval : kDefaultSort;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, PIC_E_DEVICE, "hipGetDevice failed");
  }
  size_t free_b = 0, total_b = 0;
  // (a caller's allocator may hold cached memory that hipMemGetInfo counts as
  // used: it decides by itself)
  if (!cfg->alloc && hipMemGetInfo(&free_b, &total_b) == hipSuccess && (size_t)need > free_b) {
    delete c;
    return fail(nullptr, PIC_E_NOMEM,
                "footprint " + std::to_string(need) + " B exceeds free device memory");
  }
  auto bail = [&](pic_status st, const std::string &m) {
    free_all(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return fail(nullptr, st, m);
  };
  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(PIC_E_DEVICE, "hipStreamCreate failed");
    c->own_stream = true;
  }
  // the scratch of pic_get_particles_by_id_noalloc on this device (its
  // address looked up once per device)
  if (noalloc_scratch(&c->scratch) != hipSuccess)
    return bail(PIC_E_DEVICE, "hipGetSymbolAddress of the scratch area failed");
  const Dims &L = c->L;
  const int64_t e4 = cfg->repr == PIC_REPR_FP64 ? 32 : 16;
  void *p = nullptr;
  struct Req {
    void **dst;
    int64_t bytes;
  } reqs[] = {
      {&c->E, L.nodes * e4},
      {&c->E_spare, L.nodes * e4},
      {&c->rho, L.nodes * rho_elem(cfg->deposit)},
      {(void **)&c->tally, L.nbins * L.ns * 8},
      {(void **)&c->escaped, 6 * L.ns * 8},
      {(void **)&c->stats, 64},
      {(void **)&c->err, 64},
      {(void **)&c->bad, 64},
      {(void **)&c->lay[0].base, (int64_t)L.ns * L.ntiles * 8},
      {(void **)&c->lay[1].base, (int64_t)L.ns * L.ntiles * 8},
      {(void **)&c->lay[0].cap, (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->lay[1].cap, (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->lay[0].sz, (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->lay[1].sz, (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->nst[0], (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->nst[1], (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->arr[0], (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->arr[1], (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->ovf[0], 64},
      {(void **)&c->ovf[1], 64},
      {(void **)&c->injected, 8 * PIC_MAX_SPECIES * kCountSlots},
      {(void **)&c->count, (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->cursor, (int64_t)L.ns * L.ntiles * 4},
      {(void **)&c->hist, (int64_t)L.ns * L.ntiles * kNeighbours * 4},
  };
  for (Req &r : reqs) {
    if (dmalloc(c, &p, r.bytes) != hipSuccess)
      return bail(PIC_E_NOMEM, "device memory allocation failed");
    *r.dst = p;
    if (launch_fill(p, r.bytes > 0 ? r.bytes : 256, c->stream) != hipSuccess)
      return bail(PIC_E_DEVICE, "clearing a new buffer failed");
  }
  void *fh = nullptr;
  if (hipHostMalloc(&fh, 64, hipHostMallocDefault) != hipSuccess)
    return bail(PIC_E_NOMEM, "hipHostMalloc failed");
  c->ovf_host = (volatile int32_t *)fh;
  for (int s = 0; s < PIC_MAX_SPECIES; ++s) c->ovf_host[s] = 0;
  for (int s = 0; s < L.ns; ++s) {
    pic_ctx::Species &S = c->sp[s];
    S.cap = cfg->capacity[s];
    S.slots = buffer_slots(S.cap, L.ntiles);
    S.ovf_base = region_slots(S.cap, L.ntiles);
    S.ovf_cap = overflow_slots(S.cap);
    for (int b = 0; b < 2; ++b) {
      if (dmalloc(c, &S.mem[b], species_buffer_bytes(cfg->repr, S.slots)) != hipSuccess)
        return bail(PIC_E_NOMEM, "allocation of the particle buffers failed");
      carve(S.buf[b], S.mem[b], cfg->repr, S.slots);
    }
  }
  // (only this context's stream: work of other contexts may be in flight)
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(PIC_E_DEVICE, "device error at create");
  *out = c;
  return PIC_OK;
}

void pic_destroy(pic_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

pic_status pic_load_particles(pic_ctx *c, int32_t species, int64_t n, const double *x,
                              const double *y, const double *z, const double *vx,
                              const double *vy, const double *vz, const int64_t *ids) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (species < 0 || species >= c->L.ns) return fail(c, PIC_E_INVALID, "species out of range");
  pic_ctx::Species &S = c->sp[species];
  if (n < 0 || n > S.cap) return fail(c, PIC_E_INVALID, "n must be in 0..capacity");
  if (n > 0 && (!x || !y || !z || !vx || !vy || !vz))
    return fail(c, PIC_E_INVALID, "particle arrays must not be NULL");
  const pic_config &cf = c->cfg;
  const int repr = cf.repr;
  const double *X[3] = {x, y, z}, *V[3] = {vx, vy, vz};
  const int32_t n3[3] = {cf.nx, cf.ny, cf.nz};
  const int64_t e = elem_bytes(repr);
  std::vector<char> pos(3 * n * e + 1), vel(3 * n * e + 1);
  std::vector<int32_t> cell(repr == PIC_REPR_FP32_CELL ? n : 0);
  for (int64_t p = 0; p < n; ++p) {
    int ci[3];
    for (int d = 0; d < 3; ++d) {
      const double g = (X[d][p] - cf.origin[d]) / cf.h;
      if (!(g >= 0.0 && g < (double)n3[d]))
        return fail(c, PIC_E_INVALID, "particle " + std::to_string(p) + " is outside the box");
      const double u = V[d][p] / cf.h;
      if (!is_finite(u)) return fail(c, PIC_E_INVALID, "velocities must be finite");
      if (repr == PIC_REPR_FP64) {
        ((double *)pos.data())[d * n + p] = g;
        ((double *)vel.data())[d * n + p] = u;
      } else if (repr == PIC_REPR_FP32_ABS) {
        if (!((float)g < (float)n3[d]))  // rounded up onto the upper face
          return fail(c, PIC_E_INVALID, "particle " + std::to_string(p) + " is outside the box");
        ((float *)pos.data())[d * n + p] = (float)g;
        ((float *)vel.data())[d * n + p] = (float)u;
      } else {
        int i = (int)std::floor(g);
        float o = (float)(g - (double)i);
        if (o == 1.0f) {  // offset rounded up into the next cell
          o = 0.0f;
          i += 1;
        }
        if (i >= n3[d])
          return fail(c, PIC_E_INVALID, "particle " + std::to_string(p) + " is outside the box");
        ci[d] = i;
        ((float *)pos.data())[d * n + p] = off_pack(o, i);
        ((float *)vel.data())[d * n + p] = (float)u;
      }
    }
    if (repr == PIC_REPR_FP32_CELL)
      cell[p] = ci[0] | (ci[1] << kCellBits) | (ci[2] << (2 * kCellBits));
  }
  if (ids) {
    pic_status st = ensure_ids(c, species);
    if (st != PIC_OK) return st;
  }
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  const PBuf &B = S.buf[1 - c->cur];  // the spare buffer
  for (int d = 0; d < 3 && n > 0; ++d) {
    PIC_HIP(c, hipMemcpy(B.pos[d], pos.data() + d * n * e, n * e, hipMemcpyHostToDevice));
    PIC_HIP(c, hipMemcpy(B.vel[d], vel.data() + d * n * e, n * e, hipMemcpyHostToDevice));
  }
  if (repr == PIC_REPR_FP32_CELL && n > 0)
    PIC_HIP(c, hipMemcpy(B.cell, cell.data(), n * 4, hipMemcpyHostToDevice));
  if (ids && n > 0) PIC_HIP(c, hipMemcpy(B.ids, ids, n * 8, hipMemcpyHostToDevice));
  return commit_species(c, species, n, ids != nullptr);
}

pic_status pic_load_particles_f32_dev(pic_ctx *c, int32_t species, int64_t n, const float *x,
                                      const float *y, const float *z, const float *vx,
                                      const float *vy, const float *vz, const int64_t *ids) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (species < 0 || species >= c->L.ns) return fail(c, PIC_E_INVALID, "species out of range");
  pic_ctx::Species &S = c->sp[species];
  if (n < 0 || n > S.cap) return fail(c, PIC_E_INVALID, "n must be in 0..capacity");
  if (n > 0 && (!x || !y || !z || !vx || !vy || !vz))
    return fail(c, PIC_E_INVALID, "particle arrays must not be NULL");
  if (ids) {
    pic_status st = ensure_ids(c, species);
    if (st != PIC_OK) return st;
  }
  LoadParams Lp{};
  Lp.x[0] = x;
  Lp.x[1] = y;
  Lp.x[2] = z;
  Lp.v[0] = vx;
  Lp.v[1] = vy;
  Lp.v[2] = vz;
  Lp.ids = ids;
  Lp.out = S.buf[1 - c->cur];
  Lp.n = n;
  for (int d = 0; d < 3; ++d) Lp.origin[d] = c->cfg.origin[d];
  Lp.h = c->cfg.h;
  Lp.nx = c->cfg.nx;
  Lp.ny = c->cfg.ny;
  Lp.nz = c->cfg.nz;
  Lp.bad = c->bad;
  PIC_HIP(c, launch_fill(c->bad, 4, c->stream));
  PIC_HIP(c, launch_load_f32(c->cfg.repr, Lp, c->stream));
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  int32_t bad = 0;
  PIC_HIP(c, hipMemcpy(&bad, c->bad, 4, hipMemcpyDeviceToHost));
  if (bad) return fail(c, PIC_E_INVALID, std::to_string(bad) + " particles are outside the box");
  return commit_species(c, species, n, ids != nullptr);
}

pic_status pic_set_node_E(pic_ctx *c, const double *Ex, const double *Ey, const double *Ez) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!Ex || !Ey || !Ez) return fail(c, PIC_E_INVALID, "field arrays must not be NULL");
  const int64_t nodes = c->L.nodes;
  const bool f64 = c->cfg.repr == PIC_REPR_FP64;
  std::vector<char> buf(nodes * (f64 ? 32 : 16));
  for (int64_t i = 0; i < nodes; ++i) {
    if (!is_finite(Ex[i]) || !is_finite(Ey[i]) || !is_finite(Ez[i]))
      return fail(c, PIC_E_INVALID, "node field must be finite");
    if (f64) {
      double *d = (double *)buf.data() + 4 * i;
      d[0] = Ex[i];
      d[1] = Ey[i];
      d[2] = Ez[i];
      d[3] = 0;
    } else {
      float *f = (float *)buf.data() + 4 * i;
      f[0] = (float)Ex[i];
      f[1] = (float)Ey[i];
      f[2] = (float)Ez[i];
      f[3] = 0;
    }
  }
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  PIC_HIP(c, hipMemcpy(c->E, buf.data(), buf.size(), hipMemcpyHostToDevice));
  c->E_set = true;
  return PIC_OK;
}

pic_status pic_get_node_E(pic_ctx *c, double *Ex, double *Ey, double *Ez) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!Ex || !Ey || !Ez) return fail(c, PIC_E_INVALID, "field arrays must not be NULL");
  if (!c->E_set) return fail(c, PIC_E_STATE, "no node field yet");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  const int64_t nodes = c->L.nodes;
  const bool f64 = c->cfg.repr == PIC_REPR_FP64;
  std::vector<char> buf(nodes * (f64 ? 32 : 16));
  PIC_HIP(c, hipMemcpy(buf.data(), c->E, buf.size(), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < nodes; ++i) {
    if (f64) {
      const double *d = (const double *)buf.data() + 4 * i;
      Ex[i] = d[0];
      Ey[i] = d[1];
      Ez[i] = d[2];
    } else {
      const float *f = (const float *)buf.data() + 4 * i;
      Ex[i] = f[0];
      Ey[i] = f[1];
      Ez[i] = f[2];
    }
  }
  return PIC_OK;
}

pic_status pic_set_node_E_f32_dev(pic_ctx *c, const float *Ex, const float *Ey, const float *Ez) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!Ex || !Ey || !Ez) return fail(c, PIC_E_INVALID, "field arrays must not be NULL");
  PIC_HIP(c, launch_fill(c->bad, 4, c->stream));
  PIC_HIP(c, launch_node_E_f32(c->cfg.repr, Ex, Ey, Ez, c->E_spare, c->L.nodes, c->bad,
                               c->stream));
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  int32_t bad = 0;
  PIC_HIP(c, hipMemcpy(&bad, c->bad, 4, hipMemcpyDeviceToHost));
  if (bad) return fail(c, PIC_E_INVALID, "node field must be finite");
  std::swap(c->E, c->E_spare);
  c->E_set = true;
  return PIC_OK;
}

pic_status pic_step(pic_ctx *c, int32_t nsteps) {
  const Range range("pic_step");
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (nsteps < 0) return fail(c, PIC_E_INVALID, "nsteps must be >= 0");
  if (nsteps > 0 && !c->E_set) return fail(c, PIC_E_STATE, "pic_set_node_E has not been called");
  pic_status st;
  if (nsteps == 0) {
    if (!c->sorted && (st = do_sort(c, 0)) != PIC_OK) return st;
    if ((st = clear_rho(c)) != PIC_OK) return st;
    StepParams P = step_params(c);
    const int pe = prof_begin(c, 0);
    PIC_HIP(c, launch_step(c->cfg.repr, c->cfg.deposit, false, P, c->stream));
    prof_end(c, pe);
    c->deposited = true;
    return PIC_OK;
  }
  for (int k = 0; k < nsteps; ++k) {
    // particles are re-bucketed by the step itself; a re-bucketing with fresh
    // tile capacities runs for a species after its load and when one of its
    // tiles ran out of spare room (its overflow list is not empty; seen through
    // the pinned counts, which may lag by a step: the overflow list keeps every
    // particle in the meantime), and for all species every K steps if K > 0
    int32_t want = 0;
    if (c->ovf_host)
      for (int s = 0; s < c->L.ns; ++s)
        if (c->ovf_host[s] > 0) want |= 1 << s;
    if (c->K > 0 && c->since_sort >= c->K) want = (1 << c->L.ns) - 1;
    if ((want || !c->sorted) && (st = do_sort(c, want)) != PIC_OK) return st;
    if ((st = clear_rho(c)) != PIC_OK) return st;
    StepParams P = step_params(c);
    const int pe = prof_begin(c, 0);
    PIC_HIP(c, launch_step(c->cfg.repr, c->cfg.deposit, true, P, c->stream));
    prof_end(c, pe);
    if (c->inj_on) {
      const InjParams I = inj_params(c, 1 - c->cur);
      if (I.first[c->L.ns * 6] > (int64_t(1) << 36))
        return fail(c, PIC_E_INVALID, "injection: more than 2^36 ghost slots per step");
      const int pi = prof_begin(c, 3);
      PIC_HIP(c, launch_inject(c->cfg.repr, c->cfg.deposit, I, c->stream));
      prof_end(c, pi);
    }
    if (c->pe_on) {
      InjParams I = inj_params(c, 1 - c->cur);
      I.pe = c->pe;
      const int pp = prof_begin(c, 5);
      PIC_HIP(c, launch_photo(c->cfg.repr, c->cfg.deposit, I, c->stream));
      prof_end(c, pp);
    }
    PIC_HIP(c, hipMemcpyAsync((void *)c->ovf_host, c->ovf[1 - c->cur],
                              sizeof(int32_t) * c->L.ns, hipMemcpyDeviceToHost, c->stream));
    c->cur = 1 - c->cur;
    c->since_sort++;
    c->step_index++;
    c->deposited = true;
  }
  return PIC_OK;
}

pic_status pic_synchronize(pic_ctx *c) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  return sync_and_check(c);
}

pic_status pic_get_rho(pic_ctx *c, double *rho, int64_t *rho_fixed) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!rho) return fail(c, PIC_E_INVALID, "rho must not be NULL");
  if (rho_fixed && c->cfg.deposit != PIC_DEP_FIXED64)
    return fail(c, PIC_E_INVALID, "rho_fixed is only defined for the fixed-point deposit");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  const int64_t nodes = c->L.nodes;
  const double h3 = c->cfg.h * c->cfg.h * c->cfg.h;
  if (c->cfg.deposit == PIC_DEP_FIXED64) {
    std::vector<int64_t> v(nodes);
    PIC_HIP(c, hipMemcpy(v.data(), c->rho, nodes * 8, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nodes; ++i) rho[i] = ((double)v[i] * (1.0 / kTwo32)) / h3;
    if (rho_fixed) std::memcpy(rho_fixed, v.data(), nodes * 8);
  } else if (c->cfg.deposit == PIC_DEP_ATOMIC_FP32) {
    std::vector<float> v(nodes);
    PIC_HIP(c, hipMemcpy(v.data(), c->rho, nodes * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nodes; ++i) rho[i] = (double)v[i] / h3;
  } else {
    std::vector<double> v(nodes);
    PIC_HIP(c, hipMemcpy(v.data(), c->rho, nodes * 8, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nodes; ++i) rho[i] = v[i] / h3;
  }
  return PIC_OK;
}

int64_t pic_num_bins(const pic_ctx *c) { return c ? c->L.nbins : 0; }

pic_status pic_get_surface_charge(pic_ctx *c, int64_t nbins, double *charge, int64_t *counts) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (nbins != c->L.nbins) return fail(c, PIC_E_INVALID, "nbins must equal pic_num_bins");
  if (nbins > 0 && !charge) return fail(c, PIC_E_INVALID, "charge must not be NULL");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  const int ns = c->L.ns;
  std::vector<int64_t> t(nbins * ns);
  if (nbins) PIC_HIP(c, hipMemcpy(t.data(), c->tally, t.size() * 8, hipMemcpyDeviceToHost));
  for (int64_t b = 0; b < nbins; ++b) {
    double q = 0;
    for (int s = 0; s < ns; ++s) {
      const pic_species &sp = c->cfg.species[s];
      q += (sp.q * sp.weight) * (double)t[b * ns + s];
    }
    charge[b] = q;
  }
  if (counts && nbins) std::memcpy(counts, t.data(), t.size() * 8);
  return PIC_OK;
}

pic_status pic_get_counters(pic_ctx *c, int64_t *alive, int64_t *absorbed, int64_t *escaped) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  const Dims &L = c->L;
  std::vector<int64_t> t(L.nbins * L.ns), e(6 * L.ns);
  if (L.nbins) PIC_HIP(c, hipMemcpy(t.data(), c->tally, t.size() * 8, hipMemcpyDeviceToHost));
  PIC_HIP(c, hipMemcpy(e.data(), c->escaped, e.size() * 8, hipMemcpyDeviceToHost));
  int64_t inj[PIC_MAX_SPECIES] = {0, 0, 0, 0};
  if ((st = read_injected(c, inj)) != PIC_OK) return st;
  for (int s = 0; s < L.ns; ++s) {
    int64_t a = 0, es = 0;
    for (int64_t b = 0; b < L.nbins; ++b) a += t[b * L.ns + s];
    for (int f = 0; f < 6; ++f) es += e[f * L.ns + s];
    if (absorbed) absorbed[s] = a;
    if (alive) alive[s] = c->sp[s].loaded + inj[s] - a - es;
  }
  if (escaped) std::memcpy(escaped, e.data(), e.size() * 8);
  return PIC_OK;
}

namespace {

int64_t level_nodes(const MgLevel &L) { return L.nodes; }

MgLevel make_level(int nx, int ny, int nz) {
  MgLevel L{};
  L.n[0] = nx;
  L.n[1] = ny;
  L.n[2] = nz;
  L.sx = nx + 1;
  L.sy = (int64_t)(nx + 1) * (ny + 1);
  L.nodes = L.sy * (nz + 1);
  L.G = (int32_t)((L.nodes + kBlock - 1) / kBlock);  // one node per thread (no dot products)
  return L;
}

// Levels of the V-cycle: halve all three cell counts while the level has
// more than kCoarseNodes nodes and all are even; 0 unless that ends at two
// or more levels with at most kCoarseNodes nodes on the coarsest.
int32_t mg_plan(const Dims &D, MgLevel *lv) {
  lv[0] = make_level(D.nx, D.ny, D.nz);
  int32_t n = 1;
  while (level_nodes(lv[n - 1]) > kCoarseNodes && n < kMaxLevels) {
    const MgLevel &f = lv[n - 1];
    if ((f.n[0] | f.n[1] | f.n[2]) & 1) break;
    lv[n] = make_level(f.n[0] / 2, f.n[1] / 2, f.n[2] / 2);
    ++n;
  }
  return (n >= 2 && level_nodes(lv[n - 1]) <= kCoarseNodes) ? n : 0;
}

bool level_dir(const MgLevel &L, int mask, int i, int j, int k) {
  return ((mask & 1) && i == 0) || ((mask & 2) && i == L.n[0]) || ((mask & 4) && j == 0) ||
         ((mask & 8) && j == L.n[1]) || ((mask & 16) && k == 0) || ((mask & 32) && k == L.n[2]);
}

// The coarsest level's operator on its unknowns (non-Dirichlet nodes, in node
// order), inverted on the host: A = L L^T, W = L^-1, A^-1 = W^T W. Returns
// false if A is not positive definite (it always is with a Dirichlet face).
// Level set of the object (cell units of the PIC mesh); the kernels'
// field_psi_kernel evaluates the same expression.
double geo_psi(const FieldGeom &o, double x, double y, double z) {
  if (o.kind == PIC_OBJ_SPHERE) {
    const double dx = x - o.c[0], dy = y - o.c[1], dz = z - o.c[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz) - o.r;
  }
  const double dx = x - o.c[0], dy = y - o.c[1];
  const double r2 = dx * dx + dy * dy;
  const double ground = r2 < o.a2 ? o.zc - std::sqrt(o.rc2 - r2) : o.z_flat;
  return z - ground;
}

double link_eps(double a, double b, double ein, double eout) {
  const bool ia = a < 0.0, ib = b < 0.0;
  if (ia == ib) return ia ? ein : eout;
  const double t = a / (a - b);
  const double f = ia ? t : 1.0 - t;
  return (ein * eout) / (f * eout + (1.0 - f) * ein);
}

// Field geometry of the context's object in cell units.
FieldGeom field_geom(const pic_ctx *c) {
  const Geom g = geometry_of(c->cfg);
  FieldGeom o{};
  o.kind = c->cfg.object.kind;
  for (int d = 0; d < 3; ++d) o.c[d] = g.c[d];
  o.patches = c->cfg.object.patches;
  if (o.kind == PIC_OBJ_SPHERE) {
    o.r = c->cfg.object.radius / c->cfg.h;
    o.rs = std::sqrt(g.r2);
  } else if (o.kind == PIC_OBJ_CRATER) {
    const double a = c->cfg.object.rim_radius / c->cfg.h;
    o.z_flat = g.z_flat;
    o.a2 = a * a;
    o.zc = g.c[2];
    o.rc2 = g.r2;
  }
  return o;
}

bool coarse_inverse(const MgLevel &C, int mask, double s, const FieldGeom *obj, double ein,
                    double eout, std::vector<double> &inv, std::vector<int32_t> &umap) {
  std::vector<int64_t> pos(C.nodes, -1);
  umap.clear();
  for (int k = 0; k <= C.n[2]; ++k)
    for (int j = 0; j <= C.n[1]; ++j)
      for (int i = 0; i <= C.n[0]; ++i)
        if (!level_dir(C, mask, i, j, k)) {
          const int64_t q = i + C.sx * j + C.sy * k;
          pos[q] = (int64_t)umap.size();
          umap.push_back((int32_t)q);
        }
  const int64_t m = (int64_t)umap.size();
  std::vector<double> A(m * m, 0.0), W(m * m, 0.0);
  auto cw = [&](int a, int n) { return (a == 0 || a == n) ? 0.5 : 1.0; };
  for (int64_t u = 0; u < m; ++u) {
    const int64_t q = umap[u];
    const int i = (int)(q % C.sx), j = (int)((q / C.sx) % (C.n[1] + 1)), k = (int)(q / C.sy);
    const double wx = cw(j, C.n[1]) * cw(k, C.n[2]), wy = cw(i, C.n[0]) * cw(k, C.n[2]),
                 wz = cw(i, C.n[0]) * cw(j, C.n[1]);
    const struct { bool ok; int64_t nb; double w; } links[6] = {
        {i > 0, q - 1, wx},         {i < C.n[0], q + 1, wx},    {j > 0, q - C.sx, wy},
        {j < C.n[1], q + C.sx, wy}, {k > 0, q - C.sy, wz},      {k < C.n[2], q + C.sy, wz}};
    for (const auto &L : links) {
      if (!L.ok) continue;
      double cf = s * L.w;
      if (obj) {  // series permittivity of the link, lower-index end first
        const int64_t lo = std::min(q, L.nb), hi = std::max(q, L.nb);
        auto psi = [&](int64_t n) {
          const int a = (int)(n % C.sx), b = (int)((n / C.sx) % (C.n[1] + 1)),
                    cc = (int)(n / C.sy);
          return geo_psi(*obj, C.scale * a, C.scale * b, C.scale * cc);
        };
        cf = link_eps(psi(lo), psi(hi), ein, eout) * L.w * C.ih2;
      }
      A[u * m + u] += cf;
      if (pos[L.nb] >= 0) A[u * m + pos[L.nb]] -= cf;
    }
  }
  for (int64_t r = 0; r < m; ++r)  // Cholesky, lower factor in place
    for (int64_t c = 0; c <= r; ++c) {
      double v = A[r * m + c];
      for (int64_t t = 0; t < c; ++t) v -= A[r * m + t] * A[c * m + t];
      if (r == c) {
        if (!(v > 0.0)) return false;
        A[r * m + r] = std::sqrt(v);
      } else {
        A[r * m + c] = v / A[c * m + c];
      }
    }
  for (int64_t c = 0; c < m; ++c) {  // W = L^-1 (lower)
    W[c * m + c] = 1.0 / A[c * m + c];
    for (int64_t r = c + 1; r < m; ++r) {
      double v = 0.0;
      for (int64_t t = c; t < r; ++t) v += A[r * m + t] * W[t * m + c];
      W[r * m + c] = -v / A[r * m + r];
    }
  }
  inv.assign(m * m, 0.0);  // A^-1 = W^T W, by rows of W
  for (int64_t t = 0; t < m; ++t)
    for (int64_t a = 0; a <= t; ++a) {
      const double wa = W[t * m + a];
      for (int64_t b = a; b <= t; ++b) inv[a * m + b] += wa * W[t * m + b];
    }
  for (int64_t a = 0; a < m; ++a)
    for (int64_t b = 0; b < a; ++b) inv[a * m + b] = inv[b * m + a];
  return true;
}

}  // namespace

namespace {

// The immersed finite elements of the fine grid for the object as an
// interface (iface, eps inside ein) or not, eps outside eout: the reference
// links of interior nodes in P, and, when not yet made for these settings,
// the rows of the nodes that need one (box faces, vertices of cut
// tetrahedra) and the fine level's diagonal. P must carry the level set.
pic_status ife_setup(pic_ctx *c, FieldParams &P, bool iface, double ein, double eout) {
  const int64_t nodes = c->L.nodes;
  for (int par = 0; par < 2; ++par) {
    double rl[kIfeLinks];
    ife_reference_links(par, rl);
    double d = 0.0;
    for (int l = 0; l < kIfeLinks; ++l) {
      P.rl[par][l] = rl[l] * P.ih2;
      d = d + P.rl[par][l];
    }
    P.rld[par] = d;
  }
  if (c->ife_ready && c->ife_key_iface == (int32_t)iface && c->ife_key_in == ein &&
      c->ife_key_out == eout)
    return PIC_OK;
  if (!c->ife_srow) {
    void **const outs[3] = {(void **)&c->ife_srow, (void **)&c->ife_count,
                            (void **)&c->ife_diag};
    const int64_t bytes[3] = {nodes * 4, 256, nodes * 8};
    if (!dmalloc_all(c, 3, outs, bytes))
      return fail(c, PIC_E_NOMEM, "device memory allocation failed");
  }
  P.ife = 1;
  PIC_HIP(c, launch_fill(c->ife_count, 8, c->stream));
  PIC_HIP(c, launch_ife_mark(P, c->ife_srow, c->ife_count, c->stream));
  int32_t count = 0;
  PIC_HIP(c, hipMemcpyAsync(&count, c->ife_count, 4, hipMemcpyDeviceToHost, c->stream));
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  if (count > c->ife_rows_cap) {
    void *q = nullptr;
    const int64_t cap = (int64_t)count + count / 8 + 64;
    if (dmalloc(c, &q, cap * (kIfeLinks + 1) * 8) != hipSuccess)
      return fail(c, PIC_E_NOMEM, "device memory allocation failed");
    c->ife_rows = (double *)q;  // (a smaller earlier one stays with the context)
    c->ife_rows_cap = cap;
  }
  PIC_HIP(c, launch_fill(c->ife_count + 1, 4, c->stream));
  PIC_HIP(c, launch_ife_rows(P, c->ife_srow, c->ife_rows, c->ife_count + 1, c->ife_diag,
                             c->stream));
  c->ife_ready = true;
  c->ife_key_iface = iface;
  c->ife_key_in = ein;
  c->ife_key_out = eout;
  return PIC_OK;
}

}  // namespace

pic_status pic_get_field_levels(pic_ctx *c, int32_t *levels) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!levels) return fail(c, PIC_E_INVALID, "levels must not be NULL");
  if (!c->solved) return fail(c, PIC_E_STATE, "no field solve yet");
  *levels = c->field_levels;
  return PIC_OK;
}

pic_status pic_solve_field(pic_ctx *c, const pic_field *fs, int32_t *iterations,
                           double *rel_residual) {
  const Range range("pic_solve_field");
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!fs) return fail(c, PIC_E_INVALID, "field settings must not be NULL");
  if ((fs->dirichlet & 63) == 0 || (fs->dirichlet & ~63))
    return fail(c, PIC_E_INVALID, "dirichlet: bits 0..5, at least one face");
  if (!(fs->eps > 0) || !is_finite(fs->eps)) return fail(c, PIC_E_INVALID, "eps must be > 0");
  if (!(fs->tol > 0) || !is_finite(fs->tol)) return fail(c, PIC_E_INVALID, "tol must be > 0");
  if (fs->max_iter < 0) return fail(c, PIC_E_INVALID, "max_iter must be >= 0");
  if (fs->preconditioner != PIC_PRECOND_MULTIGRID && fs->preconditioner != PIC_PRECOND_JACOBI)
    return fail(c, PIC_E_INVALID, "preconditioner: PIC_PRECOND_MULTIGRID or PIC_PRECOND_JACOBI");
  for (int f = 0; f < 6; ++f)
    if (!is_finite(fs->value[f])) return fail(c, PIC_E_INVALID, "face values must be finite");
  if (!(fs->eps_object >= 0) || !is_finite(fs->eps_object))
    return fail(c, PIC_E_INVALID, "eps_object must be >= 0 (0: no interface)");
  if (fs->surface_charge != 0 && fs->surface_charge != 1)
    return fail(c, PIC_E_INVALID, "surface_charge must be 0 or 1");
  if (fs->op != PIC_FIELD_FV && fs->op != PIC_FIELD_IFE)
    return fail(c, PIC_E_INVALID, "op: PIC_FIELD_FV or PIC_FIELD_IFE");
  if ((fs->eps_object > 0 || fs->surface_charge) && c->cfg.object.kind == PIC_OBJ_NONE)
    return fail(c, PIC_E_INVALID, "eps_object and surface_charge need an object");
  if (fs->surface_charge && c->cfg.object.kind == PIC_OBJ_SPHERE && c->cfg.object.patches < 1)
    return fail(c, PIC_E_INVALID, "surface_charge on a sphere needs surface patches");
  if (!c->deposited) return fail(c, PIC_E_STATE, "no deposit yet (call pic_step first)");
  const Dims &L = c->L;
  const int64_t nodes = L.nodes;
  const int32_t G = field_groups(nodes);
  if (!c->fx) {
    void *q = nullptr;
    if (!c->fctrl_host) {
      if (hipHostMalloc(&q, sizeof(FieldCtrl), hipHostMallocDefault) != hipSuccess)
        return fail(c, PIC_E_NOMEM, "hipHostMalloc failed");
      c->fctrl_host = (FieldCtrl *)q;
    }
    void **const outs[7] = {(void **)&c->fx,    (void **)&c->fr, (void **)&c->fz,
                            (void **)&c->fp,    (void **)&c->fAp, (void **)&c->fpart,
                            (void **)&c->fctrl};
    const int64_t bytes[7] = {nodes * 8, nodes * 8, nodes * 8, nodes * 8, nodes * 8,
                              6 * kFieldGroups * 8, (int64_t)sizeof(FieldCtrl)};
    if (!dmalloc_all(c, 7, outs, bytes))
      return fail(c, PIC_E_NOMEM, "device memory allocation failed");
    PIC_HIP(c, launch_fill(c->fx, nodes * 8, c->stream));
  }
  // multigrid plan (once): level 0 is the PIC mesh; levels >= 2 when it coarsens
  if (c->mg_levels < 0) {
    MgLevel lv[kMaxLevels];
    const int32_t n = mg_plan(L, lv);
    for (int l = 0; l < std::max(n, 1); ++l) {
      lv[l].scale = (double)(1 << l);
      const double hl = c->cfg.h * lv[l].scale;
      lv[l].ih2 = 1.0 / (hl * hl);
      c->mg[l] = lv[l];
    }
    c->mg_levels = n;
  }
  const bool use_mg = fs->preconditioner == PIC_PRECOND_MULTIGRID && c->mg_levels >= 2;
  const int32_t levels = use_mg ? c->mg_levels : 0;
  const int32_t nl = std::max(levels, 1);  // grids the solve uses
  if (use_mg && !c->mg_bufs) {
    std::vector<void **> outs;
    std::vector<int64_t> bytes;
    for (int l = 0; l < levels; ++l) {
      MgLevel &lv = c->mg[l];
      double **bufs[4] = {&lv.e, &lv.e2, &lv.res, &lv.rhs};
      for (int t = 0; t < 4; ++t) {
        if (l == 0 && (t == 0 || t == 3)) continue;  // level 0: e = z, rhs = r
        outs.push_back((void **)bufs[t]);
        bytes.push_back(lv.nodes * 8);
      }
    }
    const int64_t cn = c->mg[levels - 1].nodes;
    outs.push_back((void **)&c->mg_ainv);
    bytes.push_back(cn * cn * 8);
    outs.push_back((void **)&c->mg_umap);
    bytes.push_back(cn * 4);
    if (!dmalloc_all(c, (int)outs.size(), outs.data(), bytes.data()))
      return fail(c, PIC_E_NOMEM, "device memory allocation failed");
    c->mg_bufs = true;
  }
  const bool iface = fs->eps_object > 0;
  const FieldGeom geo = field_geom(c);
  if (iface) {
    for (int l = 0; l < nl; ++l) {
      if (c->mg[l].psi) continue;
      void **const outs[3] = {(void **)&c->mg[l].psi, (void **)&c->mg[l].diag,
                              (void **)&c->mg[l].side};
      const int64_t b = c->mg[l].nodes * 8;
      const int64_t bytes[3] = {b, b, c->mg[l].nodes};
      if (!dmalloc_all(c, 3, outs, bytes))
        return fail(c, PIC_E_NOMEM, "device memory allocation failed");
    }
  }
  if (levels >= 2) {
    const double eobj = iface ? fs->eps_object : 0.0;
    if (c->mg_mask != fs->dirichlet || c->mg_eps != fs->eps || c->mg_eps_obj != eobj) {
      const MgLevel &C = c->mg[levels - 1];
      const double hc = c->cfg.h * C.scale;
      std::vector<double> inv;
      std::vector<int32_t> umap;
      if (!coarse_inverse(C, fs->dirichlet, fs->eps / (hc * hc), iface ? &geo : nullptr,
                          fs->eps_object, fs->eps, inv, umap))
        return fail(c, PIC_E_DEVICE, "coarsest multigrid operator is not positive definite");
      c->mg_m = (int32_t)umap.size();
      if (c->mg_m > 0) {
        PIC_HIP(c, hipMemcpyAsync(c->mg_ainv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice,
                                  c->stream));
        PIC_HIP(c, hipMemcpyAsync(c->mg_umap, umap.data(), umap.size() * 4,
                                  hipMemcpyHostToDevice, c->stream));
        PIC_HIP(c, hipStreamSynchronize(c->stream));
      }
      c->mg_mask = fs->dirichlet;
      c->mg_eps = fs->eps;
      c->mg_eps_obj = eobj;
    }
  }
  FieldParams P{};
  P.rho = c->rho;
  P.x = c->fx;
  P.r = c->fr;
  P.z = c->fz;
  P.p = c->fp;
  P.Ap = c->fAp;
  P.part = c->fpart;
  P.ctrl = c->fctrl;
  P.E = c->E;
  P.n[0] = L.nx;
  P.n[1] = L.ny;
  P.n[2] = L.nz;
  P.sx = L.nx + 1;
  P.sy = (int64_t)(L.nx + 1) * (L.ny + 1);
  P.nodes = nodes;
  P.h = c->cfg.h;
  P.eps = fs->eps;
  P.s = fs->eps / (c->cfg.h * c->cfg.h);
  P.mask = fs->dirichlet;
  for (int f = 0; f < 6; ++f) P.g[f] = fs->value[f];
  P.tol = fs->tol;
  P.max_iter = fs->max_iter;
  P.G = G;
  P.levels = levels;
  for (int l = 0; l < nl; ++l) {
    P.lv[l] = c->mg[l];
    P.lv[l].mask = fs->dirichlet;
    const double hl = c->cfg.h * c->mg[l].scale;
    P.lv[l].s = fs->eps / (hl * hl);
  }
  P.lv[0].e = c->fz;
  P.lv[0].rhs = c->fr;
  if (levels >= 2) {
    P.ainv = c->mg_ainv;
    P.umap = c->mg_umap;
    P.m = c->mg_m;
  }
  P.iface = iface ? 1 : 0;
  P.e_in = fs->eps_object;
  P.e_out = fs->eps;
  P.geo = geo;
  P.psi = c->mg[0].psi;
  P.diag = c->mg[0].diag;
  P.side = c->mg[0].side;
  P.ih2 = c->mg[0].ih2;
  const int pe = prof_begin(c, 4);
  if (iface) {  // level sets once, diagonals when the permittivities change
    for (int l = c->if_psi_levels; l < nl; ++l) PIC_HIP(c, launch_field_psi(P, l, c->stream));
    c->if_psi_levels = std::max(c->if_psi_levels, nl);
    if (c->if_eps_in != fs->eps_object || c->if_eps_out != fs->eps) c->if_diag_levels = 0;
    for (int l = c->if_diag_levels; l < nl; ++l) PIC_HIP(c, launch_field_diag(P, l, c->stream));
    c->if_diag_levels = std::max(c->if_diag_levels, nl);
    c->if_eps_in = fs->eps_object;
    c->if_eps_out = fs->eps;
  }
  if (fs->op == PIC_FIELD_IFE) {
    pic_status st = ife_setup(c, P, iface, fs->eps_object, fs->eps);
    if (st != PIC_OK) return st;
    P.ife = 1;
    P.srow = c->ife_srow;
    P.rows = c->ife_rows;
    P.diag = c->ife_diag;
    P.lv[0].diag = c->ife_diag;
  }
  if (fs->surface_charge) {
    if (!c->rho_surf) {
      void *q = nullptr;
      if (dmalloc(c, &q, nodes * 8) != hipSuccess)
        return fail(c, PIC_E_NOMEM, "device memory allocation failed");
      c->rho_surf = (int64_t *)q;
    }
    PIC_HIP(c, launch_fill(c->rho_surf, nodes * 8, c->stream));
    SurfParams S{};
    S.tally = c->tally;
    for (int sp = 0; sp < L.ns; ++sp) S.chg[sp] = c->cfg.species[sp].q * c->cfg.species[sp].weight;
    S.ns = L.ns;
    S.nbins = L.nbins;
    S.n[0] = L.nx;
    S.n[1] = L.ny;
    S.n[2] = L.nz;
    S.sx = P.sx;
    S.sy = P.sy;
    S.geo = geo;
    S.rho_surf = c->rho_surf;
    S.err = c->err;
    PIC_HIP(c, launch_surface_rho(S, c->stream));
    P.rho_surf = c->rho_surf;
  }
  PIC_HIP(c, launch_field_init(c->cfg.deposit, P, c->stream));
  if (levels >= 2) PIC_HIP(c, launch_field_mg_start(P, c->stream));
  // iterations in chunks; the kernels themselves stop at convergence or
  // max_iter, the host only stops enqueueing (a multigrid iteration is some
  // 6 launches per level, so it checks more often)
  const int kChunkIters = levels >= 2 ? 2 : 16;
  for (int it = 1; it <= fs->max_iter; it += kChunkIters) {
    for (int k = it; k < it + kChunkIters && k <= fs->max_iter; ++k)
      PIC_HIP(c, launch_field_iter(P, (k - 1) & 1, c->stream));
    PIC_HIP(c, hipMemcpyAsync(c->fctrl_host, c->fctrl, sizeof(FieldCtrl), hipMemcpyDeviceToHost,
                              c->stream));
    PIC_HIP(c, hipStreamSynchronize(c->stream));
    if (c->fctrl_host->converged) break;
  }
  PIC_HIP(c, launch_field_E(c->cfg.repr, P, c->stream));
  prof_end(c, pe);
  PIC_HIP(c, hipMemcpyAsync(c->fctrl_host, c->fctrl, sizeof(FieldCtrl), hipMemcpyDeviceToHost,
                            c->stream));
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  const FieldCtrl f = *c->fctrl_host;
  if (fs->surface_charge) {
    const pic_status st = sync_and_check(c);
    if (st != PIC_OK) return st;
  }
  if (c->prof) c->acc.field_iterations += f.iters;
  if (iterations) *iterations = f.iters;
  if (rel_residual) *rel_residual = f.bb > 0 ? std::sqrt(f.rr) / std::sqrt(f.bb) : 0.0;
  c->E_set = true;
  c->solved = true;
  c->field_levels = levels;
  return PIC_OK;
}

pic_status pic_get_phi(pic_ctx *c, double *phi) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!phi) return fail(c, PIC_E_INVALID, "phi must not be NULL");
  if (!c->solved) return fail(c, PIC_E_STATE, "no field solve yet");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  PIC_HIP(c, hipMemcpy(phi, c->fx, c->L.nodes * 8, hipMemcpyDeviceToHost));
  return PIC_OK;
}

pic_status pic_set_injection(pic_ctx *c, const pic_injection *inj) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!inj || inj->faces == 0) {
    c->inj_on = false;
    return PIC_OK;
  }
  if (inj->faces & ~63) return fail(c, PIC_E_INVALID, "faces: only bits 0..5");
  if (inj->faces & c->cfg.reflect) return fail(c, PIC_E_INVALID, "a face cannot reflect and inject");
  if (c->cfg.object.kind == PIC_OBJ_CRATER && (inj->faces & 16))
    return fail(c, PIC_E_INVALID, "the crater's z- face is the terrain");
  for (int s = 0; s < c->L.ns; ++s) {
    if (!(inj->density[s] >= 0) || !is_finite(inj->density[s]) || !(inj->vth[s] >= 0) ||
        !is_finite(inj->vth[s]))
      return fail(c, PIC_E_INVALID, "density and vth must be finite and >= 0");
    double sp = 13.0 * inj->vth[s];
    for (int d = 0; d < 3; ++d) {
      if (!is_finite(inj->drift[s][d])) return fail(c, PIC_E_INVALID, "drift must be finite");
      sp += std::fabs(inj->drift[s][d]);
    }
    if (!(c->cfg.dt * sp / c->cfg.h <= 1048576.0))
      return fail(c, PIC_E_INVALID, "ambient speeds move more than 2^20 cells per step");
    if (!(inj->density[s] * c->cfg.h * c->cfg.h * c->cfg.h <= 1048576.0))
      return fail(c, PIC_E_INVALID, "density above 2^20 particles per cell");
  }
  c->inj = *inj;
  c->inj_on = true;
  return PIC_OK;
}

pic_status pic_set_photoemission(pic_ctx *c, const pic_photoemission *pe) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!pe) {
    c->pe_on = false;
    return PIC_OK;
  }
  const pic_config &cfg = c->cfg;
  if (cfg.object.kind != PIC_OBJ_CRATER)
    return fail(c, PIC_E_INVALID, "photoemission needs the crater terrain");
  if (pe->species < 0 || pe->species >= c->L.ns)
    return fail(c, PIC_E_INVALID, "photoemission species out of range");
  if (!(cfg.species[pe->species].weight > 0))
    return fail(c, PIC_E_INVALID, "the photoelectron species needs a weight > 0");
  if (!(pe->flux >= 0) || !is_finite(pe->flux) || !(pe->vth >= 0) || !is_finite(pe->vth))
    return fail(c, PIC_E_INVALID, "flux and vth must be finite and >= 0");
  for (int d = 0; d < 3; ++d)
    if (!is_finite(pe->sun[d])) return fail(c, PIC_E_INVALID, "sun must be finite");
  if (!(pe->sun[2] > 0)) return fail(c, PIC_E_INVALID, "the Sun must be above the ground (sun[2] > 0)");
  if (!(cfg.dt * 13.0 * pe->vth / cfg.h <= 1048576.0))
    return fail(c, PIC_E_INVALID, "photoelectron speeds move more than 2^20 cells per step");
  PhotoParams P{};
  P.s = pe->species;
  P.seed = pe->seed;
  const double len =
      std::sqrt(pe->sun[0] * pe->sun[0] + pe->sun[1] * pe->sun[1] + pe->sun[2] * pe->sun[2]);
  for (int d = 0; d < 3; ++d) P.sun[d] = pe->sun[d] / len;
  P.rate = (pe->flux / cfg.species[pe->species].weight) * (cfg.h * cfg.h) * cfg.dt;
  P.vth = pe->vth / cfg.h;
  const double a = cfg.object.rim_radius / cfg.h, dep = cfg.object.depth / cfg.h;
  P.rc = (a * a + dep * dep) / (2.0 * dep);
  P.rc2 = P.rc * P.rc;
  P.a2 = a * a;
  P.z_flat = (cfg.object.z_flat - cfg.origin[2]) / cfg.h;
  P.zc = P.z_flat - dep + P.rc;
  P.cx = (cfg.object.center[0] - cfg.origin[0]) / cfg.h;
  P.cy = (cfg.object.center[1] - cfg.origin[1]) / cfg.h;
  // slots per column: floor of the largest mean + 1 (the kernel's formulas);
  // the tiles the photoelectrons start in get room for several steps of them
  const Dims &D = c->L;
  std::vector<int32_t> inflow((size_t)D.ns * D.ntiles, 0);
  double most = 0.0;
  for (int64_t j = 0; j < c->L.ny; ++j)
    for (int64_t i = 0; i < c->L.nx; ++i) {
      const double dx = ((double)i + 0.5) - P.cx, dy = ((double)j + 0.5) - P.cy;
      const double r2 = dx * dx + dy * dy;
      const bool bowl = r2 < P.a2;
      double n[3] = {0.0, 0.0, 1.0}, zg = P.z_flat;
      if (bowl) {
        zg = P.zc - std::sqrt(P.rc2 - r2);
        n[0] = -dx / P.rc;
        n[1] = -dy / P.rc;
        n[2] = (P.zc - zg) / P.rc;
      }
      const double I = (P.sun[0] * n[0] + P.sun[1] * n[1]) + P.sun[2] * n[2];
      const bool lit = I > 0.0 && (!bowl || zg + (2.0 * P.rc * I) * P.sun[2] >= P.z_flat);
      if (!lit) continue;
      const double mean = (P.rate * I) / n[2];
      most = std::max(most, mean);
      if (!(mean <= 1048576.0)) continue;
      const int64_t kz = std::min<int64_t>(std::max<int64_t>((int64_t)std::floor(zg), 0), D.nz - 1);
      const int64_t t = (i / kTile) + D.ntx * ((j / kTile) + D.nty * (kz / kTile));
      int32_t &v = inflow[(size_t)pe->species * D.ntiles + t];
      v = (int32_t)std::min<int64_t>((int64_t)v + (int64_t)std::floor(mean) + 1, 1 << 20);
    }
  if (!(most <= 1048576.0))
    return fail(c, PIC_E_INVALID, "more than 2^20 photoelectrons per column per step");
  P.gmax = (int64_t)std::floor(most) + 1;
  if ((int64_t)c->L.nx * c->L.ny * P.gmax > (int64_t(1) << 36))
    return fail(c, PIC_E_INVALID, "photoemission: more than 2^36 slots per step");
  if (!c->inflow) {
    void *q = nullptr;
    if (dmalloc(c, &q, (int64_t)inflow.size() * 4) != hipSuccess)
      return fail(c, PIC_E_NOMEM, "device memory allocation failed");
    c->inflow = (int32_t *)q;
  }
  PIC_HIP(c, hipStreamSynchronize(c->stream));  // no re-bucketing reads the old map
  PIC_HIP(c, hipMemcpy(c->inflow, inflow.data(), inflow.size() * 4, hipMemcpyHostToDevice));
  c->pe = P;
  c->pe_on = true;
  return PIC_OK;
}

pic_status pic_get_injected(pic_ctx *c, int64_t *injected) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!injected) return fail(c, PIC_E_INVALID, "injected must not be NULL");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  return read_injected(c, injected);
}

pic_status pic_set_step_index(pic_ctx *c, int64_t step) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (step < 0 || step > 0x7fffffffLL) return fail(c, PIC_E_INVALID, "step must be in 0..2^31-1");
  c->step_index = step;
  return PIC_OK;
}

pic_status pic_get_particles(pic_ctx *c, int32_t species, int64_t cap, int64_t *n_out, double *x,
                             double *y, double *z, double *vx, double *vy, double *vz,
                             int64_t *ids) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (species < 0 || species >= c->L.ns) return fail(c, PIC_E_INVALID, "species out of range");
  if (!n_out) return fail(c, PIC_E_INVALID, "n_out must not be NULL");
  pic_ctx::Species &S = c->sp[species];
  if (ids && !S.ids) return fail(c, PIC_E_STATE, "no ids were loaded for this species");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  std::vector<std::pair<int64_t, int64_t>> rg;
  std::vector<int32_t> rt;
  if ((st = species_ranges(c, species, rg, &rt)) != PIC_OK) return st;
  int64_t total = 0;
  for (auto &r : rg) total += r.second;
  *n_out = total;
  if (total > cap) return fail(c, PIC_E_INVALID, "cap is smaller than the alive count");
  if (total > 0 && (!x || !y || !z || !vx || !vy || !vz))
    return fail(c, PIC_E_INVALID, "output arrays must not be NULL");
  const int repr = c->cfg.repr;
  const int64_t e = elem_bytes(repr);
  const PBuf &B = S.buf[c->cur];
  const pic_config &cf = c->cfg;
  double *X[3] = {x, y, z}, *V[3] = {vx, vy, vz};
  std::vector<char> pos, vel;
  std::vector<int32_t> cell;
  std::vector<int64_t> id;
  int64_t k = 0;
  for (size_t ri = 0; ri < rg.size(); ++ri) {
    const int64_t o = rg[ri].first, n = rg[ri].second;
    const int32_t t = rt[ri];
    pos.resize(3 * n * e);
    vel.resize(3 * n * e);
    for (int d = 0; d < 3; ++d) {
      PIC_HIP(c, hipMemcpy(pos.data() + d * n * e, (char *)B.pos[d] + o * e, n * e,
                           hipMemcpyDeviceToHost));
      PIC_HIP(c, hipMemcpy(vel.data() + d * n * e, (char *)B.vel[d] + o * e, n * e,
                           hipMemcpyDeviceToHost));
    }
    if (repr == PIC_REPR_FP32_CELL && t < 0) {  // a region implies its tile
      cell.resize(n);
      PIC_HIP(c, hipMemcpy(cell.data(), B.cell + o, n * 4, hipMemcpyDeviceToHost));
    }
    if (ids) {
      id.resize(n);
      PIC_HIP(c, hipMemcpy(id.data(), B.ids + o, n * 8, hipMemcpyDeviceToHost));
    }
    for (int64_t p = 0; p < n; ++p, ++k) {
      double g[3], u[3];
      if (repr == PIC_REPR_FP32_CELL) {
        const float *po = (const float *)pos.data();
        int ci[3];
        if (t >= 0) {
          const int tc[3] = {t % c->L.ntx, (t / c->L.ntx) % c->L.nty, t / (c->L.ntx * c->L.nty)};
          for (int d = 0; d < 3; ++d) ci[d] = (tc[d] << kTileShift) + off_sub(po[d * n + p]);
        } else {
          ci[0] = cell[p] & kMaxDim;
          ci[1] = (cell[p] >> kCellBits) & kMaxDim;
          ci[2] = cell[p] >> (2 * kCellBits);
        }
        for (int d = 0; d < 3; ++d) {
          g[d] = (double)ci[d] + (double)off_value(po[d * n + p]);
          u[d] = (double)((float *)vel.data())[d * n + p];
        }
      } else if (repr == PIC_REPR_FP32_ABS) {
        for (int d = 0; d < 3; ++d) {
          g[d] = (double)((float *)pos.data())[d * n + p];
          u[d] = (double)((float *)vel.data())[d * n + p];
        }
      } else {
        for (int d = 0; d < 3; ++d) {
          g[d] = ((double *)pos.data())[d * n + p];
          u[d] = ((double *)vel.data())[d * n + p];
        }
      }
      for (int d = 0; d < 3; ++d) {
        X[d][k] = cf.origin[d] + g[d] * cf.h;
        V[d][k] = u[d] * cf.h;
      }
      if (ids) ids[k] = id[p];
    }
  }
  return PIC_OK;
}

pic_status pic_get_particles_by_id(pic_ctx *c, int32_t species, int64_t n,
                                   const int64_t *ids_sorted, int32_t *found, double *x,
                                   double *y, double *z, double *vx, double *vy, double *vz) {
  pic_status st = by_id_prepare(c, species, n, ids_sorted, found, x, y, z, vx, vy, vz);
  if (st != PIC_OK || n == 0) return st;
  pic_ctx::Species &S = c->sp[species];
  // staging of the id list and of the results, for this call only
  void *d_ids = dev_alloc(c->cfg, n * 8), *d_found = dev_alloc(c->cfg, n * 4),
       *d_out = dev_alloc(c->cfg, n * 6 * 8);
  auto cleanup = [&]() {
    dev_free(c->cfg, d_ids);
    dev_free(c->cfg, d_found);
    dev_free(c->cfg, d_out);
  };
  if (!d_ids || !d_found || !d_out) {
    cleanup();
    return fail(c, PIC_E_NOMEM, "no device memory for the id search");
  }
  hipError_t e = hipMemcpy(d_ids, ids_sorted, n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_fill(d_found, n * 4, c->stream);
  if (e == hipSuccess)
    e = launch_find_ids(c->cfg.repr, S.buf[c->cur], bins_of(c), c->cur, species, c->L.ntiles,
                        c->L.ntx, c->L.nty, (const int64_t *)d_ids, n, (int32_t *)d_found, (double *)d_out,
                        PhysUnits{}, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  std::vector<double> out(n * 6);
  if (e == hipSuccess) e = hipMemcpy(found, d_found, n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(out.data(), d_out, n * 6 * 8, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return hip_fail(c, e, "pic_get_particles_by_id");
  const pic_config &cf = c->cfg;
  double *X[3] = {x, y, z}, *V[3] = {vx, vy, vz};
  for (int64_t k = 0; k < n; ++k) {
    if (!found[k]) continue;
    for (int d = 0; d < 3; ++d) {
      X[d][k] = cf.origin[d] + out[d * n + k] * cf.h;
      V[d][k] = out[(3 + d) * n + k] * cf.h;
    }
  }
  return PIC_OK;
}

pic_status pic_get_particles_by_id_noalloc(pic_ctx *c, int32_t species, int64_t n,
                                           const int64_t *ids_sorted, int32_t *found, double *x,
                                           double *y, double *z, double *vx, double *vy,
                                           double *vz) {
  if (c && n > PIC_NOALLOC_MAX_IDS)
    return fail(c, PIC_E_INVALID, "n must be <= PIC_NOALLOC_MAX_IDS");
  pic_status st = by_id_prepare(c, species, n, ids_sorted, found, x, y, z, vx, vy, vz);
  if (st != PIC_OK || n == 0) return st;
  if (!c->scratch) return fail(c, PIC_E_DEVICE, "no scratch area on this device");
  // staged in the device's scratch area (c->scratch: its address on this
  // device): the ids, the caller's output arrays (entries of ids not found
  // stay as they are), the found flags cleared by a kernel; the lookup writes
  // physical units, so the results go back into the caller's arrays directly
  char *base = (char *)c->scratch;
  int64_t *d_ids = (int64_t *)(base + kNoAllocIdsOff);
  double *d_out = (double *)(base + kNoAllocOutOff);
  int32_t *d_found = (int32_t *)(base + kNoAllocFoundOff);
  double *O[6] = {x, y, z, vx, vy, vz};
  const hipStream_t s = c->stream;
  PIC_HIP(c, hipMemcpyAsync(d_ids, ids_sorted, n * 8, hipMemcpyHostToDevice, s));
  for (int d = 0; d < 6; ++d)
    PIC_HIP(c, hipMemcpyAsync(d_out + d * n, O[d], n * 8, hipMemcpyHostToDevice, s));
  PIC_HIP(c, launch_fill(d_found, n * 4, s));
  PhysUnits ph{};
  ph.on = true;
  for (int d = 0; d < 3; ++d) ph.origin[d] = c->cfg.origin[d];
  ph.h = c->cfg.h;
  PIC_HIP(c, launch_find_ids(c->cfg.repr, c->sp[species].buf[c->cur], bins_of(c), c->cur, species,
                             c->L.ntiles, c->L.ntx, c->L.nty, d_ids, n, d_found, d_out, ph,
                             s));
  PIC_HIP(c, hipMemcpyAsync(found, d_found, n * 4, hipMemcpyDeviceToHost, s));
  for (int d = 0; d < 6; ++d)
    PIC_HIP(c, hipMemcpyAsync(O[d], d_out + d * n, n * 8, hipMemcpyDeviceToHost, s));
  PIC_HIP(c, hipStreamSynchronize(s));
  return PIC_OK;
}

pic_status pic_profile_enable(pic_ctx *c, int32_t on) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  PIC_HIP(c, hipStreamSynchronize(c->stream));
  if (c->prof) prof_collect(c);
  c->prof = on != 0;
  c->acc = pic_profile{};
  PIC_HIP(c, hipMemset(c->stats, 0, 64));
  return PIC_OK;
}

pic_status pic_profile_read(pic_ctx *c, pic_profile *out) {
  if (const pic_status s0 = check_ctx(c)) return s0;
  if (!out) return fail(c, PIC_E_INVALID, "out must not be NULL");
  pic_status st = sync_and_check(c);
  if (st != PIC_OK) return st;
  int64_t ps = 0;
  PIC_HIP(c, hipMemcpy(&ps, c->stats, 8, hipMemcpyDeviceToHost));
  *out = c->acc;
  out->particle_steps = ps;
  return PIC_OK;
}

int64_t pic_footprint_bytes(const pic_config *cfg) {
  if (validate_config(cfg)) return -1;
  return footprint(*cfg);
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {
// Persistent workgroups of a batched step (enough to fill 256 CUs at the step
// kernel's occupancy; the ones that find no work exit at once).
constexpr int32_t kBatchGrid = 2048;
}  // namespace

struct pic_batch {
  pic_batch_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device: the slot table (ordered by quota), its prefix, and a control block
  // [istep, work, totals[M], flags[max_slots]]
  StepParams *d_slots = nullptr;
  int32_t *d_prefix = nullptr;
  int32_t *d_ctrl = nullptr;
  // pinned host mirrors (written only while no copy from them is pending)
  StepParams *h_slots = nullptr;
  int32_t *h_prefix = nullptr;
  int32_t *h_ctrl = nullptr;
  std::vector<pic_ctx *> ctx;       // per slot, nullptr = free
  std::vector<int64_t> remaining;   // per slot
  std::vector<int64_t> bytes;       // per slot footprint
  std::vector<int64_t> work;        // per slot: particles at attach (the cost of one step)
  std::vector<double> weight;       // per slot: share of a run's particle-steps (default 1)
  std::vector<int32_t> want_sort;   // per slot: bit s: species s ran out of spare room
  std::vector<int32_t> order;       // table entry -> slot of the run in flight
  std::vector<int32_t> quota;       // per slot: steps of the run in flight
  bool inflight = false;            // launched, not yet waited for
  bool single = false;              // the run in flight steps one context alone
  int64_t used = 0;
  std::vector<hipGraphExec_t> exec; // [2 j + r]: a run of min(2^j, M) steps; r: with the
                                    // code of reflecting faces (some slot reflects)
  std::string msg = "no error";
};

namespace {

thread_local std::string g_batch_error = "no error";

pic_status bfail(pic_batch *b, pic_status st, const std::string &m) {
  if (b) b->msg = m;
  else g_batch_error = m;
  return st;
}

pic_status bhip(pic_batch *b, hipError_t e, const char *where) {
  return bfail(b, PIC_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define PIC_BHIP(b, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return bhip(b, e_, #call);       \
  } while (0)

int32_t run_length(const pic_batch *b, int j) {
  return std::min<int32_t>(1 << j, b->cfg.steps_per_run);
}

BatchTable table_of(const pic_batch *b) {
  BatchTable T{};
  T.slots = b->d_slots;
  T.prefix = b->d_prefix;
  T.istep = b->d_ctrl;
  T.work = b->d_ctrl + 1;
  T.totals = b->d_ctrl + 2;
  T.nslots = b->cfg.max_slots;
  return T;
}

// The graph of a run of run_length(j) batched steps followed by the read-back
// of the slots' re-bucketing requests (captured on first use); refl: the step
// kernel with the code of reflecting faces.
pic_status ensure_graph(pic_batch *b, int j, bool refl) {
  hipGraphExec_t &ex = b->exec[2 * j + (refl ? 1 : 0)];
  if (ex) return PIC_OK;
  const BatchTable T = table_of(b);
  int32_t *flags_out = b->d_ctrl + 2 + b->cfg.steps_per_run;
  hipGraph_t graph = nullptr;
  PIC_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int k = 0; k < run_length(b, j) && le == hipSuccess; ++k)
    le = launch_batch_step(b->cfg.repr, b->cfg.deposit, refl, T, kBatchGrid, b->stream);
  if (le == hipSuccess) le = launch_batch_flags(T, flags_out, b->stream);
  hipError_t ce = hipStreamEndCapture(b->stream, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return bhip(b, le, "batched step launch");
  }
  if (ce != hipSuccess) return bhip(b, ce, "hipStreamEndCapture");
  hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    ex = nullptr;
    return bhip(b, ie, "hipGraphInstantiate");
  }
  return PIC_OK;
}

void free_batch(pic_batch *b) {
  for (hipGraphExec_t &e : b->exec)
    if (e) (void)hipGraphExecDestroy(e);
  if (b->d_slots) (void)hipFree(b->d_slots);
  if (b->d_prefix) (void)hipFree(b->d_prefix);
  if (b->d_ctrl) (void)hipFree(b->d_ctrl);
  if (b->h_slots) (void)hipHostFree(b->h_slots);
  if (b->h_prefix) (void)hipHostFree(b->h_prefix);
  if (b->h_ctrl) (void)hipHostFree(b->h_ctrl);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // namespace

extern "C" {

const char *pic_batch_last_error(const pic_batch *b) {
  return b ? b->msg.c_str() : g_batch_error.c_str();
}

int64_t pic_batch_used_bytes(const pic_batch *b) { return b ? b->used : 0; }

int64_t pic_batch_remaining(const pic_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->cfg.max_slots || !b->ctx[slot]) return -1;
  return b->remaining[slot];
}

pic_status pic_batch_create(const pic_batch_config *cfg, pic_batch **out) {
  if (!out) return bfail(nullptr, PIC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return bfail(nullptr, PIC_E_INVALID, "config is NULL");
  if (cfg->max_slots < 1 || cfg->max_slots > 1024)
    return bfail(nullptr, PIC_E_INVALID, "max_slots must be in 1..1024");
  if (cfg->repr < 0 || cfg->repr > 2 || cfg->deposit < 0 || cfg->deposit > 2)
    return bfail(nullptr, PIC_E_INVALID, "repr / deposit out of range");
  if (cfg->steps_per_run < 1 || cfg->steps_per_run > 4096)
    return bfail(nullptr, PIC_E_INVALID, "steps_per_run must be in 1..4096");
  if (cfg->hbm_budget_bytes <= 0) return bfail(nullptr, PIC_E_INVALID, "hbm_budget_bytes must be > 0");
  if (cfg->particle_steps_per_run < 0)
    return bfail(nullptr, PIC_E_INVALID, "particle_steps_per_run must be >= 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return bfail(nullptr, PIC_E_DEVICE, "no HIP device available");
  pic_batch *b = new pic_batch();
  b->cfg = *cfg;
  auto bail = [&](pic_status st, const std::string &m) {
    free_batch(b);
    return bfail(nullptr, st, m);
  };
  if (cfg->stream) {
    b->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(PIC_E_DEVICE, "hipStreamCreate failed");
    b->own_stream = true;
  }
  const int n = cfg->max_slots, M = cfg->steps_per_run;
  const size_t ctrl = sizeof(int32_t) * (2 + M + n);
  if (hipMalloc(&b->d_slots, sizeof(StepParams) * n) != hipSuccess ||
      hipMalloc(&b->d_prefix, sizeof(int32_t) * (n + 1)) != hipSuccess ||
      hipMalloc(&b->d_ctrl, ctrl) != hipSuccess)
    return bail(PIC_E_NOMEM, "device memory allocation failed");
  if (hipHostMalloc((void **)&b->h_slots, sizeof(StepParams) * n, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void **)&b->h_prefix, sizeof(int32_t) * (n + 1), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void **)&b->h_ctrl, ctrl, hipHostMallocDefault) != hipSuccess)
    return bail(PIC_E_NOMEM, "hipHostMalloc failed");
  for (int k = 0; k < n; ++k) b->h_slots[k] = StepParams{};
  std::memset(b->h_prefix, 0, sizeof(int32_t) * (n + 1));
  std::memset(b->h_ctrl, 0, ctrl);
  b->ctx.assign(n, nullptr);
  b->remaining.assign(n, 0);
  b->bytes.assign(n, 0);
  b->work.assign(n, 0);
  b->weight.assign(n, 1.0);
  b->want_sort.assign(n, 0);
  b->order.clear();
  b->quota.assign(n, 0);
  int nj = 1;
  while (run_length(b, nj - 1) < M) ++nj;
  b->exec.assign(2 * nj, nullptr);
  *out = b;
  return PIC_OK;
}

pic_status pic_batch_set_weight(pic_batch *b, int32_t slot, double weight) {
  if (!b) return PIC_E_INVALID;
  if (slot < 0 || slot >= b->cfg.max_slots || !b->ctx[slot])
    return bfail(b, PIC_E_INVALID, "no context in this slot");
  if (!(weight >= 0.0) || !(weight < 1e30))
    return bfail(b, PIC_E_INVALID, "weight must be in [0, 1e30)");
  b->weight[slot] = weight;
  return PIC_OK;
}

pic_status pic_batch_detach(pic_batch *b, int32_t slot) {
  if (!b) return PIC_E_INVALID;
  if (slot < 0 || slot >= b->cfg.max_slots || !b->ctx[slot])
    return bfail(b, PIC_E_INVALID, "no context in this slot");
  if (b->inflight) return bfail(b, PIC_E_STATE, "a run is in flight (pic_batch_wait first)");
  PIC_BHIP(b, hipStreamSynchronize(b->stream));
  pic_ctx *c = b->ctx[slot];
  c->batch = nullptr;
  b->ctx[slot] = nullptr;
  b->remaining[slot] = 0;
  b->used -= b->bytes[slot];
  b->bytes[slot] = 0;
  b->work[slot] = 0;
  b->weight[slot] = 1.0;
  b->want_sort[slot] = 0;
  return PIC_OK;
}

void pic_batch_destroy(pic_batch *b) {
  if (!b) return;
  (void)pic_batch_wait(b, nullptr, nullptr);
  for (int k = 0; k < b->cfg.max_slots; ++k)
    if (b->ctx[k]) (void)pic_batch_detach(b, k);
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
}

pic_status pic_batch_attach(pic_batch *b, pic_ctx *c, int64_t nsteps, int32_t *slot) {
  if (!b) return PIC_E_INVALID;
  if (!c || !slot) return bfail(b, PIC_E_INVALID, "ctx and slot must not be NULL");
  if (nsteps < 1) return bfail(b, PIC_E_INVALID, "nsteps must be >= 1");
  if (c->batch) return bfail(b, PIC_E_STATE, "the context is already attached");
  if (c->cfg.repr != b->cfg.repr || c->cfg.deposit != b->cfg.deposit)
    return bfail(b, PIC_E_INVALID, "repr / deposit differ from the batch's");
  if (!c->E_set) return bfail(b, PIC_E_STATE, "the context has no node field");
  if (c->inj_on || c->pe_on)
    return bfail(b, PIC_E_INVALID, "contexts that inject particles run alone (pic_step)");
  int free_slot = -1;
  for (int k = 0; k < b->cfg.max_slots && free_slot < 0; ++k)
    if (!b->ctx[k]) free_slot = k;
  if (free_slot < 0) return bfail(b, PIC_E_STATE, "no free slot");
  const int64_t fp = footprint(c->cfg);
  if (b->used + fp > b->cfg.hbm_budget_bytes)
    return bfail(b, PIC_E_NOMEM, "the footprint does not fit the remaining budget");
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return bfail(b, PIC_E_DEVICE, "context stream failed");
  if (!c->sorted) {
    if (do_sort(c, 0) != PIC_OK) return bfail(b, PIC_E_DEVICE, c->msg);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
      return bfail(b, PIC_E_DEVICE, "context stream failed");
  }
  int64_t n = 0;
  for (int s = 0; s < c->L.ns; ++s) n += c->sp[s].loaded;
  b->ctx[free_slot] = c;
  b->remaining[free_slot] = nsteps;
  b->bytes[free_slot] = fp;
  b->work[free_slot] = std::max<int64_t>(n, 1);
  b->weight[free_slot] = 1.0;
  b->want_sort[free_slot] = 0;
  b->used += fp;
  c->batch = b;
  *slot = free_slot;
  return PIC_OK;
}

pic_status pic_batch_launch(pic_batch *b) {
  const Range range("pic_batch_launch");
  if (!b) return PIC_E_INVALID;
  if (b->inflight) return bfail(b, PIC_E_STATE, "a run is in flight (pic_batch_wait first)");
  const int n = b->cfg.max_slots, M = b->cfg.steps_per_run;
  const int64_t P = b->cfg.particle_steps_per_run;
  // contexts of weight 0 are paused for this run, unless all are
  bool any_weight = false;
  for (int k = 0; k < n; ++k)
    if (b->ctx[k] && b->remaining[k] > 0 && b->weight[k] > 0.0) any_weight = true;
  // re-plan the tile regions of contexts whose spare room ran out
  std::vector<int32_t> &order = b->order;
  order.clear();
  for (int k = 0; k < n; ++k) {
    pic_ctx *c = b->ctx[k];
    if (!c || b->remaining[k] <= 0) continue;
    if (any_weight && !(b->weight[k] > 0.0)) continue;
    if (b->want_sort[k] || !c->sorted) {
      if (do_sort(c, b->want_sort[k]) != PIC_OK) return bfail(b, PIC_E_DEVICE, c->msg);
      PIC_BHIP(b, hipStreamSynchronize(c->stream));
      b->want_sort[k] = 0;
    }
    order.push_back(k);
  }
  const int S = (int)order.size();
  if (S == 0) return PIC_OK;
  // step quotas: M each, or a weighted share of P particle-steps
  double wsum = 0.0;
  for (int k : order) wsum += any_weight ? b->weight[k] : 1.0;
  for (int k : order) {
    int64_t qk = M;
    if (P > 0) {
      const double wk = any_weight ? b->weight[k] : 1.0;
      const double share = (double)P * (wk / wsum) / (double)b->work[k];
      qk = share >= (double)M ? M : std::max<int64_t>(1, (int64_t)share);
    }
    b->quota[k] = (int32_t)std::min<int64_t>(qk, b->remaining[k]);
  }
  if (S == 1) {
    // one context runs: its steps go through the single-context kernels, as
    // pic_step launches them (the same per-tile code, no persistent work
    // queue), then its overflow counts come back for the re-planning request
    const int k = order[0];
    pic_ctx *c = b->ctx[k];
    StepParams sp = step_params(c);
    for (int t = 0; t < b->quota[k]; ++t) {
      PIC_BHIP(b, launch_step_clear(c->rho, c->L.nodes * rho_elem(c->cfg.deposit),
                                    sp.bins.ovf[1 - sp.cur], c->L.ns, b->stream));
      PIC_BHIP(b, launch_step(c->cfg.repr, c->cfg.deposit, true, sp, b->stream));
      sp.cur = 1 - sp.cur;
    }
    PIC_BHIP(b, hipMemcpyAsync((void *)c->ovf_host, sp.bins.ovf[sp.cur],
                               sizeof(int32_t) * c->L.ns, hipMemcpyDeviceToHost, b->stream));
    b->single = true;
    b->inflight = true;
    return PIC_OK;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->quota[x] > b->quota[y]; });
  // the table: entry i holds slot order[i]; the work items of step t are
  // those of the entries with quota > t, a prefix of the table
  int32_t total = 0;
  for (int i = 0; i < n; ++i) {
    b->h_prefix[i] = total;
    if (i < S) {
      pic_ctx *c = b->ctx[order[i]];
      b->h_slots[i] = step_params(c);
      b->h_slots[i].remaining = b->quota[order[i]];
      total += c->L.ntiles + b->h_slots[i].ovf_groups;
    } else {
      b->h_slots[i] = StepParams{};
    }
  }
  b->h_prefix[n] = total;
  int32_t *totals = b->h_ctrl + 2;
  b->h_ctrl[0] = 0;
  b->h_ctrl[1] = 0;
  for (int t = 0, i = S; t < M; ++t) {
    while (i > 0 && b->quota[order[i - 1]] <= t) --i;
    totals[t] = b->h_prefix[i];
  }
  const int32_t len = b->quota[order[0]];
  int j = 0;
  while (run_length(b, j) < len) ++j;
  bool refl = false;
  for (int k : order) refl |= b->ctx[k]->cfg.reflect != 0;
  if (pic_status st = ensure_graph(b, j, refl)) return st;
  PIC_BHIP(b, hipMemcpyAsync(b->d_slots, b->h_slots, sizeof(StepParams) * n,
                             hipMemcpyHostToDevice, b->stream));
  PIC_BHIP(b, hipMemcpyAsync(b->d_prefix, b->h_prefix, sizeof(int32_t) * (n + 1),
                             hipMemcpyHostToDevice, b->stream));
  PIC_BHIP(b, hipMemcpyAsync(b->d_ctrl, b->h_ctrl, sizeof(int32_t) * (2 + M),
                             hipMemcpyHostToDevice, b->stream));
  PIC_BHIP(b, hipGraphLaunch(b->exec[2 * j + (refl ? 1 : 0)], b->stream));
  PIC_BHIP(b, hipMemcpyAsync(b->h_ctrl + 2 + M, b->d_ctrl + 2 + M, sizeof(int32_t) * S,
                             hipMemcpyDeviceToHost, b->stream));
  b->single = false;
  b->inflight = true;
  return PIC_OK;
}

pic_status pic_batch_wait(pic_batch *b, int32_t *n_done, int32_t *done_slots) {
  const Range range("pic_batch_wait");
  if (!b) return PIC_E_INVALID;
  if (n_done) *n_done = 0;
  if (!b->inflight) return PIC_OK;
  PIC_BHIP(b, hipStreamSynchronize(b->stream));
  b->inflight = false;
  const int M = b->cfg.steps_per_run;
  int32_t nd = 0;
  for (size_t i = 0; i < b->order.size(); ++i) {
    const int k = b->order[i];
    pic_ctx *c = b->ctx[k];
    const int32_t did = b->quota[k];
    if (did & 1) c->cur = 1 - c->cur;
    c->since_sort += did;
    b->remaining[k] -= did;
    if (b->single) {
      int32_t want = 0;
      for (int s = 0; s < c->L.ns; ++s)
        if (c->ovf_host[s] > 0) want |= 1 << s;
      b->want_sort[k] = want;
    } else {
      b->want_sort[k] = b->h_ctrl[2 + M + i];
    }
    if (b->remaining[k] == 0) {
      if (done_slots) done_slots[nd] = k;
      ++nd;
    }
  }
  b->order.clear();
  if (n_done) *n_done = nd;
  return PIC_OK;
}

pic_status pic_batch_run(pic_batch *b, int32_t *n_done, int32_t *done_slots) {
  if (n_done) *n_done = 0;
  if (pic_status st = pic_batch_launch(b)) return st;
  return pic_batch_wait(b, n_done, done_slots);
}

}  // extern "C"
