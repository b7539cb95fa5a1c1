// HIP kernels of the field solve on the PIC mesh for gfx950 (the boundary
// value problem of §2.1 by node-centred finite volumes or by immersed finite
// elements on five tetrahedra per cell, preconditioned conjugate gradients
// with a geometric multigrid V-cycle or Jacobi, the object as an interface
// with the collected charge as its surface source, eq. (2.2)-(2.5)), and
// E = -grad phi into the node field.
#include "pic_device.h"
#include "pic_ife.h"

namespace pic {
namespace {

// ------------------------------------------------------------------ field solve
//
// -div(eps grad phi) = rho on the nodes (node-centred finite volumes: the flux
// through the dual face of a link is eps w (phi_p - phi_q) h with w the
// product of the two tangential half-width factors, 1/2 at a boundary index),
// Dirichlet faces in a mask, zero-Neumann elsewhere; Jacobi-preconditioned
// conjugate gradients. Every kernel strides over the nodes with its grid; a
// kernel that forms a dot product runs the fine grid's G workgroups and
// leaves per-workgroup partials that every consumer adds in the same fixed
// order, so the solve is deterministic.

// The grid helpers take the fine grid (FieldParams) or a multigrid level
// (MgLevel): both carry n, sx, sy and mask.
template <class Gd>
__device__ __forceinline__ bool f_dir(const Gd &P, int i, int j, int k) {
  const int m = P.mask;
  return ((m & 1) && i == 0) || ((m & 2) && i == P.n[0]) || ((m & 4) && j == 0) ||
         ((m & 8) && j == P.n[1]) || ((m & 16) && k == 0) || ((m & 32) && k == P.n[2]);
}

// Dirichlet value of a node: the first Dirichlet face (in face order) it lies on
__device__ __forceinline__ double f_gval(const FieldParams &P, int i, int j, int k) {
  const int m = P.mask;
  if ((m & 1) && i == 0) return P.g[0];
  if ((m & 2) && i == P.n[0]) return P.g[1];
  if ((m & 4) && j == 0) return P.g[2];
  if ((m & 8) && j == P.n[1]) return P.g[3];
  if ((m & 16) && k == 0) return P.g[4];
  return P.g[5];
}

__device__ __forceinline__ double f_c(int a, int n) { return (a == 0 || a == n) ? 0.5 : 1.0; }

// node index -> (i, j, k); node counts stay below 2^31 (1024^3 cells at most)
template <class Gd>
__device__ __forceinline__ void f_ijk(const Gd &P, int64_t q, int &i, int &j, int &k) {
  const uint32_t u = (uint32_t)q, sy = (uint32_t)P.sy, sx = (uint32_t)P.sx;
  const uint32_t kk = u / sy, rem = u - kk * sy, jj = rem / sx;
  k = (int)kk;
  j = (int)jj;
  i = (int)(rem - jj * sx);
}

// The operator of a grid: node-centred finite volumes with one permittivity
// (kOpFV) or with the object as an interface (kOpIF, link permittivities), or
// immersed finite elements (kOpIFE, the fine grid only; the multigrid's
// coarser levels keep the finite volumes).
enum { kOpFV = 0, kOpIF = 1, kOpIFE = 2 };

// Visits the links of node (i, j, k) in the order -x, +x, -y, +y, -z, +z:
// f(q, w, i', j', k') with q the neighbour's node index and (i', j', k') its
// indices. Every node has all six: a link that would leave the box names the
// neighbour on the opposite side (every axis of a grid has at least one cell)
// with weight 0, and every use of it adds an exact zero (a link term is a
// weight times a finite difference or coefficient). Without a branch per link
// the loads of a stencil are independent of each other and issue together,
// instead of one memory latency after another; the stand-in is a node other
// than the centre so that the compiler cannot reuse the centre's value and
// turn the load back into a branch.
template <class Gd, class F>
__device__ __forceinline__ void f_links_n(const Gd &P, int i, int j, int k, int64_t q0, F f) {
  const double cx = f_c(i, P.n[0]), cy = f_c(j, P.n[1]), cz = f_c(k, P.n[2]);
  const bool xm = i > 0, xp = i < P.n[0], ym = j > 0, yp = j < P.n[1];
  const bool zm = k > 0, zp = k < P.n[2];
  f(xm ? q0 - 1 : q0 + 1, xm ? cy * cz : 0.0, xm ? i - 1 : i + 1, j, k);
  f(xp ? q0 + 1 : q0 - 1, xp ? cy * cz : 0.0, xp ? i + 1 : i - 1, j, k);
  f(ym ? q0 - P.sx : q0 + P.sx, ym ? cx * cz : 0.0, i, ym ? j - 1 : j + 1, k);
  f(yp ? q0 + P.sx : q0 - P.sx, yp ? cx * cz : 0.0, i, yp ? j + 1 : j - 1, k);
  f(zm ? q0 - P.sy : q0 + P.sy, zm ? cx * cy : 0.0, i, j, zm ? k - 1 : k + 1);
  f(zp ? q0 + P.sy : q0 - P.sy, zp ? cx * cy : 0.0, i, j, zp ? k + 1 : k - 1);
}

// The same, f(q, w).
template <class Gd, class F>
__device__ __forceinline__ void f_links(const Gd &P, int i, int j, int k, int64_t q0, F f) {
  f_links_n(P, i, j, k, q0, [&](int64_t nb, double w, int, int, int) { f(nb, w); });
}

// Sum over the workgroup (fixed tree order); the result in every thread.
__device__ double block_sum(double v) {
  __shared__ double sRed[kBlock];
  sRed[threadIdx.x] = v;
  __syncthreads();
  for (int o = kBlock / 2; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sRed[threadIdx.x] = sRed[threadIdx.x] + sRed[threadIdx.x + o];
    __syncthreads();
  }
  const double t = sRed[0];
  __syncthreads();
  return t;
}

// Sum of G partials, the same value in every workgroup. A thread adds its
// partials t, t + kBlock, ... in that order; they are loaded eight at a time,
// so that the loads are in flight together.
__device__ double sum_partials(const double *part, int G) {
  double v = 0.0;
  int t = threadIdx.x;
  for (; t + 7 * kBlock < G; t += 8 * kBlock) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = part[t + u * kBlock];
#pragma unroll
    for (int u = 0; u < 8; ++u) v = v + a[u];
  }
  for (; t < G; t += kBlock) v = v + part[t];
  return block_sum(v);
}

// The quotient of two such sums (numerator partials a, denominator b), both
// loaded before either is added up.
__device__ double ratio_partials(const double *a, const double *b, int G) {
  double va = 0.0, vb = 0.0;
  int t = threadIdx.x;
  for (; t + 7 * kBlock < G; t += 8 * kBlock) {
    double xa[8], xb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      xa[u] = a[t + u * kBlock];
      xb[u] = b[t + u * kBlock];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      va = va + xa[u];
      vb = vb + xb[u];
    }
  }
  for (; t < G; t += kBlock) {
    va = va + a[t];
    vb = vb + b[t];
  }
  const double sa = block_sum(va);
  return sa / block_sum(vb);
}

// Density at a node: the deposit, plus the surface source when there is one
// (fixed point; with the fixed-point deposit the two are added as integers).
template <int D>
__device__ __forceinline__ double f_rho(const FieldParams &P, int64_t q) {
  const double h3 = P.h * P.h * P.h;
  const int64_t surf = P.rho_surf ? P.rho_surf[q] : 0;
  if constexpr (D == PIC_DEP_FIXED64) {
    return ((double)(((const int64_t *)P.rho)[q] + surf) * 2.3283064365386963e-10) / h3;
  } else {
    const double v = D == PIC_DEP_ATOMIC_FP32 ? (double)((const float *)P.rho)[q]
                                              : ((const double *)P.rho)[q];
    if (!P.rho_surf) return v / h3;
    return v / h3 + ((double)surf * 2.3283064365386963e-10) / h3;
  }
}

// Series permittivity of a link: a the level set at its lower-index node, b at
// the other; the inside fraction by linear interpolation of the level set.
__device__ __forceinline__ double f_eps(double a, double b, double ein, double eout) {
  const bool ia = a < 0.0, ib = b < 0.0;
  if (ia == ib) return ia ? ein : eout;
  const double t = a / (a - b);
  const double f = ia ? t : 1.0 - t;
  return (ein * eout) / (f * eout + (1.0 - f) * ein);
}

template <class Gd>
__device__ __forceinline__ double f_link_eps(const Gd &L, const FieldParams &P, int64_t q,
                                             int64_t nb) {
  return nb < q ? f_eps(L.psi[nb], L.psi[q], P.e_in, P.e_out)
                : f_eps(L.psi[q], L.psi[nb], P.e_in, P.e_out);
}

// The same for the six links of a node at once: the seven level-set loads
// first, then the permittivities.
template <class Gd>
__device__ __forceinline__ void f_link_eps6(const Gd &L, const FieldParams &P, int64_t q,
                                            const int64_t nb[6], double eps[6]) {
  const double pq = L.psi[q];
  double pn[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) pn[l] = L.psi[nb[l]];
#pragma unroll
  for (int l = 0; l < 6; ++l)
    eps[l] = nb[l] < q ? f_eps(pn[l], pq, P.e_in, P.e_out) : f_eps(pq, pn[l], P.e_in, P.e_out);
}

// eps / h^2 of a node whose links all lie on one side (side 1 or 2)
template <class Gd>
__device__ __forceinline__ double f_cside(const FieldParams &P, const Gd &L, int sd) {
  return (sd == 2 ? P.e_in : P.e_out) * L.ih2;
}

// The diagonal of A at such a node: its link permittivity times the link
// weights, added in link order, times 1/h^2, as field_diag_kernel forms it
// for the stored diagonal (the same value).
template <class Gd>
__device__ __forceinline__ double f_dside(const FieldParams &P, const Gd &L, int i, int j, int k,
                                          int64_t q, int sd) {
  const double e = sd == 2 ? P.e_in : P.e_out;
  double d = 0.0;
  f_links(L, i, j, k, q, [&](int64_t, double w) { d = d + e * w; });
  return d * L.ih2;
}

// eps of a fine-grid node without an explicit row (all its tetrahedra on one
// side): from its side code (one byte) where that is set, which agrees with
// the sign of its level set there, else from the level set itself
__device__ __forceinline__ int ife_side(const FieldParams &P, int64_t q) {
  return P.iface ? P.side[q] : 1;  // (1: outside, without an object)
}

__device__ __forceinline__ double ife_eps(const FieldParams &P, int64_t q, int sd) {
  if (sd != 0) return sd == 2 ? P.e_in : P.e_out;
  return P.psi[q] < 0.0 ? P.e_in : P.e_out;
}

// The diagonal of the IFE operator at fine-grid node q = (i, j, k) with row
// index r = srow[q]: eps times the reference diagonal of its parity, or the
// last entry of its row; the values ife_rows_kernel stores as the diagonal.
__device__ __forceinline__ double ife_diag(const FieldParams &P, int i, int j, int k, int64_t q,
                                           int32_t r, int sd) {
  if (r < 0) return ife_eps(P, q, sd) * P.rld[(i + j + k) & 1];
  return P.rows[(int64_t)r * (kIfeLinks + 1) + kIfeLinks];
}

// Visits the links of fine-grid node q = (i, j, k) of the IFE operator in
// two passes: first val[l] = v(nb, i', j', k') for each of the 18 links l,
// the neighbour's index and indices (clamped into the box where the link
// leaves it), then f(c, val[l], i', j', k') with c = -A_q,nb (0 for a link the
// node does not have: an exact zero term). The first pass depends on the
// indices alone, so its loads issue together with the row's. A node away from
// the box faces whose tetrahedra the interface does not cut (srow < 0) has
// eps of its side times the reference links of its parity (a node of odd
// parity has no face diagonals); the others have their assembled row.
// ready(r, sd) runs between the two passes with the node's row index and
// side code, loaded with the first pass.
template <class V, class F, class R>
__device__ __forceinline__ void ife_links(const FieldParams &P, int i, int j, int k, int64_t q,
                                          V v, F f, R ready) {
  int ni[kIfeLinks], nj[kIfeLinks], nk[kIfeLinks];
  double val[kIfeLinks];
#pragma unroll
  for (int l = 0; l < kIfeLinks; ++l) {
    int o[3];
    ife_link_offset(l, o);
    // (a link leaving the box: its neighbour clamped into the box, a node
    // other than q, so that the load stays unconditional)
    ni[l] = min(max(i + o[0], 0), P.n[0]);
    nj[l] = min(max(j + o[1], 0), P.n[1]);
    nk[l] = min(max(k + o[2], 0), P.n[2]);
    val[l] = v(q + (ni[l] - i) + P.sx * (nj[l] - j) + P.sy * (nk[l] - k), ni[l], nj[l], nk[l]);
  }
  const int32_t r = P.srow[q];
  const int sd = ife_side(P, q);
  ready(r, sd);
  if (r < 0) {
    // (the coefficients are constants of the launch, the parity only selects
    // between two of them)
    const bool odd = ((i + j + k) & 1) != 0;
    const double e = ife_eps(P, q, sd);
#pragma unroll
    for (int l = 0; l < 6; ++l)
      f(e * (odd ? P.rl[1][l] : P.rl[0][l]), val[l], ni[l], nj[l], nk[l]);
#pragma unroll
    for (int l = 6; l < kIfeLinks; ++l)  // the face diagonals join nodes of even parity only
      f(odd ? 0.0 : e * P.rl[0][l], val[l], ni[l], nj[l], nk[l]);
    return;
  }
  const double *row = P.rows + (int64_t)r * (kIfeLinks + 1);
#pragma unroll
  for (int l = 0; l < kIfeLinks; ++l) f(row[l], val[l], ni[l], nj[l], nk[l]);
}

// The values of x that (A x) at node q reads at its six links, loaded (the
// finite-volume operators).
struct Nb6 {
  int64_t nb[6];
  double w[6], xn[6];
};

template <class Gd>
__device__ __forceinline__ void f_gather6(const Gd &L, const double *x, int i, int j, int k,
                                          int64_t q, Nb6 &g) {
  int n = 0;
  f_links(L, i, j, k, q, [&](int64_t m, double wl) {
    g.nb[n] = m;
    g.w[n] = wl;
    g.xn[n] = x[m];
    ++n;
  });
}

// (A x) at q from the gathered values: xq = x[q], sd the node's side code
// (the interface operator).
template <int OP, class Gd>
__device__ __forceinline__ double f_Ax6(const FieldParams &P, const Gd &L, int64_t q, double xq,
                                        int sd, const Nb6 &g) {
  double a = 0.0;
  if constexpr (OP == kOpIF) {
    if (sd != 0) {  // all six links of one permittivity (nearly every node)
#pragma unroll
      for (int l = 0; l < 6; ++l) a = a + g.w[l] * (xq - g.xn[l]);
      return f_cside(P, L, sd) * a;
    }
    double eps[6];
    f_link_eps6(L, P, q, g.nb, eps);
#pragma unroll
    for (int l = 0; l < 6; ++l) a = a + (eps[l] * g.w[l]) * (xq - g.xn[l]);
    return a * L.ih2;
  } else {
#pragma unroll
    for (int l = 0; l < 6; ++l) a = a + g.w[l] * (xq - g.xn[l]);
    return L.s * a;
  }
}

template <class V, class F>
__device__ __forceinline__ void ife_links(const FieldParams &P, int i, int j, int k, int64_t q,
                                          V v, F f) {
  ife_links(P, i, j, k, q, v, f, [](int32_t, int) {});
}

// (A x) at an unknown node q of a grid (the fine grid or a level)
template <int OP, class Gd>
__device__ __forceinline__ double f_Ax(const FieldParams &P, const Gd &L, const double *x, int i,
                                       int j, int k, int64_t q) {
  const double xq = x[q];
  double a = 0.0;
  if constexpr (OP == kOpIFE) {
    ife_links(
        P, i, j, k, q, [&](int64_t nb, int, int, int) { return x[nb]; },
        [&](double c, double xn, int, int, int) { a = a + c * (xq - xn); });
    return a;
  } else if constexpr (OP == kOpIF) {
    const int sd = L.side[q];
    int64_t nb[6];
    double w[6], d[6];
    int n = 0;
    f_links(L, i, j, k, q, [&](int64_t m, double wl) {
      nb[n] = m;
      w[n] = wl;
      d[n] = xq - x[m];
      ++n;
    });
    if (sd != 0) {  // all six links of one permittivity (nearly every node)
#pragma unroll
      for (int l = 0; l < 6; ++l) a = a + w[l] * d[l];
      return f_cside(P, L, sd) * a;
    }
    double eps[6];
    f_link_eps6(L, P, q, nb, eps);
#pragma unroll
    for (int l = 0; l < 6; ++l) a = a + (eps[l] * w[l]) * d[l];
    return a * L.ih2;
  } else {
    f_links(L, i, j, k, q, [&](int64_t nb, double w) { a = a + w * (xq - x[nb]); });
    return L.s * a;
  }
}

// r = b - A x, z = r / diag, p = z; Dirichlet nodes get x = g (and r = z = p = 0).
template <int D, int OP>
__global__ __launch_bounds__(kBlock) void field_init_kernel(FieldParams P) {
  constexpr bool IF = OP == kOpIF;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(P, q, i, j, k);
    if (f_dir(P, i, j, k)) {
      P.x[q] = f_gval(P, i, j, k);
      P.r[q] = 0.0;
      P.z[q] = 0.0;
      P.p[q] = 0.0;
      P.Ap[q] = 0.0;
      continue;
    }
    const double xq = P.x[q];
    const double rho = f_rho<D>(P, q);
    double ax = 0.0, dsum = 0.0, b = rho;
    if constexpr (OP == kOpIFE) {
      ife_links(
          P, i, j, k, q,
          [&](int64_t nb, int a, int cc, int e) {
            const double xl = P.x[nb];
            return f_dir(P, a, cc, e) ? f_gval(P, a, cc, e) : xl;
          },
          [&](double c, double xn, int a, int cc, int e) {
            ax = ax + c * (xq - xn);
            dsum = dsum + c;
            if (f_dir(P, a, cc, e)) b = b + c * xn;
          });
    } else {
      // the neighbours' values first (their loads together), then the terms
      int64_t nbs[6];
      double w[6], xn[6], cw[6];
      bool nd[6];
      int n = 0;
      f_links_n(P, i, j, k, q, [&](int64_t nb, double wl, int a, int c, int e) {
        nbs[n] = nb;
        w[n] = wl;
        nd[n] = f_dir(P, a, c, e);
        const double xl = P.x[nb];
        xn[n] = nd[n] ? f_gval(P, a, c, e) : xl;
        ++n;
      });
      if constexpr (IF) {
        const int sd = P.side[q];
        if (sd != 0) {
#pragma unroll
          for (int l = 0; l < 6; ++l) cw[l] = f_cside(P, P, sd) * w[l];
        } else {
          double eps[6];
          f_link_eps6(P, P, q, nbs, eps);
#pragma unroll
          for (int l = 0; l < 6; ++l) cw[l] = (eps[l] * w[l]) * P.ih2;
        }
      }
#pragma unroll
      for (int l = 0; l < 6; ++l) {
        if constexpr (IF) {
          ax = ax + cw[l] * (xq - xn[l]);
          dsum = dsum + cw[l];
          if (nd[l]) b = b + cw[l] * xn[l];
        } else {
          ax = ax + w[l] * (xq - xn[l]);
          dsum = dsum + w[l];
          if (nd[l]) b = b + P.s * w[l] * xn[l];
        }
      }
    }
    const double r = OP != kOpFV ? rho - ax : rho - P.s * ax;
    const double z = OP != kOpFV ? r / dsum : r / (P.s * dsum);
    P.r[q] = r;
    P.z[q] = z;
    P.p[q] = z;
    P.Ap[q] = 0.0;
    rz = rz + r * z;
    rr = rr + r * r;
    bb = bb + b * b;
  }
  rz = block_sum(rz);
  rr = block_sum(rr);
  bb = block_sum(bb);
  if (threadIdx.x == 0) {
    P.part[1 * P.G + blockIdx.x] = rz;
    P.part[3 * P.G + blockIdx.x] = rr;
    P.part[5 * P.G + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(kBlock) void field_check0_kernel(FieldParams P) {
  const double rr = sum_partials(P.part + 3 * P.G, P.G);
  const double bb = sum_partials(P.part + 5 * P.G, P.G);
  if (threadIdx.x == 0) {
    P.ctrl->rr = rr;
    P.ctrl->bb = bb;
    P.ctrl->iters = 0;
    P.ctrl->converged = __builtin_sqrt(rr) <= P.tol * __builtin_sqrt(bb) ? 1 : 0;
  }
}

// The control block, read once per workgroup (thread 0, then shared), so that
// every thread takes the same early exit even while workgroup 0 of the same
// launch updates it.
__device__ __forceinline__ FieldCtrl f_ctrl(const FieldParams &P) {
  __shared__ FieldCtrl sCtrl;
  if (threadIdx.x == 0) sCtrl = *P.ctrl;
  __syncthreads();
  const FieldCtrl c = sCtrl;
  __syncthreads();
  return c;
}

__device__ __forceinline__ bool f_done(const FieldCtrl &c, const FieldParams &P) {
  return c.converged != 0 || c.iters >= P.max_iter;
}

// The early exit of a kernel that does not write the control block: every
// thread loads the block itself (no workgroup barrier) with its data, in the
// same pass over its node, and tests it only after f_issued, so that the two
// latencies overlap instead of adding up.
__device__ __forceinline__ int2 f_ctl(const FieldParams &P) {
  // (converged and iters, the first two words of the block, in one load; an
  // opaque zero offset keeps the compiler from treating the value as uniform
  // and moving it to a scalar register at once, which would wait for it)
  static_assert(offsetof(FieldCtrl, converged) == 0 && offsetof(FieldCtrl, iters) == 4, "");
  int z = 0;
  __asm__ __volatile__("" : "+v"(z));
  return reinterpret_cast<const int2 *>(P.ctrl)[z];
}

// Compiler barrier: the loads written above it stay above it, and the test of
// the control block c stays below it (the loads are in flight when the code
// first waits, for c).
__device__ __forceinline__ void f_issued(int2 &c) {
  __asm__ __volatile__("" : "+v"(c.x), "+v"(c.y) : : "memory");
}

__device__ __forceinline__ bool f_stop(int2 c, const FieldParams &P) {
  return (c.x != 0) | (c.y >= P.max_iter);
}

// kFineExit: the kernels on the fine level (l == 0, or restricting from it)
// still test the block first and return before their loads: a V-cycle
// enqueued after the solve has converged then costs a few microseconds per
// fine-level kernel instead of a full pass over 2 M nodes, while on the small
// coarse levels the overlap saves more than the loads cost.

// Ap = A p; partial p.Ap
template <int OP>
__global__ __launch_bounds__(kBlock) void field_apply_kernel(FieldParams P) {
  if (f_done(f_ctrl(P), P)) return;  // uniform
  double pap = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(P, q, i, j, k);
    if (f_dir(P, i, j, k)) continue;
    const double pq = P.p[q];
    const double ap = f_Ax<OP>(P, P, P.p, i, j, k, q);
    P.Ap[q] = ap;
    pap = pap + pq * ap;
  }
  pap = block_sum(pap);
  if (threadIdx.x == 0) P.part[blockIdx.x] = pap;
}

// x += alpha p, r -= alpha Ap; partial r.r (parity n); Jacobi form: also
// z = r / diag and partial r.z
template <bool J, int OP>
__global__ __launch_bounds__(kBlock) void field_update_kernel(FieldParams P, int o) {
  if (f_done(f_ctrl(P), P)) return;  // uniform
  const int n = 1 - o;
  const double alpha = ratio_partials(P.part + (1 + o) * P.G, P.part, P.G);
  double rz = 0.0, rr = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(P, q, i, j, k);
    if (f_dir(P, i, j, k)) continue;
    const double x = P.x[q] + alpha * P.p[q];
    const double r = P.r[q] - alpha * P.Ap[q];
    P.x[q] = x;
    P.r[q] = r;
    if constexpr (J) {
      double d;
      if constexpr (OP != kOpFV) {
        d = P.diag[q];
      } else {
        double dsum = 0.0;
        f_links(P, i, j, k, q, [&](int64_t, double w) { dsum = dsum + w; });
        d = P.s * dsum;
      }
      const double z = r / d;
      P.z[q] = z;
      rz = rz + r * z;
    }
    rr = rr + r * r;
  }
  if constexpr (J) rz = block_sum(rz);
  rr = block_sum(rr);
  if (threadIdx.x == 0) {
    if constexpr (J) P.part[(1 + n) * P.G + blockIdx.x] = rz;
    P.part[(3 + n) * P.G + blockIdx.x] = rr;
  }
}

// The convergence test of an iteration (parity o): ||r|| <= tol ||b||; the
// iteration count, ||r||^2 and the flag go to the control block.
__device__ __forceinline__ bool f_check(const FieldParams &P, const FieldCtrl &c, int o,
                                        bool write) {
  const int n = 1 - o;
  const double rr = sum_partials(P.part + (3 + n) * P.G, P.G);
  const bool conv = __builtin_sqrt(rr) <= P.tol * __builtin_sqrt(c.bb);
  if (write && threadIdx.x == 0) {
    P.ctrl->rr = rr;
    P.ctrl->iters = c.iters + 1;
    if (conv) P.ctrl->converged = 1;
  }
  return conv;
}

// multigrid form: the test alone, one workgroup, before the V-cycle (whose
// kernels then stop at f_done)
__global__ __launch_bounds__(kBlock) void field_check_kernel(FieldParams P, int o) {
  const FieldCtrl c = f_ctrl(P);
  if (f_done(c, P)) return;  // uniform
  f_check(P, c, o, true);
}

// Jacobi form: convergence test, then p = z + beta p; multigrid form: p = z +
// beta p (the test ran before the V-cycle)
template <bool J>
__global__ __launch_bounds__(kBlock) void field_dir_kernel(FieldParams P, int o) {
  const FieldCtrl c = f_ctrl(P);
  if (f_done(c, P)) return;  // uniform
  const int n = 1 - o;
  if constexpr (J) {
    if (f_check(P, c, o, blockIdx.x == 0)) return;  // uniform
  }
  const double beta = ratio_partials(P.part + (1 + n) * P.G, P.part + (1 + o) * P.G, P.G);
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(P, q, i, j, k);
    if (f_dir(P, i, j, k)) continue;
    P.p[q] = P.z[q] + beta * P.p[q];
  }
}

// ---- multigrid V-cycle preconditioner
//
// z = B r by one V-cycle over nested node grids (level l + 1: every other node
// of level l, spacing 2h, the same faces, the finite-volume operator
// rediscretised, homogeneous Dirichlet values): two damped-Jacobi sweeps from
// zero, residual, restriction R = P^T / 8 (full weighting of the residual
// density), the coarser cycle, trilinear prolongation P, two more sweeps; the
// coarsest level (at most kCoarseNodes nodes) is solved exactly with its
// inverse. With the same sweeps before and after and R proportional to P^T,
// B is symmetric positive definite, so CG with it is still CG. Each level's
// kernels run its own G workgroups over its nodes; all of them stop at
// f_done.

constexpr double kOmega = 6.0 / 7.0;  // Jacobi damping (3-D 7-point smoothing optimum)

template <class Gd>
__device__ __forceinline__ double f_dsum(const Gd &L, int i, int j, int k) {
  return ((i > 0) + (i < L.n[0])) * (f_c(j, L.n[1]) * f_c(k, L.n[2])) +
         ((j > 0) + (j < L.n[1])) * (f_c(i, L.n[0]) * f_c(k, L.n[2])) +
         ((k > 0) + (k < L.n[2])) * (f_c(i, L.n[0]) * f_c(j, L.n[1]));
}

// diagonal of A at an unknown node of a level
// (the interface: the stored diagonal only at a node with a link across it;
// sd the node's side code, already loaded)
template <int OP>
__device__ __forceinline__ double mg_Ds(const FieldParams &P, const MgLevel &L, int i, int j,
                                        int k, int64_t q, int sd) {
  if constexpr (OP == kOpIF) {
    if (sd == 0) return L.diag[q];
    // off the box faces all six weights are 1: the sum is e + e + ... + e
    if (i > 0 && i < L.n[0] && j > 0 && j < L.n[1] && k > 0 && k < L.n[2]) {
      const double e = sd == 2 ? P.e_in : P.e_out;
      return (((((e + e) + e) + e) + e) + e) * L.ih2;
    }
    return f_dside(P, L, i, j, k, q, sd);
  } else if constexpr (OP == kOpIFE) {  // (the fine level only)
    return ife_diag(P, i, j, k, q, P.srow[q], ife_side(P, q));
  } else {
    return L.s * f_dsum(L, i, j, k);
  }
}

template <int OP>
__device__ __forceinline__ double mg_D(const FieldParams &P, const MgLevel &L, int i, int j, int k,
                                       int64_t q) {
  return mg_Ds<OP>(P, L, i, j, k, q, OP == kOpIF ? L.side[q] : 1);
}

// e = two sweeps from zero: e1 = w b / d is pointwise, so the second sweep
// computes e1 at the neighbours itself.
template <int OP>
__global__ __launch_bounds__(kBlock) void mg_pre_kernel(FieldParams P, int l) {
  constexpr bool IF = OP == kOpIF;
  const MgLevel L = P.lv[l];  // (a copy: its fields load once, unconditionally)
  if constexpr (OP == kOpIFE) {  // the neighbours' e1 from mg_e1_kernel
    if (f_done(f_ctrl(P), P)) return;  // uniform
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
         q += (int64_t)gridDim.x * kBlock) {
      int i, j, k;
      f_ijk(L, q, i, j, k);
      if (f_dir(L, i, j, k)) {
        L.e[q] = 0.0;
        continue;
      }
      const double bq = L.rhs[q];
      double a = 0.0, d = 0.0, e1 = 0.0;
      ife_links(
          P, i, j, k, q, [&](int64_t nb, int, int, int) { return L.e2[nb]; },
          [&](double c, double e1n, int, int, int) { a = a + c * (e1 - e1n); },
          [&](int32_t r, int sd) {  // (the diagonal once the row index is in)
            d = ife_diag(P, i, j, k, q, r, sd);
            e1 = kOmega * bq / d;
          });
      L.e[q] = e1 + kOmega * (bq - a) / d;
    }
  } else {
    if (l == 0 && f_done(f_ctrl(P), P)) return;  // uniform (see kFineExit)
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
         q += (int64_t)gridDim.x * kBlock) {
      int i, j, k;
      f_ijk(L, q, i, j, k);
      int2 ctl = f_ctl(P);
      if (f_dir(L, i, j, k)) {
        if (f_stop(ctl, P)) return;  // uniform
        L.e[q] = 0.0;
        continue;
      }
      // loads: the node's right-hand side, side code and (the interface)
      // stored diagonal, the same at its neighbours; the finite-volume
      // diagonals are arithmetic
      const double bq = L.rhs[q];
      const int sd = IF ? L.side[q] : 1;
      const double d = IF ? L.diag[q] : mg_Ds<OP>(P, L, i, j, k, q, sd);
      int64_t nbs[6];
      double w[6], bn[6], dn[6];
      int dirm = 0, n = 0;
      f_links_n(L, i, j, k, q, [&](int64_t nb, double wl, int a2, int b2, int c2) {
        nbs[n] = nb;
        w[n] = wl;
        bn[n] = L.rhs[nb];
        dn[n] = IF ? L.diag[nb] : mg_Ds<OP>(P, L, a2, b2, c2, nb, 1);
        dirm |= f_dir(L, a2, b2, c2) ? 1 << n : 0;
        ++n;
      });
      f_issued(ctl);
      if (f_stop(ctl, P)) return;  // uniform
      const double e1 = kOmega * bq / d;
      // e1 at a neighbour, 0 at a Dirichlet one (whose diagonal is positive
      // as well: a product instead of a branch)
      double de[6];
#pragma unroll
      for (int m = 0; m < 6; ++m)
        de[m] = e1 - ((((dirm >> m) & 1) ? 0.0 : kOmega) * bn[m]) / dn[m];
      double a = 0.0;
      const bool uni = sd != 0;  // one permittivity on all six links
      if (uni) {
#pragma unroll
        for (int m = 0; m < 6; ++m) a = a + w[m] * de[m];
      } else {
        double eps[6];
        f_link_eps6(L, P, q, nbs, eps);
#pragma unroll
        for (int m = 0; m < 6; ++m) a = a + (eps[m] * w[m]) * de[m];
      }
      const double Ae1 = IF ? (uni ? f_cside(P, L, sd) * a : a * L.ih2) : L.s * a;
      L.e[q] = e1 + kOmega * (bq - Ae1) / d;
    }
  }
}

// IFE finest level: the first (pointwise) sweep from zero, e1 = w b / d, into
// e2 (unused until the post-smoothing), so that the second sweep of
// mg_pre_kernel reads it at its up to 18 neighbours instead of evaluating it
// there (two loads and a division each); the values are the same.
__global__ __launch_bounds__(kBlock) void mg_e1_kernel(FieldParams P, int l) {
  if (f_done(f_ctrl(P), P)) return;  // uniform
  const MgLevel L = P.lv[l];  // (a copy: its fields load once, unconditionally)
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(L, q, i, j, k);
    L.e2[q] = f_dir(L, i, j, k) ? 0.0 : kOmega * L.rhs[q] / mg_D<kOpIFE>(P, L, i, j, k, q);
  }
}

// res = b - A e
template <int OP>
__global__ __launch_bounds__(kBlock) void mg_res_kernel(FieldParams P, int l) {
  const MgLevel L = P.lv[l];  // (a copy: its fields load once, unconditionally)
  if constexpr (OP == kOpIFE) {
    if (f_done(f_ctrl(P), P)) return;  // uniform
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
         q += (int64_t)gridDim.x * kBlock) {
      int i, j, k;
      f_ijk(L, q, i, j, k);
      L.res[q] = f_dir(L, i, j, k) ? 0.0 : L.rhs[q] - f_Ax<OP>(P, L, L.e, i, j, k, q);
    }
  } else {
    if (l == 0 && f_done(f_ctrl(P), P)) return;  // uniform (see kFineExit)
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
         q += (int64_t)gridDim.x * kBlock) {
      int i, j, k;
      f_ijk(L, q, i, j, k);
      int2 ctl = f_ctl(P);
      if (f_dir(L, i, j, k)) {
        if (f_stop(ctl, P)) return;  // uniform
        L.res[q] = 0.0;
        continue;
      }
      const double bq = L.rhs[q], eq = L.e[q];
      const int sd = OP == kOpIF ? L.side[q] : 1;
      Nb6 g;
      f_gather6(L, L.e, i, j, k, q, g);
      f_issued(ctl);
      if (f_stop(ctl, P)) return;  // uniform
      L.res[q] = bq - f_Ax6<OP>(P, L, q, eq, sd, g);
    }
  }
}

// rhs of level l + 1 = P^T res / 8: a coarse node gathers the fine residuals
// of its 3x3x3 fine neighbourhood (in the box) with weights 1 or 1/2 per axis.
__global__ __launch_bounds__(kBlock) void mg_restrict_kernel(FieldParams P, int l) {
  if (l == 0 && f_done(f_ctrl(P), P)) return;  // uniform (see kFineExit)
  const MgLevel F = P.lv[l], C = P.lv[l + 1];
  for (int64_t Q = (int64_t)blockIdx.x * kBlock + threadIdx.x; Q < C.nodes;
       Q += (int64_t)gridDim.x * kBlock) {
    int I, J, K;
    f_ijk(C, Q, I, J, K);
    int2 ctl = f_ctl(P);
    if (f_dir(C, I, J, K)) {
      if (f_stop(ctl, P)) return;  // uniform
      C.rhs[Q] = 0.0;
      continue;
    }
    // (a fine node outside the box contributes weight 0 at the coarse node's
    // own fine node, so that all 27 loads are unconditional)
    const int i0 = 2 * I, j0 = 2 * J, k0 = 2 * K;
    double r[27], wt[27];
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
      const int k = k0 + dk;
      const bool kin = k >= 0 && k <= F.n[2];
      const double wk = !kin ? 0.0 : dk == 0 ? 1.0 : 0.5;
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const int j = j0 + dj;
        const bool jin = j >= 0 && j <= F.n[1];
        const double wjk = wk * (!jin ? 0.0 : dj == 0 ? 1.0 : 0.5);
        const double *row = F.res + (int64_t)(kin ? k : k0) * F.sy + (int64_t)(jin ? j : j0) * F.sx;
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
          const int i = i0 + di;
          const bool iin = i >= 0 && i <= F.n[0];
          const int t = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
          wt[t] = wjk * (!iin ? 0.0 : di == 0 ? 1.0 : 0.5);
          r[t] = row[iin ? i : i0];
        }
      }
    }
    f_issued(ctl);
    if (f_stop(ctl, P)) return;  // uniform
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 27; ++t) v = v + wt[t] * r[t];
    C.rhs[Q] = v * 0.125;
  }
}

// e of the coarsest level = A^-1 rhs on its m unknowns: one wave per row,
// the right-hand side gathered into LDS. The launch has a wave for every row
// (m / 4 workgroups, rounded up), so each wave loads its row first, with the
// gather, and adds it up in the order v = lane, lane + 64, ...
__global__ __launch_bounds__(kBlock) void mg_coarse_kernel(FieldParams P) {
  const MgLevel C = P.lv[P.levels - 1];
  __shared__ double sb[kCoarseNodes];
  constexpr int kPer = (int)(kCoarseNodes / 64);  // row elements per lane
  const int m = P.m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int u = blockIdx.x * (kBlock / 64) + wave;
  int2 ctl = f_ctl(P);
  double r[kPer];
  if (u < m) {
    const double *row = P.ainv + (int64_t)u * m;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int v = lane + 64 * t;
      r[t] = row[v < m ? v : m - 1];  // (past m: an element of the row, unused)
    }
  }
  for (int v = threadIdx.x; v < m; v += kBlock) sb[v] = C.rhs[P.umap[v]];
  f_issued(ctl);
  if (f_stop(ctl, P)) return;  // uniform
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < C.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(C, q, i, j, k);
    if (f_dir(C, i, j, k)) C.e[q] = 0.0;
  }
  __syncthreads();
  if (u < m) {
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int v = lane + 64 * t;
      if (v < m) a = a + r[t] * sb[v];
    }
    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) C.e[P.umap[u]] = a;
  }
}

// e += P e_c (trilinear: per axis the coarse node itself, or the mean of two)
__global__ __launch_bounds__(kBlock) void mg_prolong_kernel(FieldParams P, int l) {
  if (l == 0 && f_done(f_ctrl(P), P)) return;  // uniform (see kFineExit)
  const MgLevel F = P.lv[l], C = P.lv[l + 1];
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < F.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(F, q, i, j, k);
    if (f_dir(F, i, j, k)) continue;
    int2 ctl = f_ctl(P);
    // (always 2 x 2 x 2 coarse nodes: along an even axis the second one is
    // the first again with weight 0, so that the loads are unconditional)
    const int ni = 1 + (i & 1), nj = 1 + (j & 1), nk = 1 + (k & 1);
    const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0, wk = (k & 1) ? 0.5 : 1.0;
    const double w = wi * wj * wk;
    const double eq = F.e[q];
    double ec[8];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double *row = C.e + (int64_t)(k / 2 + (c < nk ? c : 0)) * C.sy +
                            (int64_t)(j / 2 + (b < nj ? b : 0)) * C.sx;
#pragma unroll
        for (int a = 0; a < 2; ++a) ec[4 * c + 2 * b + a] = row[i / 2 + (a < ni ? a : 0)];
      }
    f_issued(ctl);
    if (f_stop(ctl, P)) return;  // uniform
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a)
          v = v + ((a < ni && b < nj && c < nk) ? w : 0.0) * ec[4 * c + 2 * b + a];
    F.e[q] = eq + v;
  }
}

// One damped-Jacobi sweep out = in + w (b - A in) / d. On level 0 the second
// post-sweep writes z itself and the partial r.z to part[prz].
template <bool Dot, int OP>
__global__ __launch_bounds__(kBlock) void mg_sweep_kernel(FieldParams P, int l, int to_e2, int prz) {
  const MgLevel L = P.lv[l];  // (a copy: its fields load once, unconditionally)
  const double *in = to_e2 ? L.e : L.e2;
  double *out = to_e2 ? L.e2 : L.e;
  double rz = 0.0;
  if constexpr (OP == kOpIFE) {
    if (f_done(f_ctrl(P), P)) return;  // uniform
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
         q += (int64_t)gridDim.x * kBlock) {
      int i, j, k;
      f_ijk(L, q, i, j, k);
      if (f_dir(L, i, j, k)) {
        out[q] = 0.0;
        continue;
      }
      const double bq = L.rhs[q];
      const double v =
          in[q] + kOmega * (bq - f_Ax<OP>(P, L, in, i, j, k, q)) / mg_D<OP>(P, L, i, j, k, q);
      out[q] = v;
      if constexpr (Dot) rz = rz + bq * v;
    }
  } else {
    if (l == 0 && f_done(f_ctrl(P), P)) return;  // uniform (see kFineExit)
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
         q += (int64_t)gridDim.x * kBlock) {
      int i, j, k;
      f_ijk(L, q, i, j, k);
      int2 ctl = f_ctl(P);
      if (f_dir(L, i, j, k)) {
        if (f_stop(ctl, P)) return;  // uniform
        out[q] = 0.0;
        continue;
      }
      const double bq = L.rhs[q], inq = in[q];
      const int sd = OP == kOpIF ? L.side[q] : 1;
      Nb6 g;
      f_gather6(L, in, i, j, k, q, g);
      f_issued(ctl);
      if (f_stop(ctl, P)) return;  // uniform
      const double v =
          inq + kOmega * (bq - f_Ax6<OP>(P, L, q, inq, sd, g)) / mg_Ds<OP>(P, L, i, j, k, q, sd);
      out[q] = v;
      if constexpr (Dot) rz = rz + bq * v;
    }
    if (f_stop(f_ctl(P), P)) return;  // uniform (the threads without a node)
  }
  if constexpr (Dot) {
    rz = block_sum(rz);
    if (threadIdx.x == 0) P.part[prz * P.G + blockIdx.x] = rz;
  }
}

// Level set of the object at the nodes of level l (< 0 inside; fine cell units).
__global__ __launch_bounds__(kBlock) void field_psi_kernel(FieldParams P, int l) {
  const MgLevel L = P.lv[l];  // (a copy: its fields load once, unconditionally)
  const FieldGeom &o = P.geo;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(L, q, i, j, k);
    const double x = L.scale * i, y = L.scale * j, z = L.scale * k;
    double v;
    if (o.kind == PIC_OBJ_SPHERE) {
      const double dx = x - o.c[0], dy = y - o.c[1], dz = z - o.c[2];
      v = __builtin_sqrt(dx * dx + dy * dy + dz * dz) - o.r;
    } else {
      const double dx = x - o.c[0], dy = y - o.c[1];
      const double r2 = dx * dx + dy * dy;
      const double ground = r2 < o.a2 ? o.zc - __builtin_sqrt(o.rc2 - r2) : o.z_flat;
      v = z - ground;
    }
    L.psi[q] = v;
  }
}

// Diagonal of A at the nodes of level l: sum of the link coefficients.
__global__ __launch_bounds__(kBlock) void field_diag_kernel(FieldParams P, int l) {
  const MgLevel L = P.lv[l];  // (a copy: its fields load once, unconditionally)
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < L.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(L, q, i, j, k);
    double d = 0.0;
    const bool in = L.psi[q] < 0.0;
    bool uni = true;
    f_links(L, i, j, k, q, [&](int64_t nb, double w) {
      d = d + f_link_eps(L, P, q, nb) * w;
      uni = uni && ((L.psi[nb] < 0.0) == in);
    });
    L.diag[q] = d * L.ih2;
    L.side[q] = uni ? (in ? 2 : 1) : 0;
  }
}

// ---- immersed finite elements: the rows of the operator
//
// A fine-grid node on a box face, or a vertex of a tetrahedron that the
// interface cuts, gets an explicit row; every other node applies eps of its
// side times the reference links of its parity (FieldParams.rl, evaluated on
// the host with the same element functions). A row is gathered by its node
// over the cubes around it in increasing global order and their tetrahedra in
// order: per link, a tetrahedron adds its element matrix entry; a link whose
// tetrahedra are all uncut and of one side takes that side's eps times the sum
// of the reference entries instead, exactly as a neighbour without a row
// computes it, so the operator stays exactly symmetric.

// Level set of a fine-grid node as the elements see it (+1 without an object).
__device__ __forceinline__ double ife_psi(const FieldParams &P, int64_t q) {
  return P.iface ? P.psi[q] : 1.0;
}

// The level set at the 8 corners of cube (ci, cj, ck).
__device__ __forceinline__ void ife_cube_psi(const FieldParams &P, int ci, int cj, int ck,
                                             double cp[8]) {
  const int64_t base = ci + P.sx * cj + P.sy * ck;
  for (int c = 0; c < 8; ++c)
    cp[c] = ife_psi(P, base + (c & 1) + P.sx * ((c >> 1) & 1) + P.sy * ((c >> 2) & 1));
}

// Whether node (i, j, k) needs an explicit row.
__device__ bool ife_special(const FieldParams &P, int i, int j, int k) {
  if (i == 0 || j == 0 || k == 0 || i == P.n[0] || j == P.n[1] || k == P.n[2]) return true;
  if (!P.iface) return false;
  for (int dc = -1; dc <= 0; ++dc)
    for (int db = -1; db <= 0; ++db)
      for (int da = -1; da <= 0; ++da) {
        const int ci = i + da, cj = j + db, ck = k + dc;
        double cp[8];
        ife_cube_psi(P, ci, cj, ck, cp);
        const int p = (ci + cj + ck) & 1, lp = -da - 2 * db - 4 * dc;
        for (int t = 0; t < 5; ++t) {
          int v[4];
          ife_tet(p, t, v);
          bool has = false, in = false, out = false;
          for (int r = 0; r < 4; ++r) {
            has |= v[r] == lp;
            (cp[v[r]] < 0.0 ? in : out) = true;
          }
          if (has && in && out) return true;
        }
      }
  return false;
}

// srow = -2 for the nodes that need a row, else -1; count[0] += their number.
__global__ __launch_bounds__(kBlock) void ife_mark_kernel(FieldParams P, int32_t *srow,
                                                          int32_t *count) {
  int32_t c = 0;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(P, q, i, j, k);
    const bool sp = ife_special(P, i, j, k);
    srow[q] = sp ? -2 : -1;
    c += sp;
  }
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
  if (__lane_id() == 0 && c) atomicAdd(count, c);
}

// The rows of the marked nodes (each takes the next free row index), and the
// diagonal of the fine level at every node.
__global__ __launch_bounds__(kBlock) void ife_rows_kernel(FieldParams P, int32_t *srow,
                                                          double *rows, int32_t *next,
                                                          double *diag) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    f_ijk(P, q, i, j, k);
    if (srow[q] != -2) {
      const int par = (i + j + k) & 1;
      const double e = (P.iface && P.psi[q] < 0.0) ? P.e_in : P.e_out;
      diag[q] = e * P.rld[par];
      continue;
    }
    double act[kIfeLinks], ref[kIfeLinks];
    int8_t side[kIfeLinks];  // -1 no tetrahedron yet, 0 outside, 1 inside, 2 cut or both
    for (int l = 0; l < kIfeLinks; ++l) {
      act[l] = 0.0;
      ref[l] = 0.0;
      side[l] = -1;
    }
    const double ones[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    for (int dc = -1; dc <= 0; ++dc)
      for (int db = -1; db <= 0; ++db)
        for (int da = -1; da <= 0; ++da) {
          const int ci = i + da, cj = j + db, ck = k + dc;
          if (ci < 0 || cj < 0 || ck < 0 || ci >= P.n[0] || cj >= P.n[1] || ck >= P.n[2]) continue;
          double cp[8];
          ife_cube_psi(P, ci, cj, ck, cp);
          const int p = (ci + cj + ck) & 1, lp = -da - 2 * db - 4 * dc;
          for (int t = 0; t < 5; ++t) {
            int v[4];
            double K[4][4], R[4][4];
            ife_cube_element(p, t, cp, P.e_in, P.e_out, v, K);
            ife_cube_element(p, t, ones, 1.0, 1.0, v, R);
            int rp = -1;
            bool in = false, out = false;
            for (int r = 0; r < 4; ++r) {
              if (v[r] == lp) rp = r;
              (cp[v[r]] < 0.0 ? in : out) = true;
            }
            if (rp < 0) continue;
            const int8_t sd = (in && out) ? 2 : (in ? 1 : 0);
            for (int r = 0; r < 4; ++r) {
              if (r == rp) continue;
              const int l = ife_link_of((v[r] & 1) - (lp & 1), ((v[r] >> 1) & 1) - ((lp >> 1) & 1),
                                        ((v[r] >> 2) & 1) - ((lp >> 2) & 1));
              act[l] -= K[rp][r];
              ref[l] -= R[rp][r];
              side[l] = side[l] < 0 ? sd : (side[l] == sd ? sd : 2);
            }
          }
        }
    const int32_t r = atomicAdd(next, 1);
    srow[q] = r;
    double *row = rows + (int64_t)r * (kIfeLinks + 1);
    double d = 0.0;
    for (int l = 0; l < kIfeLinks; ++l) {
      double c = 0.0;
      if (side[l] == 2) c = act[l] * P.ih2;
      else if (side[l] >= 0) c = (side[l] == 1 ? P.e_in : P.e_out) * (ref[l] * P.ih2);
      row[l] = c;
      d = d + c;
    }
    row[kIfeLinks] = d;
    diag[q] = d;
  }
}

// The collected charge of each tally bin at the bin's surface point,
// deposited to the nodes in int64 fixed point (trilinear weights, the
// remainder on the last corner so that the bin's charge is kept exactly).
__global__ __launch_bounds__(kBlock) void surface_rho_kernel(SurfParams S) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= S.nbins) return;
  double Q = 0.0;
  for (int s = 0; s < S.ns; ++s) Q = Q + S.chg[s] * (double)S.tally[b * S.ns + s];
  if (Q == 0.0) return;
  if (!(__builtin_fabs(Q) < 1073741824.0)) {
    atomicOr(S.err, kErrSurface);
    return;
  }
  const FieldGeom &o = S.geo;
  double g[3];
  if (o.kind == PIC_OBJ_CRATER) {
    g[0] = (double)(b % S.n[0]) + 0.5;
    g[1] = (double)(b / S.n[0]) + 0.5;
    const double dx = g[0] - o.c[0], dy = g[1] - o.c[1];
    const double r2 = dx * dx + dy * dy;
    g[2] = r2 < o.a2 ? o.zc - __builtin_sqrt(o.rc2 - r2) : o.z_flat;
  } else {
    const int m = o.patches;
    const int face = (int)(b / ((int64_t)m * m)), iv = (int)((b / m) % m), iu = (int)(b % m);
    const int ax = face / 2;
    const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
    double d[3];
    d[ax] = (face & 1) ? 1.0 : -1.0;
    d[u] = -1.0 + (2.0 * iu + 1.0) / m;
    d[v] = -1.0 + (2.0 * iv + 1.0) / m;
    const double len = __builtin_sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; ++k) g[k] = o.c[k] + o.rs * (d[k] / len);
  }
  int ci[3];
  double f[3];
  for (int k = 0; k < 3; ++k) {
    double fl = __builtin_floor(g[k]);
    fl = fl < 0.0 ? 0.0 : (fl > (double)(S.n[k] - 1) ? (double)(S.n[k] - 1) : fl);
    ci[k] = (int)fl;
    double of = g[k] - fl;
    f[k] = of < 0.0 ? 0.0 : (of > 1.0 ? 1.0 : of);
  }
  double W[8];
  weights(f, W);
  long long C[8], sum = 0;
  for (int n = 0; n < 7; ++n) {
    C[n] = fixq(Q * W[n]);
    sum += C[n];
  }
  C[7] = fixq(Q) - sum;
  const int64_t base = ci[0] + S.sx * ci[1] + S.sy * ci[2];
  const int64_t off[8] = {0, 1, S.sx, S.sx + 1, S.sy, S.sy + 1, S.sy + S.sx, S.sy + S.sx + 1};
  for (int n = 0; n < 8; ++n)
    atomicAdd((unsigned long long *)&S.rho_surf[base + off[n]], (unsigned long long)C[n]);
}

// multigrid start: p = z
__global__ __launch_bounds__(kBlock) void field_pstart_kernel(FieldParams P) {
  if (f_done(f_ctrl(P), P)) return;  // uniform
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock)
    P.p[q] = P.z[q];
}

// E = -grad phi at the nodes: central differences inside, 0 normal to a
// zero-Neumann face, second-order one-sided differences on a Dirichlet face.
template <int R>
__global__ __launch_bounds__(kBlock) void field_E_kernel(FieldParams P) {
  using T = typename RealOf<R>::T;
  using V4 = typename Vec4Of<T>::type;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P.nodes;
       q += (int64_t)gridDim.x * kBlock) {
    int ijk[3];
    f_ijk(P, q, ijk[0], ijk[1], ijk[2]);
    const int64_t st[3] = {1, P.sx, P.sy};
    double e[3];
    for (int d = 0; d < 3; ++d) {
      const int a = ijk[d], n = P.n[d];
      const double *x = P.x;
      if (a > 0 && a < n) {
        e[d] = -(x[q + st[d]] - x[q - st[d]]) / (2.0 * P.h);
      } else if (!((P.mask >> (2 * d + (a == 0 ? 0 : 1))) & 1)) {
        e[d] = 0.0;
      } else if (n == 1) {
        e[d] = a == 0 ? -(x[q + st[d]] - x[q]) / P.h : -(x[q] - x[q - st[d]]) / P.h;
      } else if (a == 0) {
        e[d] = -(-3.0 * x[q] + 4.0 * x[q + st[d]] - x[q + 2 * st[d]]) / (2.0 * P.h);
      } else {
        e[d] = -(3.0 * x[q] - 4.0 * x[q - st[d]] + x[q - 2 * st[d]]) / (2.0 * P.h);
      }
    }
    V4 v;
    v.x = (T)e[0];
    v.y = (T)e[1];
    v.z = (T)e[2];
    v.w = T(0);
    ((V4 *)P.E)[q] = v;
  }
}

}  // namespace

template <int OP>
static hipError_t field_init(int deposit, const FieldParams &p, hipStream_t s) {
  switch (deposit) {
    case PIC_DEP_FIXED64:
      hipLaunchKernelGGL((field_init_kernel<PIC_DEP_FIXED64, OP>), dim3(p.G), dim3(kBlock), 0, s, p);
      break;
    case PIC_DEP_ATOMIC_FP32:
      hipLaunchKernelGGL((field_init_kernel<PIC_DEP_ATOMIC_FP32, OP>), dim3(p.G), dim3(kBlock), 0, s,
                         p);
      break;
    case PIC_DEP_ATOMIC_FP64:
      hipLaunchKernelGGL((field_init_kernel<PIC_DEP_ATOMIC_FP64, OP>), dim3(p.G), dim3(kBlock), 0, s,
                         p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(field_check0_kernel, dim3(1), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_field_init(int deposit, const FieldParams &p, hipStream_t s) {
  if (p.ife) return field_init<kOpIFE>(deposit, p, s);
  return p.iface ? field_init<kOpIF>(deposit, p, s) : field_init<kOpFV>(deposit, p, s);
}

// z = V-cycle(r); the partial r.z to part[prz]. O0: the operator of the fine
// level, OC: of the coarser ones.
template <int O0, int OC>
static void field_vcycle(const FieldParams &p, int prz, hipStream_t s) {
  const int L = p.levels;
  for (int l = 0; l + 1 < L; ++l) {
    if (l == 0) {
      if constexpr (O0 == kOpIFE)
        hipLaunchKernelGGL(mg_e1_kernel, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
      hipLaunchKernelGGL(mg_pre_kernel<O0>, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
      hipLaunchKernelGGL(mg_res_kernel<O0>, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
    } else {
      hipLaunchKernelGGL(mg_pre_kernel<OC>, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
      hipLaunchKernelGGL(mg_res_kernel<OC>, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
    }
    hipLaunchKernelGGL(mg_restrict_kernel, dim3(p.lv[l + 1].G), dim3(kBlock), 0, s, p, l);
  }
  const int gc = p.m > 0 ? (p.m + kBlock / 64 - 1) / (kBlock / 64) : 1;
  hipLaunchKernelGGL(mg_coarse_kernel, dim3(gc), dim3(kBlock), 0, s, p);
  for (int l = L - 2; l >= 0; --l) {
    hipLaunchKernelGGL(mg_prolong_kernel, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
    if (l == 0) {  // the r.z partials: the fine grid's workgroups
      hipLaunchKernelGGL((mg_sweep_kernel<false, O0>), dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l,
                         1, 0);
      hipLaunchKernelGGL((mg_sweep_kernel<true, O0>), dim3(p.G), dim3(kBlock), 0, s, p, l, 0,
                         prz);
    } else {
      hipLaunchKernelGGL((mg_sweep_kernel<false, OC>), dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l,
                         1, 0);
      hipLaunchKernelGGL((mg_sweep_kernel<false, OC>), dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l,
                         0, 0);
    }
  }
}

template <int O0, int OC>
static hipError_t field_start(const FieldParams &p, hipStream_t s) {
  field_vcycle<O0, OC>(p, 1, s);
  hipLaunchKernelGGL(field_pstart_kernel, dim3(p.G), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_field_mg_start(const FieldParams &p, hipStream_t s) {
  if (p.ife) return p.iface ? field_start<kOpIFE, kOpIF>(p, s) : field_start<kOpIFE, kOpFV>(p, s);
  return p.iface ? field_start<kOpIF, kOpIF>(p, s) : field_start<kOpFV, kOpFV>(p, s);
}

template <int O0, int OC>
static hipError_t field_iter(const FieldParams &p, int o, hipStream_t s) {
  hipLaunchKernelGGL(field_apply_kernel<O0>, dim3(p.G), dim3(kBlock), 0, s, p);
  if (p.levels >= 2) {
    hipLaunchKernelGGL((field_update_kernel<false, O0>), dim3(p.G), dim3(kBlock), 0, s, p, o);
    hipLaunchKernelGGL(field_check_kernel, dim3(1), dim3(kBlock), 0, s, p, o);
    field_vcycle<O0, OC>(p, 2 - o, s);  // parity n = 1 - o
    hipLaunchKernelGGL(field_dir_kernel<false>, dim3(p.G), dim3(kBlock), 0, s, p, o);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((field_update_kernel<true, O0>), dim3(p.G), dim3(kBlock), 0, s, p, o);
  hipLaunchKernelGGL(field_dir_kernel<true>, dim3(p.G), dim3(kBlock), 0, s, p, o);
  return hipGetLastError();
}

hipError_t launch_field_iter(const FieldParams &p, int o, hipStream_t s) {
  if (p.ife) return p.iface ? field_iter<kOpIFE, kOpIF>(p, o, s) : field_iter<kOpIFE, kOpFV>(p, o, s);
  return p.iface ? field_iter<kOpIF, kOpIF>(p, o, s) : field_iter<kOpFV, kOpFV>(p, o, s);
}

hipError_t launch_field_psi(const FieldParams &p, int l, hipStream_t s) {
  hipLaunchKernelGGL(field_psi_kernel, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
  return hipGetLastError();
}

hipError_t launch_field_diag(const FieldParams &p, int l, hipStream_t s) {
  hipLaunchKernelGGL(field_diag_kernel, dim3(p.lv[l].G), dim3(kBlock), 0, s, p, l);
  return hipGetLastError();
}

hipError_t launch_ife_mark(const FieldParams &p, int32_t *srow, int32_t *count, hipStream_t s) {
  hipLaunchKernelGGL(ife_mark_kernel, dim3(p.lv[0].G), dim3(kBlock), 0, s, p, srow, count);
  return hipGetLastError();
}

hipError_t launch_ife_rows(const FieldParams &p, int32_t *srow, double *rows, int32_t *next,
                           double *diag, hipStream_t s) {
  hipLaunchKernelGGL(ife_rows_kernel, dim3(p.lv[0].G), dim3(kBlock), 0, s, p, srow, rows, next,
                     diag);
  return hipGetLastError();
}

hipError_t launch_surface_rho(const SurfParams &p, hipStream_t s) {
  if (p.nbins <= 0) return hipSuccess;
  hipLaunchKernelGGL(surface_rho_kernel, dim3((unsigned)((p.nbins + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_field_E(int repr, const FieldParams &p, hipStream_t s) {
  switch (repr) {
    case PIC_REPR_FP64:
      hipLaunchKernelGGL(field_E_kernel<PIC_REPR_FP64>, dim3(p.G), dim3(kBlock), 0, s, p);
      break;
    case PIC_REPR_FP32_ABS:
      hipLaunchKernelGGL(field_E_kernel<PIC_REPR_FP32_ABS>, dim3(p.G), dim3(kBlock), 0, s, p);
      break;
    default:
      hipLaunchKernelGGL(field_E_kernel<PIC_REPR_FP32_CELL>, dim3(p.G), dim3(kBlock), 0, s, p);
  }
  return hipGetLastError();
}

}  // namespace pic
