// p-multigrid hierarchy setup (Implementation, pMG paragraph).
//
// For each coarser order N_c of the schedule:
//   * coarse nodal coordinates: each element's fine isoparametric map
//     evaluated at the coarse GLL points, X_c = (Jcf x Jcf x Jcf) X_f;
//   * coarse global IDs: every coarse node is keyed by the mesh entity it lies
//     on, using only fine global IDs, so any conforming numbering and element
//     orientation works:
//       vertex    -> the fine ID of that vertex;
//       edge      -> the IDs of the two fine edge nodes next to the ends, plus
//                    the position counted from the end with the smaller ID;
//       face      -> the smallest ID among the four fine face nodes next to the
//                    face corners, plus the position in a frame anchored at
//                    that corner whose first axis points to the smaller of its
//                    two neighbours;
//       interior  -> (element, position);
//     equal keys get equal coarse IDs;
//   * coarse Dirichlet flag: that of a fine node on the same entity;
//   * geometric factors, gather-scatter map and Jacobi diagonal as for a user
//     mesh (re-discretised SEM operator at order N_c);
//   * rho = largest eigenvalue estimate of D^-1 A by power iteration from a
//     splitmix64 start vector keyed by global ID, and the Chebyshev
//     coefficients on [lo rho, hi rho].
#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <numeric>

#include "sem_internal.h"

namespace sem {

void chebyshev_coefficients(PmgLevel& lv, double lo, double hi, int degree) {
  const double a = lo * lv.rho, b = hi * lv.rho;
  lv.theta = 0.5 * (b + a);
  lv.delta = 0.5 * (b - a);
  const double sigma = lv.theta / lv.delta;
  double r0 = 1.0 / sigma;
  lv.c1.clear();
  lv.c2.clear();
  for (int j = 1; j < degree; ++j) {
    const double r1 = 1.0 / (2.0 * sigma - r0);
    lv.c1.push_back(r1 * r0);
    lv.c2.push_back(2.0 * r1 / lv.delta);
    r0 = r1;
  }
}

namespace {

struct Key {
  std::array<int64_t, 4> k;
  bool operator<(const Key& o) const { return k < o.k; }
  bool operator==(const Key& o) const { return k == o.k; }
};

// coarse IDs and Dirichlet flags from the fine level (host)
void coarse_ids(int Nf, int Nc, int64_t E, const std::vector<int64_t>& gf, const std::vector<uint8_t>& df,
                std::vector<int64_t>& gc, std::vector<uint8_t>& dc) {
  const int nf = Nf + 1, nc = Nc + 1;
  const int64_t npf = (int64_t)nf * nf * nf, npc = (int64_t)nc * nc * nc;
  const int64_t n = E * npc;
  std::vector<Key> keys(n);
  dc.assign(n, 0);
  auto fidx = [&](int i, int j, int k) { return (int64_t)i + nf * (j + (int64_t)nf * k); };
  for (int64_t e = 0; e < E; ++e) {
    const int64_t* g = gf.data() + e * npf;
    const uint8_t* d = df.data() + e * npf;
    for (int kc = 0; kc < nc; ++kc)
      for (int jc = 0; jc < nc; ++jc)
        for (int ic = 0; ic < nc; ++ic) {
          const int c[3] = {ic, jc, kc};
          int cls[3], fb[3], rep[3];
          int nint = 0, dint[3];
          for (int a = 0; a < 3; ++a) {
            cls[a] = (c[a] == 0) ? 0 : (c[a] == Nc ? 2 : 1);
            fb[a] = (cls[a] == 0) ? 0 : Nf;
            rep[a] = (cls[a] == 1) ? 1 : fb[a];
            if (cls[a] == 1) dint[nint++] = a;
          }
          const int64_t lc = e * npc + ic + (int64_t)nc * (jc + (int64_t)nc * kc);
          Key key{{0, 0, 0, 0}};
          if (nint == 0) {
            key.k = {0, g[fidx(fb[0], fb[1], fb[2])], 0, 0};
          } else if (nint == 1) {
            const int a = dint[0];
            int pA[3] = {fb[0], fb[1], fb[2]}, pB[3] = {fb[0], fb[1], fb[2]};
            pA[a] = 1;
            pB[a] = Nf - 1;
            const int64_t gA = g[fidx(pA[0], pA[1], pA[2])], gB = g[fidx(pB[0], pB[1], pB[2])];
            const int pos = (gA < gB) ? c[a] : Nc - c[a];
            key.k = {1, std::min(gA, gB), std::max(gA, gB), pos};
          } else if (nint == 2) {
            const int a1 = dint[0], a2 = dint[1];
            int64_t corner[2][2];
            for (int al = 0; al < 2; ++al)
              for (int be = 0; be < 2; ++be) {
                int p[3] = {fb[0], fb[1], fb[2]};
                p[a1] = al ? Nf - 1 : 1;
                p[a2] = be ? Nf - 1 : 1;
                corner[al][be] = g[fidx(p[0], p[1], p[2])];
              }
            int al = 0, be = 0;
            for (int x = 0; x < 2; ++x)
              for (int y = 0; y < 2; ++y)
                if (corner[x][y] < corner[al][be]) { al = x; be = y; }
            const int pa = al ? Nc - c[a1] : c[a1];
            const int pb = be ? Nc - c[a2] : c[a2];
            const int64_t ga = corner[1 - al][be], gb = corner[al][1 - be];
            const int p1 = (ga < gb) ? pa : pb, p2 = (ga < gb) ? pb : pa;
            key.k = {2, corner[al][be], p1, p2};
          } else {
            key.k = {3, e, ic + (int64_t)nc * (jc + (int64_t)nc * kc), 0};
          }
          keys[lc] = key;
          dc[lc] = d[fidx(rep[0], rep[1], rep[2])];
        }
  }
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  gc.assign(n, 0);
  int64_t id = -1;
  for (int64_t q = 0; q < n; ++q) {
    if (q == 0 || !(keys[order[q]] == keys[order[q - 1]])) ++id;
    gc[order[q]] = id;
  }
}

// FP64 vector helpers on one mesh (setup only)
void vec1(const MeshData& m, VecOp op, double* x, const double* r, double c0, hipStream_t s) {
  Table<VecArgs<double>> t;
  t.one.n = m.nloc;
  t.one.x = x;
  t.one.r = const_cast<double*>(r);
  t.one.dinv = m.dinv64.as<double>();
  t.one.c0 = c0;
  launch_vec<double>(op, t, vec_blocks(m.nloc), s);
}

double power_rho(const MeshData& m, int iters, hipStream_t s) {
  DevBuf v, w;
  v.alloc(sizeof(double) * m.nloc);
  w.alloc(sizeof(double) * m.nloc);
  launch_start_vector(m.nloc, m.gid.as<int64_t>(), m.dmask.as<uint8_t>(), v.as<double>(), s);
  double nrm = std::sqrt(mesh_dot(m, SEM_F64, v.p, v.p, s));
  if (!(nrm > 0)) return 1.0;  // all nodes Dirichlet
  vec1(m, V_SCALE, v.as<double>(), v.as<double>(), 1.0 / nrm, s);
  for (int it = 0; it < iters; ++it) {
    apply_A(m, SEM_F64, v.p, w.p, s);
    vec1(m, V_SCALE_DINV, v.as<double>(), w.as<double>(), 0.0, s);
    nrm = std::sqrt(mesh_dot(m, SEM_F64, v.p, v.p, s));
    vec1(m, V_SCALE, v.as<double>(), v.as<double>(), 1.0 / nrm, s);
  }
  apply_A(m, SEM_F64, v.p, w.p, s);
  const double num = mesh_dot(m, SEM_F64, v.p, w.p, s);
  vec1(m, V_DIV_DINV, w.as<double>(), v.as<double>(), 0.0, s);
  const double den = mesh_dot(m, SEM_F64, v.p, w.p, s);
  return num / den;
}

// rho of W S A (Schwarz smoother): |M A v| after normalised power iterations
double power_rho_schwarz(const MeshData& m, const SchwarzData& sw, int iters, hipStream_t s) {
  DevBuf v, w, ovl;
  v.alloc(sizeof(double) * m.nloc);
  w.alloc(sizeof(double) * m.nloc);
  ovl.alloc(sizeof(double) * 6 * (m.N + 1) * (m.N + 1) * m.E);
  launch_start_vector(m.nloc, m.gid.as<int64_t>(), m.dmask.as<uint8_t>(), v.as<double>(), s);
  double nrm = std::sqrt(mesh_dot(m, SEM_F64, v.p, v.p, s));
  if (!(nrm > 0)) return 1.0;
  vec1(m, V_SCALE, v.as<double>(), v.as<double>(), 1.0 / nrm, s);
  for (int it = 0; it <= iters; ++it) {
    apply_A(m, SEM_F64, v.p, w.p, s);
    schwarz_apply(m, sw, SEM_F64, w.p, v.p, ovl.p, s);
    nrm = std::sqrt(mesh_dot(m, SEM_F64, v.p, v.p, s));
    if (it == iters) break;
    vec1(m, V_SCALE, v.as<double>(), v.as<double>(), 1.0 / nrm, s);
  }
  return nrm;
}

void upload_matrix(DevBuf& dst, const std::vector<double>& h, hipStream_t s) {
  dst.alloc(sizeof(double) * h.size());
  SEM_HIP(hipMemcpyAsync(dst.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
}

}  // namespace
}  // namespace sem

using namespace sem;

extern "C" void sem_pmg_opts_default(sem_pmg_opts* o) {
  if (!o) return;
  *o = sem_pmg_opts{};
  o->n_levels = 0;
  o->smoother_dtype = SEM_F32;
  o->cheb_degree = 2;
  o->pre = 1;
  o->post = 1;
  o->eig_lo = 0.1;
  o->eig_hi = 1.1;
  o->power_iters = 20;
  o->rho_override = nullptr;
  o->coarse_rtol = 1e-2;
  o->coarse_maxit = 500;
  o->coarse_fixed_iters = 0;
  o->coarse_check_every = 8;
  o->smoother = SEM_SMOOTH_CHEB_JACOBI;
}

extern "C" int sem_pmg_setup(sem_mesh mh, const sem_pmg_opts* oin, sem_pmg* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!mh || !out) fail(SEM_EINVAL, "sem_pmg_setup: NULL argument");
    sem_pmg_opts o;
    if (oin) o = *oin; else sem_pmg_opts_default(&o);
    const int N = mh->d.N;
    auto P = std::make_unique<sem_pmg_s>();
    P->base = mh;
    P->o = o;
    if (o.n_levels == 0) {
      const int mid = (N - 1) / 2;
      if (mid > 1 && mid < N) {
        P->n_levels = 3;
        P->orders[0] = N; P->orders[1] = mid; P->orders[2] = 1;
      } else {
        P->n_levels = 2;
        P->orders[0] = N; P->orders[1] = 1;
      }
    } else {
      if (o.n_levels < 2 || o.n_levels > kMaxLevels)
        fail(SEM_EINVAL, "sem_pmg_setup: n_levels=%d outside [2,%d]", o.n_levels, kMaxLevels);
      P->n_levels = o.n_levels;
      for (int l = 0; l < o.n_levels; ++l) P->orders[l] = o.orders[l];
    }
    if (N < 2) fail(SEM_EINVAL, "sem_pmg_setup: the mesh order must be >= 2");
    if (P->orders[0] != N) fail(SEM_EINVAL, "sem_pmg_setup: orders[0]=%d differs from the mesh order %d", P->orders[0], N);
    if (P->orders[P->n_levels - 1] != 1) fail(SEM_EINVAL, "sem_pmg_setup: the last order must be 1");
    for (int l = 1; l < P->n_levels; ++l)
      if (P->orders[l] >= P->orders[l - 1] || P->orders[l] < 1)
        fail(SEM_EINVAL, "sem_pmg_setup: orders must strictly decrease");
    if (o.smoother_dtype != SEM_F32 && o.smoother_dtype != SEM_F64) fail(SEM_EINVAL, "sem_pmg_setup: bad smoother dtype");
    if (o.cheb_degree < 1 || o.cheb_degree > 16) fail(SEM_EINVAL, "sem_pmg_setup: cheb_degree outside [1,16]");
    if (o.pre < 0 || o.post < 0 || o.pre + o.post < 1) fail(SEM_EINVAL, "sem_pmg_setup: need pre + post >= 1");
    if (!(o.eig_hi > o.eig_lo) || !(o.eig_lo > 0)) fail(SEM_EINVAL, "sem_pmg_setup: need 0 < eig_lo < eig_hi");
    if (o.coarse_maxit < 1) fail(SEM_EINVAL, "sem_pmg_setup: coarse_maxit < 1");
    if (o.smoother < SEM_SMOOTH_CHEB_JACOBI || o.smoother > SEM_SMOOTH_CHEB_RAS)
      fail(SEM_EINVAL, "sem_pmg_setup: unknown smoother %d", o.smoother);
    if (o.coarse_check_every < 1) P->o.coarse_check_every = 8;
    // every transfer pair must have a kernel
    for (int l = 0; l + 1 < P->n_levels; ++l) (void)xfer_blocks(P->orders[l], P->orders[l + 1], 1);

    hipStream_t s = nullptr;
    P->lv.resize(P->n_levels);
    P->lv[0].mesh = mh;
    for (int l = 1; l < P->n_levels; ++l) {
      const MeshData& f = P->lv[l - 1].mesh->d;
      const int Nf = f.N, Nc = P->orders[l];
      std::vector<double> xf(Nf + 1), xc(Nc + 1);
      gll_points(Nf, xf.data(), nullptr);
      gll_points(Nc, xc.data(), nullptr);
      // fine map at coarse points
      std::vector<double> Jcf((Nc + 1) * (Nf + 1));
      lagrange_matrix(Nf + 1, xf.data(), Nc + 1, xc.data(), Jcf.data());
      DevBuf dJcf;
      upload_matrix(dJcf, Jcf, s);
      auto cm = new sem_mesh_s();
      P->owned.push_back(cm);
      cm->owned_by_pmg = true;
      MeshData& c = cm->d;
      const int64_t npc = (int64_t)(Nc + 1) * (Nc + 1) * (Nc + 1);
      c.x.alloc(sizeof(double) * f.E * npc);
      c.y.alloc(sizeof(double) * f.E * npc);
      c.z.alloc(sizeof(double) * f.E * npc);
      launch_tensor_coords(Nf, Nc, f.E, f.x.as<double>(), c.x.as<double>(), dJcf.as<double>(), s);
      launch_tensor_coords(Nf, Nc, f.E, f.y.as<double>(), c.y.as<double>(), dJcf.as<double>(), s);
      launch_tensor_coords(Nf, Nc, f.E, f.z.as<double>(), c.z.as<double>(), dJcf.as<double>(), s);
      std::vector<int64_t> gf(f.nloc), gc;
      std::vector<uint8_t> df(f.nloc), dc;
      SEM_HIP(hipMemcpyAsync(gf.data(), f.gid.p, sizeof(int64_t) * f.nloc, hipMemcpyDeviceToHost, s));
      SEM_HIP(hipMemcpyAsync(df.data(), f.dmask.p, f.nloc, hipMemcpyDeviceToHost, s));
      SEM_HIP(hipStreamSynchronize(s));
      coarse_ids(Nf, Nc, f.E, gf, df, gc, dc);
      build_mesh(c, Nc, f.E, gc.data(), dc.data(), s);
      if (l + 1 == P->n_levels) build_assembled(c, s);  // coarse solve on unique DOFs
      P->lv[l].mesh = cm;
      // prolongation J (fine x coarse) and restriction J^T for the pair (l-1, l)
      std::vector<double> J((Nf + 1) * (Nc + 1)), JT((Nc + 1) * (Nf + 1));
      lagrange_matrix(Nc + 1, xc.data(), Nf + 1, xf.data(), J.data());
      for (int i = 0; i <= Nf; ++i)
        for (int j = 0; j <= Nc; ++j) JT[j * (Nf + 1) + i] = J[i * (Nc + 1) + j];
      upload_matrix(P->lv[l - 1].J, J, s);
      upload_matrix(P->lv[l - 1].JT, JT, s);
      SEM_HIP(hipStreamSynchronize(s));
    }
    for (int l = 0; l + 1 < P->n_levels; ++l) {
      PmgLevel& lv = P->lv[l];
      if (o.smoother != SEM_SMOOTH_CHEB_JACOBI) schwarz_setup(lv.mesh->d, o.smoother == SEM_SMOOTH_CHEB_RAS, lv.sw, s);
      if (o.rho_override) lv.rho = o.rho_override[l];
      else if (lv.sw.on) lv.rho = power_rho_schwarz(lv.mesh->d, lv.sw, o.power_iters, s);
      else lv.rho = power_rho(lv.mesh->d, o.power_iters, s);
      if (!(lv.rho > 0) || !std::isfinite(lv.rho)) fail(SEM_EINVAL, "sem_pmg_setup: invalid rho %g at level %d", lv.rho, l);
      chebyshev_coefficients(lv, o.eig_lo, o.eig_hi, o.cheb_degree);
    }
    SEM_HIP(hipStreamSynchronize(s));
    *out = P.release();
  });
}

extern "C" int sem_pmg_destroy(sem_pmg p) {
  return guarded([&] { delete p; });
}

extern "C" int sem_pmg_query(sem_pmg p, sem_pmg_info* info) {
  return guarded([&] {
    if (!p || !info) fail(SEM_EINVAL, "sem_pmg_query: NULL argument");
    *info = sem_pmg_info{};
    info->n_levels = p->n_levels;
    int64_t bytes = 0;
    for (int l = 0; l < p->n_levels; ++l) {
      info->orders[l] = p->orders[l];
      info->rho[l] = p->lv[l].rho;
      info->n_unique[l] = p->lv[l].mesh->d.n_unique;
      if (l > 0) bytes += p->lv[l].mesh->d.resident_bytes();
      bytes += (int64_t)(p->lv[l].J.bytes + p->lv[l].JT.bytes);
      const SchwarzData& sw = p->lv[l].sw;
      bytes += (int64_t)(sw.desc.bytes + sw.S64.bytes + sw.L64.bytes + sw.S32.bytes + sw.L32.bytes + sw.w64.bytes +
                         sw.w32.bytes);
    }
    info->resident_bytes = bytes;
  });
}

extern "C" int sem_pmg_level(sem_pmg p, int level, sem_mesh* out) {
  return guarded([&] {
    if (!p || !out) fail(SEM_EINVAL, "sem_pmg_level: NULL argument");
    if (level < 0 || level >= p->n_levels) fail(SEM_EINVAL, "sem_pmg_level: level %d outside [0,%d)", level, p->n_levels);
    *out = p->lv[level].mesh;
  });
}

extern "C" int sem_pmg_smoother_apply(sem_pmg p, int level, const void* r, void* z, void* stream) {
  return guarded([&] {
    if (!p || !r || !z) fail(SEM_EINVAL, "sem_pmg_smoother_apply: NULL argument");
    if (level < 0 || level + 1 >= p->n_levels)
      fail(SEM_EINVAL, "sem_pmg_smoother_apply: level %d is not a smoothed level", level);
    hipStream_t s = (hipStream_t)stream;
    const PmgLevel& lv = p->lv[level];
    const MeshData& m = lv.mesh->d;
    const sem_dtype t = p->o.smoother_dtype;
    if (lv.sw.on) {
      DevBuf ovl;
      ovl.alloc((t == SEM_F64 ? 8 : 4) * (size_t)6 * (m.N + 1) * (m.N + 1) * m.E);
      schwarz_apply(m, lv.sw, t, r, z, ovl.p, s);
      SEM_HIP(hipStreamSynchronize(s));
    } else if (t == SEM_F64) {
      vec_op1(V_SCALE_DINV, m.nloc, (double*)z, (const double*)r, 0.0, m.dinv64.as<double>(), s);
    } else {
      Table<VecArgs<float>> tv;
      tv.one.n = m.nloc;
      tv.one.x = (float*)z;
      tv.one.r = (float*)const_cast<void*>(r);
      tv.one.dinv = m.dinv32.as<float>();
      launch_vec<float>(V_SCALE_DINV, tv, vec_blocks(m.nloc), s);
    }
  });
}
