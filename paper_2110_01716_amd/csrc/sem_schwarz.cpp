// Overlapping Schwarz smoother with fast-diagonalization (FDM) local solves:
// setup of one pMG level (Implementation, pMG smoothers, eq. fdm).
//
// Each element's subdomain is its (N+1)^3 nodes plus, across each face with a
// neighbour, the neighbour's node layer one step behind the shared face (face
// data only: the edges and corners of the (N+3)^3 box stay empty). The local
// operator is the separable Laplacian on a box with the element's mean
// lengths, assembled in 1D over the element and the neighbours' adjacent
// interval pairs, with homogeneous Dirichlet conditions beyond the extension;
// a boundary face without a neighbour is Dirichlet (face node excluded) when
// all its nodes are Dirichlet, otherwise it keeps a natural end. The 1D
// generalized eigenproblems A s = lambda B s (B the diagonal GLL mass) are
// solved on the host by cyclic Jacobi rotations of B^-1/2 A B^-1/2.
//
// Face neighbours are found from the four corner global IDs of every face;
// the same corners give the orientation of the neighbour's face, from which
// the gather (extension) and pull (overlap return) index maps follow as
// affine functions of the face-local coordinates (stored as 8 ints per face).
//
// Weights: ASM uses 1 / c with the counting function c = sum_e R_e^T R_e 1
// (computed by the same kernels with the local solve replaced by the
// identity); RAS keeps only each element's own nodes and averages the copies
// of shared nodes (1 / multiplicity).
#include <algorithm>
#include <array>
#include <cmath>
#include <exception>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sem_internal.h"

namespace sem {
namespace {

struct QuadHash {
  size_t operator()(const std::array<int64_t, 4>& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : k) {
      h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

// element corner (bits i, j, k) of face f's corner q, q = u + 2 v with u, v in {0, 1} (0 or N)
int face_corner(int f, int q) {
  const int axis = f >> 1, side = f & 1, u = q & 1, v = q >> 1;
  int i, j, k;
  if (axis == 0) { i = side; j = u; k = v; }
  else if (axis == 1) { i = u; j = side; k = v; }
  else { i = u; j = v; k = side; }
  return i | (j << 1) | (k << 2);
}

// local index of face-local node (u, v) at `depth`: base + u su + v sv
void face_affine(int N, int f, int depth, int& base, int& su, int& sv) {
  const int NP = N + 1, NP2 = NP * NP, axis = f >> 1, side = f & 1;
  const int d = side ? N - depth : depth;
  if (axis == 0) { base = d; su = NP; sv = NP2; }
  else if (axis == 1) { base = NP * d; su = 1; sv = NP2; }
  else { base = NP2 * d; su = 1; sv = NP; }
}

void jacobi_eigen(int n, std::vector<double>& C, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  double frob = 0.0;
  for (double c : C) frob += c * c;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += C[(size_t)p * n + q] * C[(size_t)p * n + q];
    if (off <= 1e-32 * frob) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = C[(size_t)p * n + p], aqq = C[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double ckp = C[(size_t)k * n + p], ckq = C[(size_t)k * n + q];
          C[(size_t)k * n + p] = c * ckp - s * ckq;
          C[(size_t)k * n + q] = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double cpk = C[(size_t)p * n + k], cqk = C[(size_t)q * n + k];
          C[(size_t)p * n + k] = c * cpk - s * cqk;
          C[(size_t)q * n + k] = s * cpk + c * cqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

struct Ref1D {
  int N;
  std::vector<double> w, Ahat;  // GLL weights, Dhat^T W Dhat
};

Ref1D ref1d(int N) {
  Ref1D r;
  r.N = N;
  const int NP = N + 1;
  std::vector<double> x(NP), D((size_t)NP * NP);
  r.w.resize(NP);
  gll_points(N, x.data(), r.w.data());
  deriv_matrix(N, D.data());
  r.Ahat.assign((size_t)NP * NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      double s = 0.0;
      for (int q = 0; q < NP; ++q) s += r.w[q] * D[(size_t)q * NP + i] * D[(size_t)q * NP + j];
      r.Ahat[(size_t)i * NP + j] = s;
    }
  return r;
}

// kinds: 0 neighbour, 1 Dirichlet, 2 Neumann. S: NE x NE (row ext index, column mode), lam: NE
void fdm_1d(const Ref1D& R, int kl, int kr, double ll, double lm, double lr, double* S, double* lam) {
  const int N = R.N, NP = N + 1, NE = N + 3;
  std::vector<double> A((size_t)NE * NE, 0.0), B(NE, 0.0);
  for (int i = 0; i < NP; ++i) {
    B[i + 1] += 0.5 * lm * R.w[i];
    for (int j = 0; j < NP; ++j) A[(size_t)(i + 1) * NE + (j + 1)] += (2.0 / lm) * R.Ahat[(size_t)i * NP + j];
  }
  if (kl == 0)
    for (int i = 0; i < 2; ++i) {
      B[i] += 0.5 * ll * R.w[N - 1 + i];
      for (int j = 0; j < 2; ++j) A[(size_t)i * NE + j] += (2.0 / ll) * R.Ahat[(size_t)(N - 1 + i) * NP + (N - 1 + j)];
    }
  if (kr == 0)
    for (int i = 0; i < 2; ++i) {
      B[N + 1 + i] += 0.5 * lr * R.w[i];
      for (int j = 0; j < 2; ++j) A[(size_t)(N + 1 + i) * NE + (N + 1 + j)] += (2.0 / lr) * R.Ahat[(size_t)i * NP + j];
    }
  const int lo = kl == 0 ? 0 : kl == 1 ? 2 : 1;
  const int hi = kr == 0 ? N + 2 : kr == 1 ? N : N + 1;
  std::fill(S, S + (size_t)NE * NE, 0.0);
  std::fill(lam, lam + NE, 1.0);
  const int n = hi - lo + 1;
  if (n <= 0) return;
  std::vector<double> C((size_t)n * n), V;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      C[(size_t)i * n + j] = A[(size_t)(lo + i) * NE + (lo + j)] / std::sqrt(B[lo + i] * B[lo + j]);
  jacobi_eigen(n, C, V);
  for (int m = 0; m < n; ++m) {
    lam[lo + m] = C[(size_t)m * n + m];
    for (int i = 0; i < n; ++i) S[(size_t)(lo + i) * NE + (lo + m)] = V[(size_t)i * n + m] / std::sqrt(B[lo + i]);
  }
}

template <typename T>
void apply_t(const MeshData& m, const SchwarzData& sw, int mode, const T* r, T* z, T* ovl, const T* S, const T* L,
             hipStream_t s) {
  Table<SchwarzArgs<T>> t;
  t.one.E = m.E;
  t.one.in = r;
  t.one.out = z;
  t.one.ovl = sw.ras ? nullptr : ovl;
  t.one.desc = sw.desc.as<int>();
  t.one.S = S;
  t.one.lam = L;
  launch_schwarz<T>(m.N, mode, t, schwarz_blocks(m.E), s);
  if (!sw.ras) {
    Table<SchwarzPullArgs<T>> tp;
    tp.one.E = m.E;
    tp.one.out = z;
    tp.one.ovl = ovl;
    tp.one.desc = sw.desc.as<int>();
    launch_schwarz_pull<T>(m.N, tp, schwarz_blocks(m.E), s);
  }
}

}  // namespace

void schwarz_setup(const MeshData& m, bool ras, SchwarzData& sw, hipStream_t s) {
  const int N = m.N, NP = N + 1, NP2 = NP * NP, NE = N + 3;
  const int64_t E = m.E;
  if (N < 2 || N > kMaxN) fail(SEM_EINVAL, "Schwarz smoother: order N=%d outside [2,%d]", N, kMaxN);
  // per-element corners, Dirichlet faces, lengths
  DevBuf corners, fdir, lens;
  corners.alloc(sizeof(int64_t) * 8 * E);
  fdir.alloc(6 * E);
  lens.alloc(sizeof(double) * 3 * E);
  SchwarzInfoArgs ia;
  ia.N = N;
  ia.E = E;
  ia.x = m.x.as<double>();
  ia.y = m.y.as<double>();
  ia.z = m.z.as<double>();
  ia.gid = m.gid.as<int64_t>();
  ia.dmask = m.dmask.as<uint8_t>();
  ia.corners = corners.as<int64_t>();
  ia.face_dir = fdir.as<uint8_t>();
  ia.lengths = lens.as<double>();
  launch_schwarz_info(ia, s);
  std::vector<int64_t> hc(8 * E);
  std::vector<uint8_t> hf(6 * E);
  std::vector<double> hl(3 * E);
  SEM_HIP(hipMemcpyAsync(hc.data(), corners.p, sizeof(int64_t) * 8 * E, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipMemcpyAsync(hf.data(), fdir.p, 6 * E, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipMemcpyAsync(hl.data(), lens.p, sizeof(double) * 3 * E, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));

  // face neighbours from the sorted corner IDs
  auto face_key = [&](int64_t e, int f) {
    std::array<int64_t, 4> k;
    for (int q = 0; q < 4; ++q) k[q] = hc[e * 8 + face_corner(f, q)];
    std::sort(k.begin(), k.end());
    return k;
  };
  std::unordered_map<std::array<int64_t, 4>, std::array<int64_t, 2>, QuadHash> first;
  first.reserve((size_t)(6 * E));
  std::vector<int64_t> nbr(6 * E, -1);
  std::vector<int> nface(6 * E, -1);
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      const auto k = face_key(e, f);
      if (k[0] == k[1] || k[1] == k[2] || k[2] == k[3])
        fail(SEM_EINVAL, "Schwarz smoother: element %lld face %d has repeated corner IDs", (long long)e, f);
      auto it = first.find(k);
      if (it == first.end()) {
        first.emplace(k, std::array<int64_t, 2>{e, f});
      } else {
        const int64_t e2 = it->second[0];
        const int f2 = (int)it->second[1];
        if (nbr[e2 * 6 + f2] >= 0) fail(SEM_EINVAL, "Schwarz smoother: a face is shared by more than two elements");
        nbr[e * 6 + f] = e2;
        nface[e * 6 + f] = f2;
        nbr[e2 * 6 + f2] = e;
        nface[e2 * 6 + f2] = f;
      }
    }

  // descriptors
  std::vector<int> desc(48 * E);
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      int* d = &desc[(e * 6 + f) * 8];
      const int64_t n = nbr[e * 6 + f];
      if (n < 0) {
        d[0] = -1;
        for (int q = 1; q < 7; ++q) d[q] = 0;
        d[7] = hf[e * 6 + f] ? 1 : 2;
        continue;
      }
      const int fn = nface[e * 6 + f];
      int uq[3], vq[3];  // neighbour face coords (in units of N) of this face's corners (0,0), (N,0), (0,N)
      for (int q = 0; q < 3; ++q) {
        const int64_t g = hc[e * 8 + face_corner(f, q)];
        int hit = -1;
        for (int q2 = 0; q2 < 4; ++q2)
          if (hc[n * 8 + face_corner(fn, q2)] == g) hit = q2;
        if (hit < 0) fail(SEM_EINVAL, "Schwarz smoother: inconsistent face corners");
        uq[q] = hit & 1;
        vq[q] = hit >> 1;
      }
      const int du_u = uq[1] - uq[0], du_v = vq[1] - vq[0], dv_u = uq[2] - uq[0], dv_v = vq[2] - vq[0];
      if (std::abs(du_u) + std::abs(du_v) != 1 || std::abs(dv_u) + std::abs(dv_v) != 1 || du_u * dv_u + du_v * dv_v != 0)
        fail(SEM_EINVAL, "Schwarz smoother: element %lld face %d is twisted against its neighbour", (long long)e, f);
      int base, su, sv;
      face_affine(N, fn, 1, base, su, sv);
      const int u0 = uq[0] * N, v0 = vq[0] * N;
      d[0] = (int)n;
      d[1] = base + u0 * su + v0 * sv;
      d[2] = du_u * su + du_v * sv;
      d[3] = dv_u * su + dv_v * sv;
      d[4] = fn * NP2 + v0 * NP + u0;
      d[5] = du_u + du_v * NP;
      d[6] = dv_u + dv_v * NP;
      d[7] = 0;
      // the maps are affine in (u, v): checking the four corners bounds every index
      for (int cu = 0; cu <= N; cu += N)
        for (int cv = 0; cv <= N; cv += N) {
          const int gi = d[1] + cu * d[2] + cv * d[3], pi = d[4] + cu * d[5] + cv * d[6];
          if (gi < 0 || gi >= NP2 * NP || pi < 0 || pi >= 6 * NP2)
            fail(SEM_EINVAL, "Schwarz smoother: extension map out of range at element %lld face %d", (long long)e, f);
        }
    }
  sw.desc.alloc(sizeof(int) * desc.size());
  SEM_HIP(hipMemcpyAsync(sw.desc.p, desc.data(), sizeof(int) * desc.size(), hipMemcpyHostToDevice, s));

  // 1D fast-diagonalization data per element and direction
  const Ref1D R = ref1d(N);
  const size_t per = (size_t)3 * NE * NE;
  std::vector<double> S64(per * E), L64((size_t)3 * NE * E);
  auto work = [&](int64_t e0, int64_t e1) {
    for (int64_t e = e0; e < e1; ++e)
      for (int axis = 0; axis < 3; ++axis) {
        const int fl = 2 * axis, fr = 2 * axis + 1;
        const int* dl = &desc[(e * 6 + fl) * 8];
        const int* dr = &desc[(e * 6 + fr) * 8];
        const double lm = hl[e * 3 + axis];
        const double ll = dl[7] == 0 ? hl[nbr[e * 6 + fl] * 3 + (nface[e * 6 + fl] >> 1)] : lm;
        const double lr = dr[7] == 0 ? hl[nbr[e * 6 + fr] * 3 + (nface[e * 6 + fr] >> 1)] : lm;
        fdm_1d(R, dl[7], dr[7], ll, lm, lr, &S64[per * e + (size_t)axis * NE * NE], &L64[((size_t)3 * e + axis) * NE]);
      }
  };
  const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(16, std::min<int64_t>(E / 64 + 1,
                                                       (int64_t)std::thread::hardware_concurrency())));
  // an exception in a worker (allocation) is carried back and rethrown here,
  // so it becomes the call's error status instead of ending the process
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> err(nth);
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t] {
      try {
        work(E * t / nth, E * (t + 1) / nth);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  std::vector<float> S32(S64.begin(), S64.end()), L32(L64.begin(), L64.end());
  sw.S64.alloc(sizeof(double) * S64.size());
  sw.L64.alloc(sizeof(double) * L64.size());
  sw.S32.alloc(sizeof(float) * S32.size());
  sw.L32.alloc(sizeof(float) * L32.size());
  SEM_HIP(hipMemcpyAsync(sw.S64.p, S64.data(), sizeof(double) * S64.size(), hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemcpyAsync(sw.L64.p, L64.data(), sizeof(double) * L64.size(), hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemcpyAsync(sw.S32.p, S32.data(), sizeof(float) * S32.size(), hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemcpyAsync(sw.L32.p, L32.data(), sizeof(float) * L32.size(), hipMemcpyHostToDevice, s));

  // weights
  sw.ras = ras;
  const int64_t n = m.nloc;
  DevBuf ones, cnt, ovl;
  ones.alloc(sizeof(double) * n);
  cnt.alloc(sizeof(double) * n);
  ovl.alloc(sizeof(double) * 6 * NP2 * E);
  vec_op1(V_FILL, n, ones.as<double>(), nullptr, 1.0, nullptr, s);
  if (ras) {
    SEM_HIP(hipMemcpyAsync(cnt.p, ones.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  } else {
    apply_t<double>(m, sw, 1, ones.as<double>(), cnt.as<double>(), ovl.as<double>(), nullptr, nullptr, s);
  }
  mesh_gs(m, SEM_F64, cnt.p, 1, s);
  sw.w64.alloc(sizeof(double) * n);
  sw.w32.alloc(sizeof(float) * n);
  vec_op1(V_DIV_DINV, n, sw.w64.as<double>(), ones.as<double>(), 0.0, cnt.as<double>(), s);
  Table<CastArgs<double, float>> tc;
  tc.one.n = n;
  tc.one.in = sw.w64.as<double>();
  tc.one.out = sw.w32.as<float>();
  launch_cast<double, float>(tc, vec_blocks(n), s);
  SEM_HIP(hipStreamSynchronize(s));
  sw.on = true;
}

void schwarz_apply(const MeshData& m, const SchwarzData& sw, sem_dtype t, const void* r, void* z, void* tmp_ovl,
                   hipStream_t s) {
  if (!sw.on) fail(SEM_EINVAL, "Schwarz smoother: level has no Schwarz data");
  if (t == SEM_F64) {
    apply_t<double>(m, sw, 0, (const double*)r, (double*)z, (double*)tmp_ovl, sw.S64.as<double>(),
                    sw.L64.as<double>(), s);
    mesh_gs(m, SEM_F64, z, 1, s);
    vec_op1(V_SCALE_DINV, m.nloc, (double*)z, (const double*)z, 0.0, sw.w64.as<double>(), s);
  } else {
    apply_t<float>(m, sw, 0, (const float*)r, (float*)z, (float*)tmp_ovl, sw.S32.as<float>(), sw.L32.as<float>(),
                   s);
    mesh_gs(m, SEM_F32, z, 1, s);
    Table<VecArgs<float>> tv;
    tv.one.n = m.nloc;
    tv.one.x = (float*)z;
    tv.one.r = (float*)z;
    tv.one.dinv = sw.w32.as<float>();
    launch_vec<float>(V_SCALE_DINV, tv, vec_blocks(m.nloc), s);
  }
}

}  // namespace sem
