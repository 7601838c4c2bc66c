// Host-sanitizer driver for libsem: exercises every host code path of the C
// ABI (mesh setup and its gather-scatter map, the pMG hierarchy with its
// entity-keyed coarse IDs, the Schwarz face maps, solves, batches, GMRES,
// projection and the error paths) on generated deformed boxes, with the host
// code of the library built under AddressSanitizer and UndefinedBehavior-
// Sanitizer (device code is not instrumented). Built by
// `python -m paper_2110_01716_amd.build_lib --sanitize`; needs a GPU to run.
// Exit status 0 when every check passes; a sanitizer report aborts it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <string>
#include <vector>

#include "sem.h"

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                  \
      std::fprintf(stderr, " (%s)\n", sem_last_error());  \
      ++g_fail;                                           \
    }                                                     \
  } while (0)

#define HIPCHECK(call)                                                       \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
      std::exit(2);                                                          \
    }                                                                        \
  } while (0)

// A box of nx x ny x nz hex elements on [0,1]^3 with order-N GLL nodes,
// lattice global IDs, Dirichlet flags on the outer faces, smoothly deformed.
struct Box {
  int N = 0;
  int64_t E = 0;
  std::vector<double> x, y, z;
  std::vector<int64_t> gid;
  std::vector<uint8_t> dir;
};

Box make_box(int nx, int ny, int nz, int N, double amp, uint64_t relabel_seed) {
  Box b;
  b.N = N;
  b.E = (int64_t)nx * ny * nz;
  const int NP = N + 1, Np = NP * NP * NP;
  std::vector<double> xi(NP);
  sem_reference(N, xi.data(), nullptr, nullptr);
  const int64_t gx = (int64_t)nx * N + 1, gy = (int64_t)ny * N + 1, gz = (int64_t)nz * N + 1;
  // optional relabelling of the lattice IDs by an affine permutation
  const int64_t ng = gx * gy * gz;
  int64_t mul = 1;
  if (relabel_seed) {
    mul = (int64_t)(relabel_seed % 1000003) * 2 + 1;
    while (std::gcd(mul, ng) != 1) mul += 2;
  }
  b.x.resize(b.E * Np);
  b.y.resize(b.E * Np);
  b.z.resize(b.E * Np);
  b.gid.resize(b.E * Np);
  b.dir.resize(b.E * Np);
  const double pi = 3.14159265358979323846;
  int64_t e = 0;
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex, ++e)
        for (int k = 0; k < NP; ++k)
          for (int j = 0; j < NP; ++j)
            for (int i = 0; i < NP; ++i) {
              const int64_t l = e * Np + i + NP * j + NP * NP * k;
              const int64_t I = (int64_t)ex * N + i, J = (int64_t)ey * N + j, K = (int64_t)ez * N + k;
              double X = (ex + 0.5 * (xi[i] + 1.0)) / nx, Y = (ey + 0.5 * (xi[j] + 1.0)) / ny,
                     Z = (ez + 0.5 * (xi[k] + 1.0)) / nz;
              if (i == 0 || i == N) X = (double)(ex + (i == N)) / nx;  // exact shared endpoints
              if (j == 0 || j == N) Y = (double)(ey + (j == N)) / ny;
              if (k == 0 || k == N) Z = (double)(ez + (k == N)) / nz;
              b.x[l] = X + amp * std::sin(2 * pi * Y) * std::sin(2 * pi * Z);
              b.y[l] = Y + amp * std::sin(2 * pi * Z) * std::sin(2 * pi * X);
              b.z[l] = Z + amp * std::sin(2 * pi * X) * std::sin(2 * pi * Y);
              const int64_t g = I + gx * (J + gy * K);
              b.gid[l] = relabel_seed ? (g * mul) % ng : g;
              b.dir[l] = (I == 0 || J == 0 || K == 0 || I == gx - 1 || J == gy - 1 || K == gz - 1) ? 1 : 0;
            }
  return b;
}

sem_mesh create(const Box& b) {
  sem_mesh_desc d{};
  d.N = b.N;
  d.E = b.E;
  d.x = b.x.data();
  d.y = b.y.data();
  d.z = b.z.data();
  d.gid = b.gid.data();
  d.dirichlet = b.dir.data();
  sem_mesh m = nullptr;
  const int rc = sem_mesh_create(&d, &m);
  CHECK(rc == SEM_OK && m, "sem_mesh_create N=%d E=%lld rc=%d", b.N, (long long)b.E, rc);
  return m;
}

// consistent masked right-hand side: one value per global ID (hashed), copied to every copy
std::vector<double> rhs(const Box& b, uint64_t seed) {
  std::vector<double> r(b.gid.size());
  for (size_t l = 0; l < r.size(); ++l) {
    uint64_t h = (uint64_t)b.gid[l] * 0x9e3779b97f4a7c15ull + seed;
    h ^= h >> 31;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 29;
    r[l] = b.dir[l] ? 0.0 : ((double)(h >> 11) / 9007199254740992.0) * 2.0 - 1.0;
  }
  return r;
}

struct Dev {
  double* p = nullptr;
  size_t n = 0;
  explicit Dev(size_t n_) : n(n_) { HIPCHECK(hipMalloc(&p, sizeof(double) * n)); }
  Dev(const std::vector<double>& h) : n(h.size()) {
    HIPCHECK(hipMalloc(&p, sizeof(double) * n));
    HIPCHECK(hipMemcpy(p, h.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  }
  ~Dev() { (void)hipFree(p); }
  Dev(const Dev&) = delete;
  Dev& operator=(const Dev&) = delete;
};

void solve_checks(const Box& b, sem_mesh m, int smoother) {
  sem_pmg_opts o;
  sem_pmg_opts_default(&o);
  o.smoother = smoother;
  sem_pmg p = nullptr;
  CHECK(sem_pmg_setup(m, &o, &p) == SEM_OK, "sem_pmg_setup N=%d smoother=%d", b.N, smoother);
  if (!p) return;
  sem_pmg_info pi;
  CHECK(sem_pmg_query(p, &pi) == SEM_OK && pi.n_levels >= 2, "sem_pmg_query");
  Dev bd(rhs(b, 7)), x(b.gid.size());
  sem_solve_opts so;
  sem_solve_opts_default(&so);
  so.rtol = 1e-8;
  sem_solve_info info;
  CHECK(sem_pcg_solve(m, p, bd.p, x.p, &so, &info, nullptr) == SEM_OK && info.relres_true <= 1.1e-8,
        "FlexCG+pMG N=%d smoother=%d relres_true=%g", b.N, smoother, info.relres_true);
  CHECK(sem_gmres_solve(m, p, 4, bd.p, x.p, &so, &info, nullptr) == SEM_OK && info.relres_true <= 1.1e-8,
        "GMRES(4)+pMG N=%d relres_true=%g", b.N, info.relres_true);
  Dev z(b.gid.size());
  CHECK(sem_pmg_apply(p, bd.p, z.p, nullptr) == SEM_OK, "sem_pmg_apply");
  // projection onto prior solutions over a few right-hand sides
  sem_proj pr = nullptr;
  CHECK(sem_proj_create(m, 4, &pr) == SEM_OK, "sem_proj_create");
  for (int k = 0; k < 6 && pr; ++k) {
    Dev bk(rhs(b, 100 + (k % 3)));
    CHECK(sem_pcg_solve_projected(pr, p, bk.p, x.p, &so, &info, nullptr) == SEM_OK &&
              info.relres_true <= 1.1e-8,
          "projected solve %d relres_true=%g", k, info.relres_true);
  }
  if (pr) sem_proj_destroy(pr);
  CHECK(sem_pmg_destroy(p) == SEM_OK, "sem_pmg_destroy");
}

}  // namespace

int main(int argc, char** argv) {
  if (argc > 1 && std::string(argv[1]) == "--self-check") {
    // host only, no GPU call: a heap overflow that AddressSanitizer must catch
    std::vector<int>* v = new std::vector<int>(4);
    volatile int* p = v->data();
    p[argc + 3] = 1;  // one past the end
    std::printf("self-check: overflow not detected\n");
    return 3;
  }
  std::printf("sanitizer driver: meshes, operators, solves, batches, error paths\n");
  std::fflush(stdout);
  // meshes of several orders; one with relabelled IDs, one single element
  struct Case { int nx, ny, nz, N; double amp; uint64_t relabel; };
  const Case cases[] = {{3, 2, 2, 7, 0.05, 0}, {3, 3, 2, 5, 0.05, 11}, {2, 2, 3, 9, 0.04, 0},
                        {2, 3, 2, 3, 0.05, 5}, {1, 1, 1, 7, 0.0, 0}, {4, 2, 1, 4, 0.03, 0}};
  std::vector<Box> boxes;
  std::vector<sem_mesh> meshes;
  for (const Case& c : cases) {
    boxes.push_back(make_box(c.nx, c.ny, c.nz, c.N, c.amp, c.relabel));
    meshes.push_back(create(boxes.back()));
  }
  for (size_t k = 0; k < boxes.size(); ++k) {
    const Box& b = boxes[k];
    sem_mesh m = meshes[k];
    if (!m) continue;
    std::printf("case %zu: N=%d E=%lld\n", k, b.N, (long long)b.E);
    std::fflush(stdout);
    sem_mesh_info mi;
    CHECK(sem_mesh_query(m, &mi) == SEM_OK && mi.n_local == (int64_t)b.gid.size(), "sem_mesh_query");
    const size_t n = b.gid.size();
    Dev u(rhs(b, 3)), Au(n);
    CHECK(sem_ax(m, SEM_F64, u.p, Au.p, 0, b.E, nullptr) == SEM_OK, "sem_ax");
    CHECK(sem_helmholtz(m, SEM_F64, u.p, Au.p, 2.0, nullptr) == SEM_OK, "sem_helmholtz");
    CHECK(sem_gs(m, SEM_F64, Au.p, 1, nullptr) == SEM_OK, "sem_gs");
    CHECK(sem_mass(m, SEM_F64, u.p, Au.p, nullptr) == SEM_OK, "sem_mass");
    double d1 = 0, d2 = 0;
    CHECK(sem_dot(m, SEM_F64, u.p, u.p, &d1, nullptr) == SEM_OK, "sem_dot");
    CHECK(sem_dot_noalloc(m, SEM_F64, u.p, u.p, &d2, nullptr) == SEM_OK && std::fabs(d1 - d2) <= 1e-12 * d1,
          "sem_dot_noalloc %g vs %g", d2, d1);
    Dev Gd(6 * n), Bd(n), Dd(n);
    CHECK(sem_mesh_export(m, Gd.p, Bd.p, Dd.p, nullptr) == SEM_OK, "sem_mesh_export");
    // Jacobi-PCG and Helmholtz Jacobi-PCG
    Dev bd(rhs(b, 5)), x(n);
    sem_solve_opts so;
    sem_solve_opts_default(&so);
    sem_solve_info info;
    CHECK(sem_pcg_solve(m, nullptr, bd.p, x.p, &so, &info, nullptr) == SEM_OK && info.relres_true <= 1.1e-8,
          "Jacobi-PCG relres_true=%g", info.relres_true);
    so.lambda = 10.0;
    CHECK(sem_pcg_solve(m, nullptr, bd.p, x.p, &so, &info, nullptr) == SEM_OK && info.relres_true <= 1.1e-8,
          "Helmholtz PCG relres_true=%g", info.relres_true);
    if (b.N >= 3) {
      solve_checks(b, m, SEM_SMOOTH_CHEB_JACOBI);
      solve_checks(b, m, SEM_SMOOTH_CHEB_RAS);
      solve_checks(b, m, SEM_SMOOTH_CHEB_ASM);
    }
  }
  // batched solve and the continuous-batching API over the first three meshes
  {
    std::vector<sem_pmg> pm;
    std::vector<Dev*> bs, xs;
    std::vector<const double*> bp;
    std::vector<double*> xp;
    for (int k = 0; k < 3; ++k) {
      sem_pmg p = nullptr;
      CHECK(sem_pmg_setup(meshes[k], nullptr, &p) == SEM_OK, "pmg for batch");
      pm.push_back(p);
      bs.push_back(new Dev(rhs(boxes[k], 50 + k)));
      xs.push_back(new Dev(boxes[k].gid.size()));
      bp.push_back(bs.back()->p);
      xp.push_back(xs.back()->p);
    }
    std::vector<sem_solve_info> infos(3);
    CHECK(sem_pcg_solve_batched(3, meshes.data(), pm.data(), bp.data(), xp.data(), nullptr, infos.data(), nullptr) ==
              SEM_OK,
          "sem_pcg_solve_batched");
    sem_batch bt = nullptr;
    CHECK(sem_batch_create(2, nullptr, &bt) == SEM_OK, "sem_batch_create");
    int s0 = -1, s1 = -1, s2 = -1, act = 0;
    CHECK(sem_batch_add(bt, meshes[0], pm[0], bp[0], xp[0], nullptr, &s0) == SEM_OK, "batch add 0");
    CHECK(sem_batch_add(bt, meshes[1], pm[1], bp[1], xp[1], nullptr, &s1) == SEM_OK, "batch add 1");
    CHECK(sem_batch_add(bt, meshes[2], pm[2], bp[2], xp[2], nullptr, &s2) == SEM_EBUSY, "batch full -> EBUSY");
    for (int it = 0; it < 500; ++it) {
      CHECK(sem_batch_step(bt, 1, &act) == SEM_OK, "sem_batch_step");
      sem_solve_info si;
      for (int s : {s0, s1}) {
        if (s < 0) continue;
        if (sem_batch_poll(bt, s, &si) == SEM_OK && si.status != 1) {
          CHECK(si.status == SEM_OK && si.relres_true <= 1.1e-8, "batch slot %d status %d", s, si.status);
          CHECK(sem_batch_release(bt, s) == SEM_OK, "batch release");
          if (s == s0) s0 = -1; else s1 = -1;
        }
      }
      if (s0 < 0 && s1 < 0) break;
    }
    CHECK(s0 < 0 && s1 < 0, "batch did not finish");
    CHECK(sem_batch_destroy(bt) == SEM_OK, "sem_batch_destroy");
    for (sem_pmg p : pm) sem_pmg_destroy(p);
    for (Dev* d : bs) delete d;
    for (Dev* d : xs) delete d;
  }
  // error paths
  {
    sem_mesh m = nullptr;
    CHECK(sem_mesh_create(nullptr, &m) == SEM_EINVAL, "NULL desc");
    // one copy of a shared face node flagged Dirichlet, its twin not
    Box bad = make_box(2, 1, 1, 3, 0.0, 0);
    const int NP = 4;
    bad.dir[3 + NP * 1 + NP * NP * 1] = 1;  // element 0, face i = N, an interior node of the face
    sem_mesh_desc d{};
    d.N = bad.N;
    d.E = bad.E;
    d.x = bad.x.data();
    d.y = bad.y.data();
    d.z = bad.z.data();
    d.gid = bad.gid.data();
    d.dirichlet = bad.dir.data();
    CHECK(sem_mesh_create(&d, &m) == SEM_EINVAL && m == nullptr, "inconsistent Dirichlet flags -> EINVAL");
    d.N = 0;
    CHECK(sem_mesh_create(&d, &m) == SEM_EINVAL, "N = 0 -> EINVAL");
    d.N = 3;
    std::vector<int64_t> neg(bad.gid);
    neg[7] = -1;
    d.gid = neg.data();
    CHECK(sem_mesh_create(&d, &m) == SEM_EINVAL, "negative gid -> EINVAL");
    CHECK(sem_ax(nullptr, SEM_F64, nullptr, nullptr, 0, 1, nullptr) == SEM_EINVAL, "sem_ax NULL -> EINVAL");
  }
  for (sem_mesh m : meshes)
    if (m) sem_mesh_destroy(m);
  std::printf("sanitizer driver: %s (%d failures)\n", g_fail ? "FAILED" : "ok", g_fail);
  return g_fail ? 1 : 0;
}
