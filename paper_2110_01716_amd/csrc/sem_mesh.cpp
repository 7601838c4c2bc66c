// Mesh construction and the single-mesh operators of the C ABI.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <mutex>

#include "sem_internal.h"

namespace sem {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  throw Error{code};
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) n = 16;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? SEM_ENOMEM : SEM_EHIP, "hipMalloc(%zu bytes) failed: %s", n,
         hipGetErrorString(e));
  }
  bytes = n;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

int64_t MeshData::resident_bytes() const {
  const DevBuf* bufs[] = {&Dg64, &Dg32, &wg, &x, &y, &z, &gid, &dmask, &owner, &G64, &G32, &B64, &B32,
                          &dinv64, &dinv32, &gs_off, &gs_idx, &gs_dir, &dir_idx, &umap, &u2l_off, &u2l_idx,
                          &udir, &dinv_u, &ell_col, &ell_val};
  int64_t s = 0;
  for (const DevBuf* b : bufs) s += (int64_t)b->bytes;
  return s;
}

// ---------------------------------------------------------------------------
// helpers on one mesh
// ---------------------------------------------------------------------------
template <typename T>
static const T* G_of(const MeshData& m) {
  if constexpr (sizeof(T) == 8) return m.G64.as<double>(); else return m.G32.as<float>();
}
template <typename T>
static const T* D_of(const MeshData& m) {
  if constexpr (sizeof(T) == 8) return m.Dg64.as<double>(); else return m.Dg32.as<float>();
}

template <typename T>
static void ax_range(const MeshData& m, const T* u, T* Au, int64_t e0, int64_t ne, const T* B, double lambda,
                     double* partial, hipStream_t s) {
  Table<AxArgs<T>> t;
  t.one.G = G_of<T>(m);
  t.one.B = B;
  t.one.lambda = lambda;
  t.one.u = u;
  t.one.Au = Au;
  t.one.e0 = e0;
  t.one.ne = ne;
  t.one.partial = partial;
  launch_ax<T>(m.N, t, ax_blocks(m.N, ne, sizeof(T) == 4), D_of<T>(m), s);
}

template <typename T>
static void gs_apply(const MeshData& m, T* v, int mask, hipStream_t s) {
  Table<GsArgs<T>> t;
  t.one.v = v;
  t.one.off = m.gs_off.as<int>();
  t.one.idx = m.gs_idx.as<int>();
  t.one.sdir = m.gs_dir.as<uint8_t>();
  t.one.dir_idx = m.dir_idx.as<int>();
  t.one.n_shared = m.n_shared;
  t.one.n_dir = mask ? m.n_dir_single : 0;
  t.one.mask = mask;
  launch_gs<T>(t, gs_blocks(m.n_shared, t.one.n_dir), s);
}

void mesh_gs(const MeshData& m, sem_dtype t, void* v, int mask, hipStream_t s) {
  if (t == SEM_F64) gs_apply<double>(m, (double*)v, mask, s);
  else gs_apply<float>(m, (float*)v, mask, s);
}

void apply_A(const MeshData& m, sem_dtype t, const void* u, void* Au, hipStream_t s) {
  if (t == SEM_F64) {
    ax_range<double>(m, (const double*)u, (double*)Au, 0, m.E, nullptr, 0.0, nullptr, s);
    gs_apply<double>(m, (double*)Au, 1, s);
  } else {
    ax_range<float>(m, (const float*)u, (float*)Au, 0, m.E, nullptr, 0.0, nullptr, s);
    gs_apply<float>(m, (float*)Au, 1, s);
  }
}

void apply_H(const MeshData& m, double lambda, const double* u, double* Hu, hipStream_t s) {
  ax_range<double>(m, u, Hu, 0, m.E, lambda != 0.0 ? m.B64.as<double>() : nullptr, lambda, nullptr, s);
  gs_apply<double>(m, Hu, 1, s);
}

void helmholtz_dinv(const MeshData& m, double lambda, double* out, double* tmp, hipStream_t s) {
  // local diagonal of A^e + lambda B, summed over copies, inverted, masked
  launch_diag_local(m, tmp, s);
  Table<VecArgs<double>> t;
  t.one.n = m.nloc;
  t.one.x = tmp;
  t.one.r = const_cast<double*>(m.B64.as<double>());
  t.one.c0 = lambda;
  launch_vec<double>(V_AXPY, t, vec_blocks(m.nloc), s);
  gs_apply<double>(m, tmp, 0, s);
  launch_dinv_to(m, tmp, out, s);
}

double mesh_dot_ws(const MeshData& m, const double* a, const double* b, double* partial, hipStream_t s) {
  const int64_t nb = vec_blocks(m.nloc);
  Table<VecArgs<double>> tb;
  tb.one.n = m.nloc;
  tb.one.z = const_cast<double*>(a);
  tb.one.w = const_cast<double*>(b);
  tb.one.r = const_cast<double*>(b);
  tb.one.owner = m.owner.as<uint8_t>();
  tb.one.partial = partial;
  tb.one.stride = nb;
  launch_vec<double>(V_DOT2, tb, nb, s);
  std::vector<double> h(nb);
  SEM_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  double sum = 0.0;
  for (int64_t k = 0; k < nb; ++k) sum += h[k];
  return sum;
}

void mesh_multidot(const MeshData& m, const double* const* v, int K, const double* y, double* partial,
                   int64_t stride, double* out, hipStream_t s) {
  MdotArgs a;
  a.n = m.nloc;
  a.K = K;
  a.v = v;
  a.y = y;
  a.owner = m.owner.as<uint8_t>();
  a.partial = partial;
  a.stride = stride;
  launch_mdot(a, s);
  launch_mfin(partial, stride, vec_blocks(m.nloc), K, out, s);
}

void mesh_lincomb(const MeshData& m, const double* const* v, int K, const double* coef, const double* y, double a0,
                  double sign, double scale, double* out, hipStream_t s) {
  LincombArgs a;
  a.n = m.nloc;
  a.K = K;
  a.v = v;
  a.coef = coef;
  a.y = y;
  a.a0 = a0;
  a.sign = sign;
  a.scale = scale;
  a.out = out;
  launch_lincomb(a, s);
}

void vec_op1(VecOp op, int64_t n, double* x, const double* r, double c0, const double* dinv, hipStream_t s) {
  Table<VecArgs<double>> t;
  t.one.n = n;
  t.one.x = x;
  t.one.r = const_cast<double*>(r);
  t.one.dinv = dinv;
  t.one.c0 = c0;
  launch_vec<double>(op, t, vec_blocks(n), s);
}

// per-block partial sums of the unique-DOF product a.b into partial[0, nb)
// (V_DOT2 also fills partial[nb, 2 nb)), nb = vec_blocks(m.nloc)
static void dot_partials(const MeshData& m, sem_dtype t, const void* a, const void* b, double* partial,
                         hipStream_t s) {
  const int64_t nb = vec_blocks(m.nloc);
  if (t == SEM_F64) {
    Table<VecArgs<double>> tb;
    tb.one.n = m.nloc;
    tb.one.z = (double*)a;
    tb.one.w = (double*)b;
    tb.one.r = (double*)b;
    tb.one.owner = m.owner.as<uint8_t>();
    tb.one.partial = partial;
    tb.one.stride = nb;
    launch_vec<double>(V_DOT2, tb, nb, s);
  } else {
    Table<VecArgs<float>> tb;
    tb.one.n = m.nloc;
    tb.one.z = (float*)a;
    tb.one.w = (float*)b;
    tb.one.r = (float*)b;
    tb.one.owner = m.owner.as<uint8_t>();
    tb.one.partial = partial;
    tb.one.stride = nb;
    launch_vec<float>(V_DOT2, tb, nb, s);
  }
}

double mesh_dot(const MeshData& m, sem_dtype t, const void* a, const void* b, hipStream_t s) {
  const int64_t nb = vec_blocks(m.nloc);
  DevBuf part;
  part.alloc(sizeof(double) * 2 * nb);
  dot_partials(m, t, a, b, part.as<double>(), s);
  std::vector<double> h(nb);
  SEM_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  double sum = 0.0;
  for (int64_t k = 0; k < nb; ++k) sum += h[k];
  return sum;
}

// ---------------------------------------------------------------------------
// allocation-free inner product (sem_dot_noalloc)
//
// The partial sums live in a file-scope device array instead of a buffer
// allocated per call. In host code `scratch` only names the symbol: its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is ever handed to kernels or copies.
// Every slot a call reads is written earlier in the same call (partials, then
// the reduced result), so nothing needs clearing between calls; calls that
// overlap on one device share the array and race.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kDotScratchBlocks = 65536;  // partial sums per row: vec_blocks(n_local) <= this
constexpr int64_t kDotResult = 2 * kDotScratchBlocks;  // slot of the reduced sum
constexpr int64_t kDotScratchDoubles = kDotResult + 32;  // 1 MiB + 256 B
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kDotScratchDoubles];
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

double* scratch_address() {
  int dev = 0;
  SEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(SEM_EINVAL, "sem_dot_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(SEM_EHIP, "sem_dot_noalloc: no device address for the scratch array on device %d", dev);
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

// ---------------------------------------------------------------------------
// mesh construction
// ---------------------------------------------------------------------------
void build_mesh(MeshData& m, int N, int64_t E, const int64_t* gid_host, const uint8_t* dir_host, hipStream_t s) {
  m.N = N;
  m.NP = N + 1;
  m.Np = m.NP * m.NP * m.NP;
  m.E = E;
  m.nloc = E * m.Np;
  const int NP = m.NP;

  m.D.assign(NP * NP, 0.0);
  m.w.assign(NP, 0.0);
  std::vector<double> xg(NP);
  gll_points(N, xg.data(), m.w.data());
  deriv_matrix(N, m.D.data());
  std::vector<float> Df(m.D.begin(), m.D.end());
  m.Dg64.alloc(sizeof(double) * NP * NP);
  m.Dg32.alloc(sizeof(float) * NP * NP);
  m.wg.alloc(sizeof(double) * NP);
  SEM_HIP(hipMemcpyAsync(m.Dg64.p, m.D.data(), sizeof(double) * NP * NP, hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemcpyAsync(m.Dg32.p, Df.data(), sizeof(float) * NP * NP, hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemcpyAsync(m.wg.p, m.w.data(), sizeof(double) * NP, hipMemcpyHostToDevice, s));

  m.gid.alloc(sizeof(int64_t) * m.nloc);
  SEM_HIP(hipMemcpyAsync(m.gid.p, gid_host, sizeof(int64_t) * m.nloc, hipMemcpyHostToDevice, s));
  m.dmask.alloc(m.nloc);
  if (dir_host)
    SEM_HIP(hipMemcpyAsync(m.dmask.p, dir_host, m.nloc, hipMemcpyHostToDevice, s));
  else
    SEM_HIP(hipMemsetAsync(m.dmask.p, 0, m.nloc, s));

  // geometric factors
  m.G64.alloc(sizeof(double) * 6 * m.nloc);
  m.G32.alloc(sizeof(float) * 6 * m.nloc);
  m.B64.alloc(sizeof(double) * m.nloc);
  m.B32.alloc(sizeof(float) * m.nloc);
  const int64_t nb = (m.nloc + 255) / 256;
  DevBuf pmin, pvol, bad;
  pmin.alloc(sizeof(double) * nb);
  pvol.alloc(sizeof(double) * nb);
  bad.alloc(sizeof(int64_t));
  SEM_HIP(hipMemsetAsync(bad.p, 0xff, sizeof(int64_t), s));
  launch_geometry(m, pmin.as<double>(), pvol.as<double>(), bad.as<int64_t>(), s);
  std::vector<double> hmin(nb), hvol(nb);
  uint64_t hbad = 0;
  SEM_HIP(hipMemcpyAsync(hmin.data(), pmin.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipMemcpyAsync(hvol.data(), pvol.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  if (hbad != ~0ull) {
    fail(SEM_EGEOM, "sem_mesh_create: Jacobian determinant <= 0 at element %lld, point %lld",
         (long long)(hbad / m.Np), (long long)(hbad % m.Np));
  }
  double mn = INFINITY, vol = 0.0;
  for (int64_t k = 0; k < nb; ++k) {
    mn = std::min(mn, hmin[k]);
    vol += hvol[k];
  }
  m.min_detJ = mn;
  m.volume = vol;

  build_gs_map(m, s);

  // inverse Jacobi diagonal: local diagonal, summed over copies, inverted, masked
  DevBuf dl;
  dl.alloc(sizeof(double) * m.nloc);
  launch_diag_local(m, dl.as<double>(), s);
  gs_apply<double>(m, dl.as<double>(), 0, s);
  m.dinv64.alloc(sizeof(double) * m.nloc);
  m.dinv32.alloc(sizeof(float) * m.nloc);
  launch_dinv_finish(m, dl.as<double>(), s);
  SEM_HIP(hipStreamSynchronize(s));
}

}  // namespace sem

using namespace sem;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int sem_mesh_create(const sem_mesh_desc* d, sem_mesh* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!d || !out) fail(SEM_EINVAL, "sem_mesh_create: NULL argument");
    if (d->N < 1 || d->N > kMaxN) fail(SEM_EINVAL, "sem_mesh_create: N=%d outside [1,%d]", d->N, kMaxN);
    if (d->E < 1) fail(SEM_EINVAL, "sem_mesh_create: E=%lld < 1", (long long)d->E);
    if (!d->x || !d->y || !d->z || !d->gid) fail(SEM_EINVAL, "sem_mesh_create: NULL coordinate or gid array");
    const int64_t Np = (int64_t)(d->N + 1) * (d->N + 1) * (d->N + 1);
    if (d->E > 2147483647LL / Np)
      fail(SEM_EINVAL, "sem_mesh_create: %lld elements of %lld points exceed 2^31-1 local points", (long long)d->E,
           (long long)Np);
    const int64_t nloc = d->E * Np;
    for (int64_t l = 0; l < nloc; ++l)
      if (d->gid[l] < 0)
        fail(SEM_EINVAL, "sem_mesh_create: negative global ID at element %lld, point %lld", (long long)(l / Np),
             (long long)(l % Np));
    hipStream_t s = (hipStream_t)d->stream;
    auto mesh = std::make_unique<sem_mesh_s>();
    MeshData& m = mesh->d;
    m.x.alloc(sizeof(double) * nloc);
    m.y.alloc(sizeof(double) * nloc);
    m.z.alloc(sizeof(double) * nloc);
    SEM_HIP(hipMemcpyAsync(m.x.p, d->x, sizeof(double) * nloc, hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(m.y.p, d->y, sizeof(double) * nloc, hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(m.z.p, d->z, sizeof(double) * nloc, hipMemcpyHostToDevice, s));
    build_mesh(m, d->N, d->E, d->gid, d->dirichlet, s);
    *out = mesh.release();
  });
}

extern "C" int sem_mesh_destroy(sem_mesh m) {
  return guarded([&] {
    if (!m) return;
    if (m->owned_by_pmg) fail(SEM_EINVAL, "sem_mesh_destroy: level mesh is owned by its pMG hierarchy");
    delete m;
  });
}

extern "C" int sem_mesh_query(sem_mesh mh, sem_mesh_info* info) {
  return guarded([&] {
    if (!mh || !info) fail(SEM_EINVAL, "sem_mesh_query: NULL argument");
    const MeshData& m = mh->d;
    info->N = m.N;
    info->E = m.E;
    info->n_local = m.nloc;
    info->n_unique = m.n_unique;
    info->n_interior = m.n_interior;
    info->n_shared_nodes = m.n_shared;
    info->n_shared_entries = m.n_shared_entries;
    info->resident_bytes = m.resident_bytes();
    info->min_detJ = m.min_detJ;
    info->volume = m.volume;
  });
}

extern "C" int sem_mesh_export(sem_mesh mh, double* G, double* B, double* dinv, void* stream) {
  return guarded([&] {
    if (!mh) fail(SEM_EINVAL, "sem_mesh_export: NULL mesh");
    const MeshData& m = mh->d;
    hipStream_t s = (hipStream_t)stream;
    if (G) SEM_HIP(hipMemcpyAsync(G, m.G64.p, sizeof(double) * 6 * m.nloc, hipMemcpyDeviceToDevice, s));
    if (B) SEM_HIP(hipMemcpyAsync(B, m.B64.p, sizeof(double) * m.nloc, hipMemcpyDeviceToDevice, s));
    if (dinv) SEM_HIP(hipMemcpyAsync(dinv, m.dinv64.p, sizeof(double) * m.nloc, hipMemcpyDeviceToDevice, s));
  });
}

extern "C" int sem_mesh_export_nodes(sem_mesh mh, double* x, double* y, double* z, int64_t* gid, uint8_t* dir,
                                     void* stream) {
  return guarded([&] {
    if (!mh) fail(SEM_EINVAL, "sem_mesh_export_nodes: NULL mesh");
    const MeshData& m = mh->d;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)m.nloc;
    if (x) SEM_HIP(hipMemcpyAsync(x, m.x.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (y) SEM_HIP(hipMemcpyAsync(y, m.y.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (z) SEM_HIP(hipMemcpyAsync(z, m.z.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (gid) SEM_HIP(hipMemcpyAsync(gid, m.gid.p, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
    if (dir) SEM_HIP(hipMemcpyAsync(dir, m.dmask.p, n, hipMemcpyDeviceToDevice, s));
  });
}

static void check_dtype(sem_dtype t, const char* who) {
  if (t != SEM_F64 && t != SEM_F32) fail(SEM_EINVAL, "%s: unknown dtype %d", who, (int)t);
}

extern "C" int sem_ax(sem_mesh mh, sem_dtype t, const void* u, void* Au, int64_t e0, int64_t ne, void* stream) {
  return guarded([&] {
    if (!mh || !u || !Au) fail(SEM_EINVAL, "sem_ax: NULL argument");
    check_dtype(t, "sem_ax");
    const MeshData& m = mh->d;
    if (e0 < 0 || ne < 0 || e0 + ne > m.E)
      fail(SEM_EINVAL, "sem_ax: element range [%lld, %lld) outside [0, %lld)", (long long)e0,
           (long long)(e0 + ne), (long long)m.E);
    if (ne == 0) return;
    hipStream_t s = (hipStream_t)stream;
    if (t == SEM_F64) ax_range<double>(m, (const double*)u, (double*)Au, e0, ne, nullptr, 0.0, nullptr, s);
    else ax_range<float>(m, (const float*)u, (float*)Au, e0, ne, nullptr, 0.0, nullptr, s);
  });
}

extern "C" int sem_helmholtz(sem_mesh mh, sem_dtype t, const void* u, void* Au, double lambda, void* stream) {
  return guarded([&] {
    if (!mh || !u || !Au) fail(SEM_EINVAL, "sem_helmholtz: NULL argument");
    check_dtype(t, "sem_helmholtz");
    const MeshData& m = mh->d;
    hipStream_t s = (hipStream_t)stream;
    if (t == SEM_F64)
      ax_range<double>(m, (const double*)u, (double*)Au, 0, m.E, m.B64.as<double>(), lambda, nullptr, s);
    else
      ax_range<float>(m, (const float*)u, (float*)Au, 0, m.E, m.B32.as<float>(), lambda, nullptr, s);
  });
}

extern "C" int sem_gs(sem_mesh mh, sem_dtype t, void* v, int apply_mask, void* stream) {
  return guarded([&] {
    if (!mh || !v) fail(SEM_EINVAL, "sem_gs: NULL argument");
    check_dtype(t, "sem_gs");
    hipStream_t s = (hipStream_t)stream;
    if (t == SEM_F64) gs_apply<double>(mh->d, (double*)v, apply_mask ? 1 : 0, s);
    else gs_apply<float>(mh->d, (float*)v, apply_mask ? 1 : 0, s);
  });
}

extern "C" int sem_mass(sem_mesh mh, sem_dtype t, const void* u, void* Bu, void* stream) {
  return guarded([&] {
    if (!mh || !u || !Bu) fail(SEM_EINVAL, "sem_mass: NULL argument");
    check_dtype(t, "sem_mass");
    const MeshData& m = mh->d;
    launch_mass(m.N, m.nloc, t == SEM_F32, t == SEM_F32 ? (const void*)m.B32.p : (const void*)m.B64.p, u, Bu,
                (hipStream_t)stream);
  });
}

extern "C" int sem_dot(sem_mesh mh, sem_dtype t, const void* a, const void* b, double* result, void* stream) {
  return guarded([&] {
    if (!mh || !a || !b || !result) fail(SEM_EINVAL, "sem_dot: NULL argument");
    check_dtype(t, "sem_dot");
    *result = mesh_dot(mh->d, t, a, b, (hipStream_t)stream);
  });
}

extern "C" int sem_dot_noalloc(sem_mesh mh, sem_dtype t, const void* a, const void* b, double* result,
                               void* stream) {
  return guarded([&] {
    if (!mh || !a || !b || !result) fail(SEM_EINVAL, "sem_dot_noalloc: NULL argument");
    check_dtype(t, "sem_dot_noalloc");
    const MeshData& m = mh->d;
    const int64_t nb = vec_blocks(m.nloc);
    if (nb > kDotScratchBlocks)
      fail(SEM_EINVAL,
           "sem_dot_noalloc: %lld local points need %lld partial sums, more than the %lld of the static scratch "
           "(at most 134217728 local points)",
           (long long)m.nloc, (long long)nb, (long long)kDotScratchBlocks);
    hipStream_t s = (hipStream_t)stream;
    double* part = scratch_address();
    dot_partials(m, t, a, b, part, s);
    launch_mfin(part, nb, nb, 1, part + kDotResult, s);
    SEM_HIP(hipMemcpyAsync(result, part + kDotResult, sizeof(double), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
  });
}

extern "C" const char* sem_status_string(int status) {
  switch (status) {
    case SEM_OK: return "SEM_OK";
    case SEM_EINVAL: return "SEM_EINVAL: invalid argument";
    case SEM_EGEOM: return "SEM_EGEOM: non-positive Jacobian";
    case SEM_ENOMEM: return "SEM_ENOMEM: out of device memory";
    case SEM_EHIP: return "SEM_EHIP: HIP runtime error";
    case SEM_ENOCONV: return "SEM_ENOCONV: iteration limit reached";
    case SEM_ENAN: return "SEM_ENAN: NaN or Inf encountered";
    case SEM_EBUSY: return "SEM_EBUSY: no free batch slot";
    default: return "unknown status";
  }
}

extern "C" const char* sem_last_error(void) { return sem::g_last_error.c_str(); }
