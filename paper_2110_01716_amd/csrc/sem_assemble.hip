// Assembled form of a mesh level on unique degrees of freedom (used for the
// coarsest pMG level).
//
// The operator is the same re-discretised SEM Laplacian as the matrix-free
// path: A = M Q^T blockdiag(A^e) Q M with A^e = sum_mn D_m^T diag(G_mn) D_n.
// The paper hands its coarse problem to an algebraic solver as an assembled
// matrix (Performance Measurements, coarse-grid discussion); here it stays on
// the GPU. On unique DOFs the coarse vectors are (N+1)^3 E / n_unique times
// shorter (7.5x at N=1 on a box), which is what makes the latency-bound
// coarse Jacobi-PCG loop cheap.
//
// Construction (device):
//   1. element matrices A^e (Np x Np per element) from G and Dhat;
//   2. triplets (row, col, value) with row/col = unique index of the copies,
//      entries touching a Dirichlet ID dropped;
//   3. stable radix sort by row * n + col (element order kept within a key),
//      sums of equal keys in that order (deterministic);
//   4. ELL storage [W][n_unique] (column-major: consecutive rows are
//      consecutive in memory), columns ascending within a row, padded with
//      (col = row, value = 0).
#include <hip/hip_runtime.h>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "sem_internal.h"

namespace sem {
namespace {

constexpr int kT = 256;
inline unsigned nb(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

// unique index of every local copy: run id of its position in the gid order
__global__ void k_umap(int nloc, int nrun, const int* __restrict__ start, const int* __restrict__ val,
                       int* umap) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r >= nrun) return;
  const int q1 = (r + 1 < nrun) ? start[r + 1] : nloc;
  for (int q = start[r]; q < q1; ++q) umap[val[q]] = r;
}

// A^e[p][q] = sum_x sum_mn Dm[x][p] G_mn(x) Dn[x][q], Dr[x][p] = D[ix][ip] d(jx,jp) d(kx,kp), ...
__global__ void k_elem_triplets(int N, int64_t E, int nun, const double* __restrict__ G,
                                const double* __restrict__ Dg, const int* __restrict__ umap,
                                const uint8_t* __restrict__ udir, uint64_t* key, double* valv) {
  const int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= E * NP3 * NP3) return;
  const int64_t e = t / ((int64_t)NP3 * NP3);
  const int pq = (int)(t - e * NP3 * NP3);
  const int p = pq / NP3, q = pq % NP3;
  const int ip = p % NP, jp = (p / NP) % NP, kp = p / NP2;
  const int iq = q % NP, jq = (q / NP) % NP, kq = q / NP2;
  const double* g = G + e * 6 * NP3;
  double a = 0.0;
  // derivative of basis p along direction m at quadrature point x is nonzero only when
  // x shares p's other two indices; enumerate x over the union of such lines
  for (int x = 0; x < NP3; ++x) {
    const int ix = x % NP, jx = (x / NP) % NP, kx = x / NP2;
    double dp[3], dq[3];
    dp[0] = (jx == jp && kx == kp) ? Dg[ix * NP + ip] : 0.0;
    dp[1] = (ix == ip && kx == kp) ? Dg[jx * NP + jp] : 0.0;
    dp[2] = (ix == ip && jx == jp) ? Dg[kx * NP + kp] : 0.0;
    dq[0] = (jx == jq && kx == kq) ? Dg[ix * NP + iq] : 0.0;
    dq[1] = (ix == iq && kx == kq) ? Dg[jx * NP + jq] : 0.0;
    dq[2] = (ix == iq && jx == jq) ? Dg[kx * NP + kq] : 0.0;
    if (dp[0] == 0.0 && dp[1] == 0.0 && dp[2] == 0.0) continue;
    if (dq[0] == 0.0 && dq[1] == 0.0 && dq[2] == 0.0) continue;
    const double grr = g[0 * NP3 + x], grs = g[1 * NP3 + x], grt = g[2 * NP3 + x];
    const double gss = g[3 * NP3 + x], gst = g[4 * NP3 + x], gtt = g[5 * NP3 + x];
    const double w0 = grr * dq[0] + grs * dq[1] + grt * dq[2];
    const double w1 = grs * dq[0] + gss * dq[1] + gst * dq[2];
    const double w2 = grt * dq[0] + gst * dq[1] + gtt * dq[2];
    a += dp[0] * w0 + dp[1] * w1 + dp[2] * w2;
  }
  const int row = umap[e * NP3 + p], col = umap[e * NP3 + q];
  const bool drop = udir[row] || udir[col];
  key[t] = drop ? ~0ull : (uint64_t)row * (uint64_t)nun + (uint64_t)col;
  valv[t] = drop ? 0.0 : a;
}

__global__ void k_udir(int nloc, const int* __restrict__ umap, const uint8_t* __restrict__ dmask, uint8_t* udir) {
  const int l = blockIdx.x * kT + threadIdx.x;
  if (l < nloc && dmask[l]) udir[umap[l]] = 1;
}

__global__ void k_heads64(int64_t n, const uint64_t* __restrict__ key, int* head) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) head[i] = (key[i] != ~0ull && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
}

// entry id (inclusive scan - 1) -> summed value (in sorted order), row, col
__global__ void k_reduce_entries(int64_t n, int nun, const uint64_t* __restrict__ key,
                                 const int* __restrict__ head, const int* __restrict__ incl,
                                 const int* __restrict__ perm, const double* __restrict__ valv, double* ent_val,
                                 int* ent_row, int* ent_col) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n || !head[i]) return;
  const uint64_t k = key[i];
  double s = 0.0;
  for (int64_t j = i; j < n && key[j] == k; ++j) s += valv[perm[j]];
  const int id = incl[i] - 1;
  ent_val[id] = s;
  ent_row[id] = (int)(k / (uint64_t)nun);
  ent_col[id] = (int)(k % (uint64_t)nun);
}

__global__ void k_row_count(int nent, const int* __restrict__ ent_row, int* cnt) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < nent && (i == 0 || ent_row[i] != ent_row[i - 1])) {
    int j = i;
    while (j < nent && ent_row[j] == ent_row[i]) ++j;
    cnt[ent_row[i]] = j - i;
  }
}

__global__ void k_ell_fill(int nun, int W, const int* __restrict__ rowoff, const int* __restrict__ cnt,
                           const double* __restrict__ ent_val, const int* __restrict__ ent_col, int* ell_col,
                           double* ell_val, double* diag) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r >= nun) return;
  const int c = cnt[r], o = rowoff[r];
  double d = 0.0;
  for (int k = 0; k < W; ++k) {
    int col = r;
    double v = 0.0;
    if (k < c) {
      col = ent_col[o + k];
      v = ent_val[o + k];
      if (col == r) d = v;
    }
    ell_col[(int64_t)k * nun + r] = col;
    ell_val[(int64_t)k * nun + r] = v;
  }
  diag[r] = d;
}

__global__ void k_dinv_u(int nun, const double* __restrict__ diag, const uint8_t* __restrict__ udir, double* dinv) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r < nun) dinv[r] = (udir[r] || diag[r] == 0.0) ? 0.0 : 1.0 / diag[r];
}

template <typename F>
void with_temp(F&& f, hipStream_t s) {
  size_t bytes = 0;
  SEM_HIP(f(nullptr, bytes));
  DevBuf tmp;
  tmp.alloc(bytes > 0 ? bytes : 16);
  SEM_HIP(f(tmp.p, bytes));
  SEM_HIP(hipStreamSynchronize(s));
}

template <typename T>
T read1(const T* dev, int64_t i, hipStream_t s) {
  T v{};
  SEM_HIP(hipMemcpyAsync(&v, dev + i, sizeof(T), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  return v;
}

__global__ void k_run_start(int n, const int* __restrict__ head, const int* __restrict__ incl, int* start) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n && head[i]) start[incl[i] - 1] = i;
}

__global__ void k_iota(int64_t n, int* v) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) v[i] = (int)i;
}

}  // namespace

void build_assembled(MeshData& m, hipStream_t s) {
  const int nloc = (int)m.nloc;
  const int nun = (int)m.n_unique;
  const int NP3 = m.Np;
  // unique index of each copy, and the unique -> copies CSR (ascending local index)
  {
    DevBuf keys_out, vals_in, head, incl, start;
    keys_out.alloc(sizeof(int64_t) * nloc);
    vals_in.alloc(sizeof(int) * nloc);
    m.u2l_idx.alloc(sizeof(int) * nloc);
    hipLaunchKernelGGL(k_iota, dim3(nb(nloc)), dim3(kT), 0, s, (int64_t)nloc, vals_in.as<int>());
    with_temp([&](void* tmp, size_t& bytes) {
      return rocprim::radix_sort_pairs(tmp, bytes, m.gid.as<int64_t>(), keys_out.as<int64_t>(), vals_in.as<int>(),
                                       m.u2l_idx.as<int>(), (size_t)nloc, 0, 64, s);
    }, s);
    head.alloc(sizeof(int) * nloc);
    incl.alloc(sizeof(int) * nloc);
    hipLaunchKernelGGL(k_heads64, dim3(nb(nloc)), dim3(kT), 0, s, (int64_t)nloc,
                       reinterpret_cast<const uint64_t*>(keys_out.p), head.as<int>());
    with_temp([&](void* tmp, size_t& bytes) {
      return rocprim::inclusive_scan(tmp, bytes, head.as<int>(), incl.as<int>(), (size_t)nloc, rocprim::plus<int>(), s);
    }, s);
    m.u2l_off.alloc(sizeof(int) * (nun + 1));
    // run starts: position of each head
    DevBuf st;
    st.alloc(sizeof(int) * (nun + 1));
    hipLaunchKernelGGL(k_run_start, dim3(nb(nloc)), dim3(kT), 0, s, nloc, head.as<int>(), incl.as<int>(),
                       st.as<int>());
    SEM_HIP(hipMemcpyAsync(st.as<int>() + nun, &nloc, sizeof(int), hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(m.u2l_off.p, st.p, sizeof(int) * (nun + 1), hipMemcpyDeviceToDevice, s));
    m.umap.alloc(sizeof(int) * nloc);
    hipLaunchKernelGGL(k_umap, dim3(nb(nun)), dim3(kT), 0, s, nloc, nun, st.as<int>(), m.u2l_idx.as<int>(),
                       m.umap.as<int>());
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipStreamSynchronize(s));
  }
  m.udir.alloc(nun);
  SEM_HIP(hipMemsetAsync(m.udir.p, 0, nun, s));
  hipLaunchKernelGGL(k_udir, dim3(nb(nloc)), dim3(kT), 0, s, nloc, m.umap.as<int>(), m.dmask.as<uint8_t>(),
                     m.udir.as<uint8_t>());
  // triplets
  const int64_t ntr = m.E * (int64_t)NP3 * NP3;
  DevBuf key, key2, valv, perm, perm2;
  key.alloc(sizeof(uint64_t) * ntr);
  key2.alloc(sizeof(uint64_t) * ntr);
  valv.alloc(sizeof(double) * ntr);
  perm.alloc(sizeof(int) * ntr);
  perm2.alloc(sizeof(int) * ntr);
  hipLaunchKernelGGL(k_elem_triplets, dim3(nb(ntr)), dim3(kT), 0, s, m.N, m.E, nun, m.G64.as<double>(),
                     m.Dg64.as<double>(), m.umap.as<int>(), m.udir.as<uint8_t>(), key.as<uint64_t>(),
                     valv.as<double>());
  hipLaunchKernelGGL(k_iota, dim3(nb(ntr)), dim3(kT), 0, s, ntr, perm.as<int>());
  SEM_HIP(hipGetLastError());
  with_temp([&](void* tmp, size_t& bytes) {
    return rocprim::radix_sort_pairs(tmp, bytes, key.as<uint64_t>(), key2.as<uint64_t>(), perm.as<int>(),
                                     perm2.as<int>(), (size_t)ntr, 0, 64, s);
  }, s);
  DevBuf head, incl;
  head.alloc(sizeof(int) * ntr);
  incl.alloc(sizeof(int) * ntr);
  hipLaunchKernelGGL(k_heads64, dim3(nb(ntr)), dim3(kT), 0, s, ntr, key2.as<uint64_t>(), head.as<int>());
  with_temp([&](void* tmp, size_t& bytes) {
    return rocprim::inclusive_scan(tmp, bytes, head.as<int>(), incl.as<int>(), (size_t)ntr, rocprim::plus<int>(), s);
  }, s);
  const int nent = read1(incl.as<int>(), ntr - 1, s);
  DevBuf ent_val, ent_row, ent_col, cnt, rowoff;
  ent_val.alloc(sizeof(double) * (nent > 0 ? nent : 1));
  ent_row.alloc(sizeof(int) * (nent > 0 ? nent : 1));
  ent_col.alloc(sizeof(int) * (nent > 0 ? nent : 1));
  hipLaunchKernelGGL(k_reduce_entries, dim3(nb(ntr)), dim3(kT), 0, s, ntr, nun, key2.as<uint64_t>(), head.as<int>(),
                     incl.as<int>(), perm2.as<int>(), valv.as<double>(), ent_val.as<double>(), ent_row.as<int>(),
                     ent_col.as<int>());
  cnt.alloc(sizeof(int) * (nun + 1));
  rowoff.alloc(sizeof(int) * (nun + 1));
  SEM_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (nun + 1), s));
  // a level whose every node is Dirichlet has no entries (and no launch)
  if (nent > 0)
    hipLaunchKernelGGL(k_row_count, dim3(nb(nent)), dim3(kT), 0, s, nent, ent_row.as<int>(), cnt.as<int>());
  with_temp([&](void* tmp, size_t& bytes) {
    return rocprim::exclusive_scan(tmp, bytes, cnt.as<int>(), rowoff.as<int>(), 0, (size_t)nun + 1,
                                   rocprim::plus<int>(), s);
  }, s);
  // ELL width = longest row
  std::vector<int> hcnt(nun);
  SEM_HIP(hipMemcpyAsync(hcnt.data(), cnt.p, sizeof(int) * nun, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  int W = 1;
  for (int c : hcnt) W = c > W ? c : W;
  m.ell_w = W;
  m.ell_col.alloc(sizeof(int) * (int64_t)W * nun);
  m.ell_val.alloc(sizeof(double) * (int64_t)W * nun);
  DevBuf diag;
  diag.alloc(sizeof(double) * nun);
  hipLaunchKernelGGL(k_ell_fill, dim3(nb(nun)), dim3(kT), 0, s, nun, W, rowoff.as<int>(), cnt.as<int>(),
                     ent_val.as<double>(), ent_col.as<int>(), m.ell_col.as<int>(), m.ell_val.as<double>(),
                     diag.as<double>());
  m.dinv_u.alloc(sizeof(double) * nun);
  hipLaunchKernelGGL(k_dinv_u, dim3(nb(nun)), dim3(kT), 0, s, nun, diag.as<double>(), m.udir.as<uint8_t>(),
                     m.dinv_u.as<double>());
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipStreamSynchronize(s));
  m.assembled = true;
}

}  // namespace sem
