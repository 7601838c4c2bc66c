// Gather-scatter map from user global IDs (single-GPU form of the paper's
// gs-setup: "the user simply provides a global ID for each vertex"; the setup
// discovers which local copies are the same degree of freedom, Implementation,
// Autotuned Communication).
//
// Steps (all on the device):
//   1. stable radix sort of (gid, local index): copies of an ID become a run,
//      ordered by ascending local index;
//   2. run heads -> run ids -> run starts and counts;
//   3. per run: Dirichlet flags and coordinates must agree across copies,
//      the first copy is the owner (used for unique-DOF inner products);
//   4. shared runs (count > 1) are compacted and re-sorted by their first local
//      index, so consecutive gs threads touch nearby memory whatever the ID
//      numbering; their copies form the CSR (gs_off, gs_idx);
//   5. Dirichlet copies of unshared IDs form a plain list for the mask.
#include <hip/hip_runtime.h>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce.hpp>
#include <rocprim/device/device_scan.hpp>

#include "sem_internal.h"

namespace sem {

namespace {

constexpr int kT = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

__global__ void k_iota(int n, int* v) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) v[i] = i;
}

__global__ void k_heads(int n, const int64_t* __restrict__ key, int* head) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// run id (inclusive scan of heads minus 1) -> run start
__global__ void k_run_start(int n, const int* __restrict__ head, const int* __restrict__ incl, int* start) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n && head[i]) start[incl[i] - 1] = i;
}

// per run: consistency checks, owner flag, multiplicity of each copy
__global__ void k_runs(int nrun, int n, const int* __restrict__ start, const int* __restrict__ val,
                       const uint8_t* __restrict__ dmask, const double* __restrict__ X,
                       const double* __restrict__ Y, const double* __restrict__ Z, uint8_t* owner,
                       int* mult, int* shared_flag, int* interior_flag, int* err_dir, int* err_xyz) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r >= nrun) return;
  const int q0 = start[r], q1 = (r + 1 < nrun) ? start[r + 1] : n;
  const int cnt = q1 - q0;
  const int l0 = val[q0];
  const uint8_t d0 = dmask[l0];
  const double x0 = X[l0], y0 = Y[l0], z0 = Z[l0];
  const double tol = 1e-9;
  for (int q = q0; q < q1; ++q) {
    const int l = val[q];
    if (dmask[l] != d0) atomicMax(err_dir, l + 1);
    const double ex = fabs(X[l] - x0), ey = fabs(Y[l] - y0), ez = fabs(Z[l] - z0);
    if (ex > tol * (1.0 + fabs(x0)) || ey > tol * (1.0 + fabs(y0)) || ez > tol * (1.0 + fabs(z0)))
      atomicMax(err_xyz, l + 1);
    mult[l] = cnt;
  }
  owner[l0] = d0 ? 0 : 1;
  shared_flag[r] = cnt > 1 ? 1 : 0;
  interior_flag[r] = d0 ? 0 : 1;
}

// compact shared runs: key = first local index, value = run id
__global__ void k_shared_keys(int nrun, const int* __restrict__ start, const int* __restrict__ val,
                              const int* __restrict__ shared_flag, const int* __restrict__ excl,
                              int* key, int* runid) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r >= nrun || !shared_flag[r]) return;
  const int k = excl[r];
  key[k] = val[start[r]];
  runid[k] = r;
}

__global__ void k_shared_counts(int nsh, int nrun, int n, const int* __restrict__ start,
                                const int* __restrict__ runid, int* cnt) {
  const int k = blockIdx.x * kT + threadIdx.x;
  if (k >= nsh) return;
  const int r = runid[k];
  cnt[k] = ((r + 1 < nrun) ? start[r + 1] : n) - start[r];
}

__global__ void k_shared_fill(int nsh, const int* __restrict__ start, const int* __restrict__ runid,
                              const int* __restrict__ off, const int* __restrict__ val,
                              const uint8_t* __restrict__ dmask, int* idx, uint8_t* sdir) {
  const int k = blockIdx.x * kT + threadIdx.x;
  if (k >= nsh) return;
  const int s = start[runid[k]];
  const int c = off[k + 1] - off[k];
  for (int q = 0; q < c; ++q) idx[off[k] + q] = val[s + q];
  sdir[k] = dmask[val[s]];
}

__global__ void k_dir_single_flag(int n, const uint8_t* __restrict__ dmask, const int* __restrict__ mult,
                                  int* flag) {
  const int l = blockIdx.x * kT + threadIdx.x;
  if (l < n) flag[l] = (dmask[l] && mult[l] == 1) ? 1 : 0;
}

__global__ void k_dir_single_fill(int n, const int* __restrict__ flag, const int* __restrict__ excl, int* out) {
  const int l = blockIdx.x * kT + threadIdx.x;
  if (l < n && flag[l]) out[excl[l]] = l;
}

template <typename F>
void with_temp(F&& f, hipStream_t s) {
  size_t bytes = 0;
  SEM_HIP(f(nullptr, bytes));
  DevBuf tmp;
  tmp.alloc(bytes > 0 ? bytes : 16);
  SEM_HIP(f(tmp.p, bytes));
  SEM_HIP(hipStreamSynchronize(s));  // tmp is freed on return
}

int last_value(const int* dev, int64_t index, hipStream_t s) {
  int v = 0;
  SEM_HIP(hipMemcpyAsync(&v, dev + index, sizeof(int), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  return v;
}

}  // namespace

void build_gs_map(MeshData& m, hipStream_t s) {
  const int n = (int)m.nloc;
  DevBuf keys_out, vals_in, vals_out;
  keys_out.alloc(sizeof(int64_t) * n);
  vals_in.alloc(sizeof(int) * n);
  vals_out.alloc(sizeof(int) * n);
  hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(kT), 0, s, n, vals_in.as<int>());
  SEM_HIP(hipGetLastError());
  with_temp([&](void* tmp, size_t& bytes) {
    return rocprim::radix_sort_pairs(tmp, bytes, m.gid.as<int64_t>(), keys_out.as<int64_t>(), vals_in.as<int>(),
                                     vals_out.as<int>(), (size_t)n, 0, 64, s);
  }, s);

  DevBuf head, incl;
  head.alloc(sizeof(int) * n);
  incl.alloc(sizeof(int) * n);
  hipLaunchKernelGGL(k_heads, dim3(nblk(n)), dim3(kT), 0, s, n, keys_out.as<int64_t>(), head.as<int>());
  SEM_HIP(hipGetLastError());
  with_temp([&](void* tmp, size_t& bytes) {
    return rocprim::inclusive_scan(tmp, bytes, head.as<int>(), incl.as<int>(), (size_t)n, rocprim::plus<int>(), s);
  }, s);
  const int nrun = last_value(incl.as<int>(), n - 1, s);
  m.n_unique = nrun;

  DevBuf start, mult, shared_flag, interior_flag, errs;
  start.alloc(sizeof(int) * nrun);
  mult.alloc(sizeof(int) * n);
  shared_flag.alloc(sizeof(int) * nrun);
  interior_flag.alloc(sizeof(int) * nrun);
  errs.alloc(sizeof(int) * 2);
  SEM_HIP(hipMemsetAsync(errs.p, 0, sizeof(int) * 2, s));
  m.owner.alloc(n);
  SEM_HIP(hipMemsetAsync(m.owner.p, 0, n, s));
  hipLaunchKernelGGL(k_run_start, dim3(nblk(n)), dim3(kT), 0, s, n, head.as<int>(), incl.as<int>(), start.as<int>());
  SEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_runs, dim3(nblk(nrun)), dim3(kT), 0, s, nrun, n, start.as<int>(), vals_out.as<int>(),
                     m.dmask.as<uint8_t>(), m.x.as<double>(), m.y.as<double>(), m.z.as<double>(),
                     m.owner.as<uint8_t>(), mult.as<int>(), shared_flag.as<int>(), interior_flag.as<int>(),
                     errs.as<int>(), errs.as<int>() + 1);
  SEM_HIP(hipGetLastError());
  int herr[2];
  SEM_HIP(hipMemcpyAsync(herr, errs.p, sizeof(herr), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  if (herr[0]) {
    const int64_t l = herr[0] - 1;
    fail(SEM_EINVAL, "sem_mesh_create: Dirichlet flags differ between copies of one global ID "
                     "(element %lld, point %lld)", (long long)(l / m.Np), (long long)(l % m.Np));
  }
  if (herr[1]) {
    const int64_t l = herr[1] - 1;
    fail(SEM_EINVAL, "sem_mesh_create: coordinates differ between copies of one global ID "
                     "(element %lld, point %lld)", (long long)(l / m.Np), (long long)(l % m.Np));
  }

  // number of interior unique IDs
  {
    DevBuf sum;
    sum.alloc(sizeof(int));
    with_temp([&](void* tmp, size_t& bytes) {
      return rocprim::reduce(tmp, bytes, interior_flag.as<int>(), sum.as<int>(), 0, (size_t)nrun,
                             rocprim::plus<int>(), s);
    }, s);
    m.n_interior = last_value(sum.as<int>(), 0, s);
  }

  // shared runs
  DevBuf excl;
  excl.alloc(sizeof(int) * (nrun + 1));
  with_temp([&](void* tmp, size_t& bytes) {
    return rocprim::exclusive_scan(tmp, bytes, shared_flag.as<int>(), excl.as<int>(), 0, (size_t)nrun,
                                   rocprim::plus<int>(), s);
  }, s);
  const int nsh = last_value(excl.as<int>(), nrun - 1, s) + last_value(shared_flag.as<int>(), nrun - 1, s);
  m.n_shared = nsh;
  m.gs_off.alloc(sizeof(int) * (nsh + 1));
  m.gs_dir.alloc(nsh > 0 ? nsh : 1);
  if (nsh > 0) {
    DevBuf key, runid, key2, runid2, cnt;
    key.alloc(sizeof(int) * nsh);
    runid.alloc(sizeof(int) * nsh);
    key2.alloc(sizeof(int) * nsh);
    runid2.alloc(sizeof(int) * nsh);
    cnt.alloc(sizeof(int) * (nsh + 1));
    hipLaunchKernelGGL(k_shared_keys, dim3(nblk(nrun)), dim3(kT), 0, s, nrun, start.as<int>(), vals_out.as<int>(),
                       shared_flag.as<int>(), excl.as<int>(), key.as<int>(), runid.as<int>());
    SEM_HIP(hipGetLastError());
    with_temp([&](void* tmp, size_t& bytes) {
      return rocprim::radix_sort_pairs(tmp, bytes, key.as<int>(), key2.as<int>(), runid.as<int>(), runid2.as<int>(),
                                       (size_t)nsh, 0, 32, s);
    }, s);
    hipLaunchKernelGGL(k_shared_counts, dim3(nblk(nsh)), dim3(kT), 0, s, nsh, nrun, n, start.as<int>(),
                       runid2.as<int>(), cnt.as<int>());
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipMemsetAsync(cnt.as<int>() + nsh, 0, sizeof(int), s));
    with_temp([&](void* tmp, size_t& bytes) {
      return rocprim::exclusive_scan(tmp, bytes, cnt.as<int>(), m.gs_off.as<int>(), 0, (size_t)nsh + 1,
                                     rocprim::plus<int>(), s);
    }, s);
    m.n_shared_entries = last_value(m.gs_off.as<int>(), nsh, s);
    m.gs_idx.alloc(sizeof(int) * m.n_shared_entries);
    hipLaunchKernelGGL(k_shared_fill, dim3(nblk(nsh)), dim3(kT), 0, s, nsh, start.as<int>(), runid2.as<int>(),
                       m.gs_off.as<int>(), vals_out.as<int>(), m.dmask.as<uint8_t>(), m.gs_idx.as<int>(),
                       m.gs_dir.as<uint8_t>());
    SEM_HIP(hipGetLastError());
  } else {
    SEM_HIP(hipMemsetAsync(m.gs_off.p, 0, sizeof(int), s));
    m.n_shared_entries = 0;
    m.gs_idx.alloc(sizeof(int));
  }

  // Dirichlet copies of unshared IDs, ascending local index
  {
    DevBuf flag, ex;
    flag.alloc(sizeof(int) * n);
    ex.alloc(sizeof(int) * n);
    hipLaunchKernelGGL(k_dir_single_flag, dim3(nblk(n)), dim3(kT), 0, s, n, m.dmask.as<uint8_t>(), mult.as<int>(),
                       flag.as<int>());
    SEM_HIP(hipGetLastError());
    with_temp([&](void* tmp, size_t& bytes) {
      return rocprim::exclusive_scan(tmp, bytes, flag.as<int>(), ex.as<int>(), 0, (size_t)n, rocprim::plus<int>(), s);
    }, s);
    const int nd = last_value(ex.as<int>(), n - 1, s) + last_value(flag.as<int>(), n - 1, s);
    m.n_dir_single = nd;
    m.dir_idx.alloc(sizeof(int) * (nd > 0 ? nd : 1));
    if (nd > 0) {
      hipLaunchKernelGGL(k_dir_single_fill, dim3(nblk(n)), dim3(kT), 0, s, n, flag.as<int>(), ex.as<int>(),
                         m.dir_idx.as<int>());
      SEM_HIP(hipGetLastError());
    }
  }
  SEM_HIP(hipStreamSynchronize(s));
}

}  // namespace sem
