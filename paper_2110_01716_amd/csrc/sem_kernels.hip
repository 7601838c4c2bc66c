// HIP kernels of the SEM Poisson solve for gfx950 (MI355X).
//
//  * k_ax      matrix-free local Laplacian A_L u = sum_m D_m^T sum_n G_mn D_n u
//              (the paper's "Ax", Performance Measurements, per-kernel table).
//              Thread (i,j) of an element owns the GLL column (i,j,0..N): the t
//              derivative and its transpose run in registers, the r and s
//              derivatives read the element staged in LDS. G is streamed once,
//              coalesced (64 consecutive points per instruction at N=7).
//  * k_gs      direct-stiffness summation QQ^T with the Dirichlet mask fused in
//              (exchange-and-sum of shared values, Implementation, Autotuned
//              Communication). One thread per shared node, copies summed in
//              ascending local-index order.
//  * k_vec     fused PCG / flexible-CG / Chebyshev vector updates with
//              deterministic per-block partial dot products.
//  * k_fin     per-problem reduction of the partials in a fixed order plus the
//              scalar recurrences (alpha, beta, convergence tests).
//  * k_xfer    pMG prolongation (J x J x J) and restriction (transpose), sum
//              factorised in LDS (Implementation, pMG paragraph).
//  * k_cg_pspmv, k_cg_update
//              coarse-level Jacobi-PCG on the assembled N=1 operator.
//  * k_schwarz_mfma, k_schwarz, k_schwarz_pull
//              overlapping Schwarz smoother: fast-diagonalization solve on
//              each element's extended box (Implementation, pMG smoothers,
//              eq. fdm) on the matrix cores, or on the vector units for
//              N >= 14; the additive variant's overlap exchange.
//  * k_mdot, k_mfin, k_lincomb
//              multi-dot products and linear combinations of up to 64
//              vectors (GMRES Arnoldi steps, projection onto prior solutions).
//  * setup     geometric factors, Jacobi diagonal, start vectors, coordinates.
//
// Every kernel accepts a Table: either inline arguments for one problem or a
// device array of per-problem arguments with block prefix offsets, so one
// launch can serve many independent solves (blocks never straddle problems,
// so each problem's arithmetic is independent of the others; the persistent
// Schwarz kernel walks elements of several problems, one element at a time).
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "sem_internal.h"

namespace sem {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Pointers that arrive inside argument structs are generic to the compiler,
// which then emits flat loads (counted on both the vector-memory and LDS
// counters, so every load waits before the next LDS access). All solver
// buffers are global memory: say so.
#if defined(__HIP_DEVICE_COMPILE__)
#define SEM_GLOBAL __attribute__((address_space(1)))
#else
#define SEM_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ SEM_GLOBAL T* gl(T* p) { return (SEM_GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ const SEM_GLOBAL T* gl(const T* p) { return (const SEM_GLOBAL T*)p; }

template <typename A>
__device__ __forceinline__ A fetch_args(const Table<A>& t, int b, int& lb) {
  if (t.many == nullptr) {
    lb = b;
    return t.one;
  }
  const SEM_GLOBAL int* st = gl(t.starts);
  int lo = 0, hi = t.n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (st[mid] <= b) lo = mid; else hi = mid;
  }
  lb = b - st[lo];
  return gl(t.many)[lo];
}

__device__ __forceinline__ bool skipped(const Skip& s) {
  return (s.f0 && *(volatile const SEM_GLOBAL int*)gl(s.f0)) || (s.f1 && *(volatile const SEM_GLOBAL int*)gl(s.f1));
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// For kernels whose neighbouring work items share cache lines (gather-scatter:
// the copies of a face node live in adjacent elements), give every XCD one
// contiguous range of logical blocks instead, so shared lines meet in one L2
// (a bijection of [0, nblocks)).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, slot = b / kXcds;
  return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// Barrier for LDS hand-offs only: unlike __syncthreads() it does not wait for
// outstanding global loads, so an element's geometric factors stay in flight
// across it. A one-wave workgroup needs no hardware barrier at all.
template <int THREADS>
__device__ __forceinline__ void lds_sync() {
  if constexpr (THREADS <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block sum with a fixed order (wave butterfly, then waves in index order);
// result valid in thread 0. scratch: >= nwaves doubles of LDS.
template <int THREADS>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  constexpr int NW = (THREADS + 63) / 64;
  if constexpr (NW == 1) {
    return v;
  } else {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
      for (int k = 0; k < NW; ++k) s += scratch[k];
    return s;
  }
}

// ---------------------------------------------------------------------------
// Ax
// ---------------------------------------------------------------------------
// elements per block, by order and precision (measured). In FP32 a block
// that is one wave streams fastest where it fits: at N = 4 two elements (50
// lanes, 14% faster than ten per block), at N = 5 one (10% faster than seven).
// In FP64 at N = 5 three elements per block are 4% faster than seven.
template <typename T>
constexpr int ax_epb(int N) {
  return N == 1 ? 64 : N == 2 ? 28 : N == 3 ? 16 : N == 4 ? (sizeof(T) == 4 ? 2 : 10) : N == 5 ? (sizeof(T) == 4 ? 1 : 3)
       : N == 6 ? 5 : N == 7 ? 1 : N == 8 ? 3 : N == 9 ? 1 : N == 10 ? 2 : 1;
}

template <int N, typename T>
struct AxCfg {
  static constexpr int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  static constexpr int EPB = ax_epb<T>(N);
  static constexpr int THREADS = ((EPB * NP2 + 63) / 64) * 64;
  static constexpr int NPAD = NP | 1;  // odd row stride: conflict-free column reads
};

// ax-kernel-begin
template <int N, typename T, bool HELM>
__global__ __launch_bounds__((AxCfg<N, T>::THREADS)) void k_ax(Table<AxArgs<T>> tab, const T* __restrict__ Dg) {
  using C = AxCfg<N, T>;
  constexpr int NP = C::NP, NP2 = C::NP2, NP3 = C::NP3, EPB = C::EPB, NPAD = C::NPAD;
  __shared__ T s_u[EPB][NP][NP][NPAD];
  __shared__ T s_wr[EPB][NP][NP][NPAD];
  __shared__ T s_ws[EPB][NP][NP][NPAD];
  __shared__ double s_red[C::THREADS / 64];

  int lb;
  const AxArgs<T> a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;

  const int tid = threadIdx.x;
  const int el = tid / NP2;
  const int ij = tid - el * NP2;
  const int i = ij % NP, j = ij / NP;
  const int64_t el_local = (int64_t)lb * EPB + el;
  const bool active = (el < EPB) && (el_local < a.ne);
  const int elc = el < EPB ? el : 0;
  const int64_t e = a.e0 + el_local;

  const SEM_GLOBAL T* Dgl = gl(Dg);
  // FP64 at N >= 8: the four per-lane rows of Dhat would take 8 NP registers
  // and leave one wave per SIMD; they are read from LDS instead
  constexpr bool DLDS = sizeof(T) == 8 && N >= 8;
  __shared__ T s_D[DLDS ? NP2 : 1];
  T Dr[DLDS ? 1 : NP], Ds[DLDS ? 1 : NP], DrT[DLDS ? 1 : NP], DsT[DLDS ? 1 : NP];
  if constexpr (DLDS) {
    for (int t = tid; t < NP2; t += C::THREADS) s_D[t] = Dgl[t];
  } else {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      Dr[q] = Dgl[i * NP + q];
      Ds[q] = Dgl[j * NP + q];
      DrT[q] = Dgl[q * NP + i];
      DsT[q] = Dgl[q * NP + j];
    }
  }
  auto dr = [&](int q) -> T { if constexpr (DLDS) return s_D[i * NP + q]; else return Dr[q]; };
  auto ds = [&](int q) -> T { if constexpr (DLDS) return s_D[j * NP + q]; else return Ds[q]; };
  auto drt = [&](int q) -> T { if constexpr (DLDS) return s_D[q * NP + i]; else return DrT[q]; };
  auto dst = [&](int q) -> T { if constexpr (DLDS) return s_D[q * NP + j]; else return DsT[q]; };

  // issue every load of the column up front: u (NP values) and the six
  // geometric factors (6 NP values), so a wave has its whole element in flight
  T uk[NP], gk[6][NP];
  if (active) {
    const SEM_GLOBAL T* up = gl(a.u) + e * NP3 + ij;
    const SEM_GLOBAL T* gp = gl(a.G) + e * 6 * NP3 + ij;
#pragma unroll
    for (int k = 0; k < NP; ++k) uk[k] = __builtin_nontemporal_load(up + k * NP2);
    // k-major issue order: the factors of slice k arrive before those of k+1
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int m = 0; m < 6; ++m) gk[m][k] = __builtin_nontemporal_load(gp + m * NP3 + k * NP2);
#pragma unroll
    for (int k = 0; k < NP; ++k) s_u[elc][k][j][i] = uk[k];
  }
  lds_sync<C::THREADS>();

  T wt[NP];
  if (active) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T ur = 0, us = 0, ut = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        ur += dr(q) * s_u[elc][k][j][q];
        us += ds(q) * s_u[elc][k][q][i];
        ut += Dgl[k * NP + q] * uk[q];
      }
      const T grr = gk[0][k], grs = gk[1][k], grt = gk[2][k];
      const T gss = gk[3][k], gst = gk[4][k], gtt = gk[5][k];
      s_wr[elc][k][j][i] = grr * ur + grs * us + grt * ut;
      s_ws[elc][k][j][i] = grs * ur + gss * us + gst * ut;
      wt[k] = grt * ur + gst * us + gtt * ut;
    }
  }
  lds_sync<C::THREADS>();

  double dsum = 0.0;
  if (active) {
    SEM_GLOBAL T* out = gl(a.Au) + e * NP3 + ij;
    T bk[NP];
    if constexpr (HELM) {
      const SEM_GLOBAL T* Bp = gl(a.B) + e * NP3 + ij;
#pragma unroll
      for (int k = 0; k < NP; ++k) bk[k] = (T)a.lambda * Bp[k * NP2];
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T au = 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        au += drt(q) * s_wr[elc][k][j][q];
        au += dst(q) * s_ws[elc][k][q][i];
        au += Dgl[q * NP + k] * wt[q];
      }
      if constexpr (HELM) au += bk[k] * uk[k];
      __builtin_nontemporal_store(au, out + k * NP2);
      dsum += (double)uk[k] * (double)au;
    }
  }
  if (a.partial) {
    double s = block_sum<C::THREADS>(dsum, s_red);
    if (tid == 0) gl(a.partial)[lb] = s;
  }
}

// ax-kernel-end

int ax_blocks(int N, int64_t ne, bool f32) {
  int epb = 1;
  switch (N) {
#define SEM_EPB_CASE(n) case n: epb = f32 ? AxCfg<n, float>::EPB : AxCfg<n, double>::EPB; break;
    SEM_EPB_CASE(1) SEM_EPB_CASE(2) SEM_EPB_CASE(3) SEM_EPB_CASE(4) SEM_EPB_CASE(5)
    SEM_EPB_CASE(6) SEM_EPB_CASE(7) SEM_EPB_CASE(8) SEM_EPB_CASE(9) SEM_EPB_CASE(10)
    SEM_EPB_CASE(11) SEM_EPB_CASE(12) SEM_EPB_CASE(13) SEM_EPB_CASE(14) SEM_EPB_CASE(15)
#undef SEM_EPB_CASE
    default: break;
  }
  return (int)((ne + epb - 1) / epb);
}

template <typename T>
void launch_ax(int N, const Table<AxArgs<T>>& t, int64_t total_blocks, const T* D, hipStream_t s, bool helm) {
  if (total_blocks <= 0) return;
  if (t.many == nullptr && t.one.B != nullptr) helm = true;
  switch (N) {
#define SEM_AX_CASE(n)                                                                        \
  case n:                                                                                     \
    if (helm)                                                                                 \
      hipLaunchKernelGGL((k_ax<n, T, true>), dim3((unsigned)total_blocks), dim3(AxCfg<n, T>::THREADS), 0, s, t, D); \
    else                                                                                      \
      hipLaunchKernelGGL((k_ax<n, T, false>), dim3((unsigned)total_blocks), dim3(AxCfg<n, T>::THREADS), 0, s, t, D); \
    break;
    SEM_AX_CASE(1) SEM_AX_CASE(2) SEM_AX_CASE(3) SEM_AX_CASE(4) SEM_AX_CASE(5)
    SEM_AX_CASE(6) SEM_AX_CASE(7) SEM_AX_CASE(8) SEM_AX_CASE(9) SEM_AX_CASE(10)
    SEM_AX_CASE(11) SEM_AX_CASE(12) SEM_AX_CASE(13) SEM_AX_CASE(14) SEM_AX_CASE(15)
#undef SEM_AX_CASE
    default:
      fail(SEM_EINVAL, "Ax: unsupported order N=%d", N);
  }
  SEM_HIP(hipGetLastError());
}
template void launch_ax<double>(int, const Table<AxArgs<double>>&, int64_t, const double*, hipStream_t, bool);
template void launch_ax<float>(int, const Table<AxArgs<float>>&, int64_t, const float*, hipStream_t, bool);

// ---------------------------------------------------------------------------
// gather-scatter
// ---------------------------------------------------------------------------
constexpr int kGsThreads = 128;

template <typename T>
__global__ __launch_bounds__(kGsThreads) void k_gs(Table<GsArgs<T>> tab) {
  int lb;
  const GsArgs<T> a = fetch_args(tab, xcd_block(blockIdx.x, gridDim.x), lb);
  if (skipped(a.skip)) return;
  SEM_GLOBAL T* v = gl(a.v);
  const SEM_GLOBAL int* idx = gl(a.idx);
  const int64_t t = (int64_t)lb * kGsThreads + threadIdx.x;
  if (t < a.n_shared) {
    const int q0 = gl(a.off)[t], q1 = gl(a.off)[t + 1];
    const int c = q1 - q0;
    if (a.mask && gl(a.sdir)[t]) {
      for (int q = q0; q < q1; ++q) v[idx[q]] = T(0);
    } else if (c <= 8) {
      // conforming hex meshes: at most 8 copies; issue all loads together
      int id[8];
      T val[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) id[q] = q < c ? idx[q0 + q] : 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) val[q] = q < c ? v[id[q]] : T(0);
      T sum = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) if (q < c) sum += val[q];
#pragma unroll
      for (int q = 0; q < 8; ++q) if (q < c) v[id[q]] = sum;
    } else {
      T sum = 0;
      for (int q = q0; q < q1; ++q) sum += v[idx[q]];
      for (int q = q0; q < q1; ++q) v[idx[q]] = sum;
    }
  } else if (a.mask) {
    const int64_t d = t - a.n_shared;
    if (d < a.n_dir) v[gl(a.dir_idx)[d]] = T(0);
  }
}

int64_t gs_blocks(int64_t n_shared, int64_t n_dir) {
  return (n_shared + n_dir + kGsThreads - 1) / kGsThreads;
}

template <typename T>
void launch_gs(const Table<GsArgs<T>>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL((k_gs<T>), dim3((unsigned)total_blocks), dim3(kGsThreads), 0, s, t);
  SEM_HIP(hipGetLastError());
}
template void launch_gs<double>(const Table<GsArgs<double>>&, int64_t, hipStream_t);
template void launch_gs<float>(const Table<GsArgs<float>>&, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// vector updates
// ---------------------------------------------------------------------------
constexpr int kVecThreads = 256;
constexpr int kVecPer = 8;

// points per thread: few for small vectors (enough blocks to fill 256 CUs),
// more for large ones (fewer partial sums to reduce)
__host__ __device__ __forceinline__ int vec_per(int64_t n) {
  return n >= (int64_t(1) << 24) ? 8 : n >= (int64_t(1) << 21) ? 4 : n >= (int64_t(1) << 19) ? 2 : 1;
}

int64_t vec_blocks(int64_t n) {
  const int64_t chunk = (int64_t)kVecThreads * vec_per(n);
  return (n + chunk - 1) / chunk;
}

// operands each vector op reads (bit mask), so all of a thread's loads are
// issued before any of its stores
enum : unsigned {
  RD_X = 1, RD_R = 2, RD_P = 4, RD_W = 8, RD_Z = 16, RD_T = 32, RD_RES = 64, RD_D = 128, RD_DINV = 256,
  RD_IN64 = 512, RD_W64 = 1024, RD_OWN = 2048
};
constexpr unsigned vec_reads(int op) {
  switch (op) {
    case V_PCG_UPDATE: return RD_X | RD_P | RD_R | RD_W | RD_OWN | RD_DINV;
    case V_P_JACOBI: return RD_DINV | RD_R | RD_P;
    case V_P_FLEX: return RD_Z | RD_P;
    case V_DOT2: return RD_OWN | RD_Z | RD_W | RD_R;
    case V_DOT1: return RD_OWN | RD_R;
    case V_RZ_JACOBI: return RD_DINV | RD_R | RD_OWN;
    case V_CHEB_INIT0: return RD_DINV | RD_R;
    case V_CHEB_INITX: return RD_R | RD_T | RD_DINV | RD_X;
    case V_CHEB_STEP0: return RD_R | RD_T | RD_D | RD_DINV | RD_X;
    case V_CHEB_STEP: return RD_RES | RD_T | RD_D | RD_DINV | RD_X;
    case V_CHEB_INIT0D: return RD_DINV | RD_R;
    case V_CHEB_INIT0D_IN64: return RD_IN64 | RD_DINV;
    case V_CHEB_STEP0X: return RD_R | RD_T | RD_D | RD_DINV;
    case V_CHEB_LAST0X: return RD_D | RD_DINV | RD_R | RD_T;
    case V_CHEB_LAST: return RD_X | RD_D | RD_DINV | RD_RES | RD_T;
    case V_CHEB_LAST_OUT64: return RD_X | RD_D | RD_DINV | RD_RES | RD_T | RD_OWN | RD_W64 | RD_IN64;
    case V_CHEB_INITX_LAST: return RD_X | RD_DINV | RD_R | RD_T;
    case V_CHEB_INITX_OUT64: return RD_X | RD_DINV | RD_R | RD_T | RD_OWN | RD_W64 | RD_IN64;
    case V_RES0: return RD_R | RD_T;
    case V_RES: return RD_RES | RD_T;
    case V_CHEB_UPD: return RD_D | RD_DINV | RD_R | RD_X;
    case V_CHEB_UPD0: return RD_DINV | RD_R | RD_X;
    case V_CHEB_UPD_OUT64: return RD_D | RD_DINV | RD_R | RD_X | RD_OWN | RD_W64 | RD_IN64;
    case V_CHEB_UPD0_OUT64: return RD_DINV | RD_R | RD_X | RD_OWN | RD_W64 | RD_IN64;
    case V_COPY: return RD_R;
    case V_SCALE_DINV: return RD_DINV | RD_R;
    case V_NORMALIZE: return RD_R;
    case V_TRUE_RES: return RD_OWN | RD_R | RD_T;
    case V_DIV_DINV: return RD_DINV | RD_R;
    case V_SCALE: return RD_R;
    case V_AXPY: return RD_X | RD_R;
    default: return 0;  // V_ZERO, V_FILL
  }
}

template <typename P>
__device__ __forceinline__ P vld(const SEM_GLOBAL P* a, int64_t l) {
  return __builtin_nontemporal_load(a + l);
}
template <typename P>
__device__ __forceinline__ void vst(SEM_GLOBAL P* a, int64_t l, P v) {
  __builtin_nontemporal_store(v, a + l);
}

template <typename T, int OP>
__global__ __launch_bounds__(kVecThreads) void k_vec(Table<VecArgs<T>> tab) {
  __shared__ double s_red[2][kVecThreads / 64];
  int lb;
  const VecArgs<T> a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  SEM_GLOBAL T* X = gl(a.x);
  SEM_GLOBAL T* R = gl(a.r);
  SEM_GLOBAL T* P = gl(a.p);
  SEM_GLOBAL T* W = gl(a.w);
  SEM_GLOBAL T* Z = gl(a.z);
  SEM_GLOBAL T* Tt = gl(a.t);
  SEM_GLOBAL T* RES = gl(a.res);
  SEM_GLOBAL T* Dd = gl(a.d);
  const SEM_GLOBAL T* DINV = gl(a.dinv);
  const SEM_GLOBAL uint8_t* OWN = gl(a.owner);  // null: every entry counts (unique-DOF vectors)
  const int per = vec_per(a.n);
  const int64_t base = (int64_t)lb * kVecThreads * per + threadIdx.x;
  double acc0 = 0.0, acc1 = 0.0;
  T alpha = 0, beta = 0, scale = 0;
  if constexpr (OP == V_PCG_UPDATE) alpha = (T)gl(a.scal)[S_ALPHA];
  if constexpr (OP == V_P_JACOBI || OP == V_P_FLEX) beta = (T)gl(a.scal)[S_BETA];
  if constexpr (OP == V_NORMALIZE) scale = (T)gl(a.scal)[S_TMP];
  const T c0 = (T)a.c0, c1 = (T)a.c1, c2 = (T)a.c2;
  constexpr unsigned RD = vec_reads(OP);
  // every point a thread owns touches only its own index, so all loads may
  // go first even where two of the vectors alias (in-place updates)
  T xv[kVecPer], rv[kVecPer], pv[kVecPer], wv[kVecPer], zv[kVecPer], tv[kVecPer], resv[kVecPer], dv[kVecPer],
      dinvv[kVecPer];
  double in64v[kVecPer], w64v[kVecPer];
  bool own[kVecPer], ok[kVecPer];
#pragma unroll
  for (int q = 0; q < kVecPer; ++q) {
    const int64_t l = base + (int64_t)q * kVecThreads;
    ok[q] = q < per && l < a.n;
    if (!ok[q]) continue;
    if constexpr ((RD & RD_X) != 0) xv[q] = vld(X, l);
    if constexpr ((RD & RD_R) != 0) rv[q] = vld(R, l);
    if constexpr ((RD & RD_P) != 0) pv[q] = vld(P, l);
    if constexpr ((RD & RD_W) != 0) wv[q] = vld(W, l);
    if constexpr ((RD & RD_Z) != 0) zv[q] = vld(Z, l);
    if constexpr ((RD & RD_T) != 0) tv[q] = vld(Tt, l);
    if constexpr ((RD & RD_RES) != 0) resv[q] = vld(RES, l);
    if constexpr ((RD & RD_D) != 0) dv[q] = vld(Dd, l);
    if constexpr ((RD & RD_DINV) != 0) dinvv[q] = DINV ? vld(DINV, l) : T(0);
    if constexpr ((RD & RD_IN64) != 0) in64v[q] = vld(gl(a.in64), l);
    if constexpr ((RD & RD_W64) != 0) w64v[q] = vld(gl(a.w64), l);
    if constexpr ((RD & RD_OWN) != 0) own[q] = !OWN || vld(OWN, l);
  }
#pragma unroll
  for (int q = 0; q < kVecPer; ++q) {
    if (!ok[q]) continue;
    const int64_t l = base + (int64_t)q * kVecThreads;
    if constexpr (OP == V_PCG_UPDATE) {
      vst(X, l, xv[q] + alpha * pv[q]);
      const T rn = rv[q] - alpha * wv[q];
      vst(R, l, rn);
      if (own[q]) {
        acc0 += (double)rn * (double)rn;
        if (DINV) acc1 += (double)rn * (double)dinvv[q] * (double)rn;
      }
    } else if constexpr (OP == V_P_JACOBI) {
      vst(P, l, dinvv[q] * rv[q] + beta * pv[q]);
    } else if constexpr (OP == V_P_FLEX) {
      vst(P, l, zv[q] + beta * pv[q]);
    } else if constexpr (OP == V_DOT2) {
      if (own[q]) {
        const double zl = (double)zv[q];
        acc0 += zl * (double)wv[q];
        acc1 += zl * (double)rv[q];
      }
    } else if constexpr (OP == V_DOT1) {
      if (own[q]) acc0 += (double)rv[q] * (double)rv[q];
    } else if constexpr (OP == V_RZ_JACOBI) {
      const T pz = dinvv[q] * rv[q];
      vst(P, l, pz);
      if (own[q]) acc0 += (double)rv[q] * (double)pz;
    } else if constexpr (OP == V_CHEB_INIT0) {
      const T d = c0 * dinvv[q] * rv[q];
      vst(Dd, l, d);
      vst(X, l, d);
    } else if constexpr (OP == V_CHEB_INITX) {
      const T res = rv[q] - tv[q];
      vst(RES, l, res);
      const T d = c0 * dinvv[q] * res;
      vst(Dd, l, d);
      vst(X, l, xv[q] + d);
    } else if constexpr (OP == V_CHEB_STEP0) {
      const T res = rv[q] - tv[q];
      vst(RES, l, res);
      const T d = c1 * dv[q] + c2 * dinvv[q] * res;
      vst(Dd, l, d);
      vst(X, l, xv[q] + d);
    } else if constexpr (OP == V_CHEB_STEP) {
      const T res = resv[q] - tv[q];
      vst(RES, l, res);
      const T d = c1 * dv[q] + c2 * dinvv[q] * res;
      vst(Dd, l, d);
      vst(X, l, xv[q] + d);
    } else if constexpr (OP == V_CHEB_INIT0D) {
      vst(Dd, l, c0 * dinvv[q] * rv[q]);
    } else if constexpr (OP == V_CHEB_INIT0D_IN64) {
      const T r = (T)in64v[q];
      vst(R, l, r);
      vst(Dd, l, c0 * dinvv[q] * r);
    } else if constexpr (OP == V_CHEB_STEP0X) {
      const T res = rv[q] - tv[q];
      vst(RES, l, res);
      const T dold = dv[q];
      const T d = c1 * dold + c2 * dinvv[q] * res;
      vst(Dd, l, d);
      vst(X, l, dold + d);
    } else if constexpr (OP == V_CHEB_LAST0X) {
      const T dold = dv[q];
      vst(X, l, dold + (c1 * dold + c2 * dinvv[q] * (rv[q] - tv[q])));
    } else if constexpr (OP == V_CHEB_LAST) {
      vst(X, l, xv[q] + (c1 * dv[q] + c2 * dinvv[q] * (resv[q] - tv[q])));
    } else if constexpr (OP == V_CHEB_LAST_OUT64) {
      const double z = (double)(xv[q] + (c1 * dv[q] + c2 * dinvv[q] * (resv[q] - tv[q])));
      vst(gl(a.out64), l, z);
      if (own[q]) {
        acc0 += z * w64v[q];
        acc1 += z * in64v[q];
      }
    } else if constexpr (OP == V_CHEB_INITX_LAST) {
      vst(X, l, xv[q] + c0 * dinvv[q] * (rv[q] - tv[q]));
    } else if constexpr (OP == V_CHEB_INITX_OUT64) {
      const double z = (double)(xv[q] + c0 * dinvv[q] * (rv[q] - tv[q]));
      vst(gl(a.out64), l, z);
      if (own[q]) {
        acc0 += z * w64v[q];
        acc1 += z * in64v[q];
      }
    } else if constexpr (OP == V_RES0) {
      vst(RES, l, rv[q] - tv[q]);
    } else if constexpr (OP == V_RES) {
      vst(RES, l, resv[q] - tv[q]);
    } else if constexpr (OP == V_CHEB_UPD) {
      const T d = c1 * dv[q] + c2 * dinvv[q] * rv[q];
      vst(Dd, l, d);
      vst(X, l, xv[q] + d);
    } else if constexpr (OP == V_CHEB_UPD0) {
      const T d = c2 * dinvv[q] * rv[q];
      vst(Dd, l, d);
      vst(X, l, xv[q] + d);
    } else if constexpr (OP == V_CHEB_UPD_OUT64 || OP == V_CHEB_UPD0_OUT64) {
      T d;
      if constexpr (OP == V_CHEB_UPD_OUT64) d = c1 * dv[q] + c2 * dinvv[q] * rv[q];  // as V_CHEB_UPD
      else d = c2 * dinvv[q] * rv[q];
      const double z = (double)(xv[q] + d);
      vst(gl(a.out64), l, z);
      if (own[q]) {
        acc0 += z * w64v[q];
        acc1 += z * in64v[q];
      }
    } else if constexpr (OP == V_ZERO) {
      vst(X, l, T(0));
    } else if constexpr (OP == V_FILL) {
      vst(X, l, c0);
    } else if constexpr (OP == V_COPY) {
      vst(X, l, rv[q]);
    } else if constexpr (OP == V_SCALE_DINV) {
      vst(X, l, dinvv[q] * rv[q]);
    } else if constexpr (OP == V_NORMALIZE) {
      vst(X, l, rv[q] * scale);
    } else if constexpr (OP == V_TRUE_RES) {
      if (own[q]) {
        const double e = (double)rv[q] - (double)tv[q];
        acc0 += e * e;
      }
    } else if constexpr (OP == V_DIV_DINV) {
      vst(X, l, dinvv[q] != T(0) ? rv[q] / dinvv[q] : T(0));
    } else if constexpr (OP == V_SCALE) {
      vst(X, l, c0 * rv[q]);
    } else if constexpr (OP == V_AXPY) {
      vst(X, l, xv[q] + c0 * rv[q]);
    }
  }
  constexpr bool RED = (OP == V_PCG_UPDATE || OP == V_DOT2 || OP == V_DOT1 || OP == V_RZ_JACOBI ||
                        OP == V_TRUE_RES || OP == V_CHEB_LAST_OUT64 || OP == V_CHEB_INITX_OUT64 ||
                        OP == V_CHEB_UPD_OUT64 || OP == V_CHEB_UPD0_OUT64);
  if constexpr (RED) {
    double s0 = wave_sum(acc0), s1 = wave_sum(acc1);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { s_red[0][wid] = s0; s_red[1][wid] = s1; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int k = 0; k < kVecThreads / 64; ++k) { t0 += s_red[0][k]; t1 += s_red[1][k]; }
      gl(a.partial)[lb] = t0;
      gl(a.partial)[a.stride + lb] = t1;
    }
  }
}

template <typename T>
void launch_vec(VecOp op, const Table<VecArgs<T>>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  const dim3 g((unsigned)total_blocks), b(kVecThreads);
  switch (op) {
#define SEM_VEC_CASE(o) case o: hipLaunchKernelGGL((k_vec<T, o>), g, b, 0, s, t); break;
    SEM_VEC_CASE(V_PCG_UPDATE) SEM_VEC_CASE(V_P_JACOBI) SEM_VEC_CASE(V_P_FLEX)
    SEM_VEC_CASE(V_DOT2) SEM_VEC_CASE(V_DOT1) SEM_VEC_CASE(V_RZ_JACOBI)
    SEM_VEC_CASE(V_CHEB_INIT0) SEM_VEC_CASE(V_CHEB_INITX) SEM_VEC_CASE(V_CHEB_STEP0)
    SEM_VEC_CASE(V_CHEB_STEP) SEM_VEC_CASE(V_ZERO) SEM_VEC_CASE(V_COPY)
    SEM_VEC_CASE(V_SCALE_DINV) SEM_VEC_CASE(V_NORMALIZE) SEM_VEC_CASE(V_TRUE_RES)
    SEM_VEC_CASE(V_DIV_DINV) SEM_VEC_CASE(V_SCALE) SEM_VEC_CASE(V_AXPY)
    SEM_VEC_CASE(V_RES0) SEM_VEC_CASE(V_RES) SEM_VEC_CASE(V_CHEB_UPD) SEM_VEC_CASE(V_CHEB_UPD0) SEM_VEC_CASE(V_FILL)
    SEM_VEC_CASE(V_CHEB_INIT0D) SEM_VEC_CASE(V_CHEB_INIT0D_IN64) SEM_VEC_CASE(V_CHEB_STEP0X)
    SEM_VEC_CASE(V_CHEB_LAST0X) SEM_VEC_CASE(V_CHEB_LAST) SEM_VEC_CASE(V_CHEB_LAST_OUT64)
    SEM_VEC_CASE(V_CHEB_INITX_LAST) SEM_VEC_CASE(V_CHEB_INITX_OUT64)
    SEM_VEC_CASE(V_CHEB_UPD_OUT64) SEM_VEC_CASE(V_CHEB_UPD0_OUT64)
#undef SEM_VEC_CASE
    default:
      fail(SEM_EINVAL, "unknown vector op %d", (int)op);
  }
  SEM_HIP(hipGetLastError());
}
template void launch_vec<double>(VecOp, const Table<VecArgs<double>>&, int64_t, hipStream_t);
template void launch_vec<float>(VecOp, const Table<VecArgs<float>>&, int64_t, hipStream_t);

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kVecThreads) void k_cast(Table<CastArgs<Tin, Tout>> tab) {
  int lb;
  const CastArgs<Tin, Tout> a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  const int per = vec_per(a.n);
  const int64_t base = (int64_t)lb * kVecThreads * per + threadIdx.x;
#pragma unroll
  for (int q = 0; q < kVecPer; ++q) {
    const int64_t l = base + (int64_t)q * kVecThreads;
    if (q < per && l < a.n) gl(a.out)[l] = (Tout)gl(a.in)[l];
  }
}

template <typename Tin, typename Tout>
void launch_cast(const Table<CastArgs<Tin, Tout>>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3((unsigned)total_blocks), dim3(kVecThreads), 0, s, t);
  SEM_HIP(hipGetLastError());
}
template void launch_cast<double, float>(const Table<CastArgs<double, float>>&, int64_t, hipStream_t);
template void launch_cast<float, double>(const Table<CastArgs<float, double>>&, int64_t, hipStream_t);
template void launch_cast<double, double>(const Table<CastArgs<double, double>>&, int64_t, hipStream_t);
template void launch_cast<float, float>(const Table<CastArgs<float, float>>&, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// finalize: per-problem fixed-order reduction + scalar recurrences
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFinThreads) void k_fin(Table<FinArgs> tab, int op) {
  __shared__ double s_red[2][kFinThreads / 64];
  FinArgs a = tab.one;
  if (tab.many) a = gl(tab.many)[blockIdx.x];
  if (skipped(a.skip)) return;
  double s0 = 0.0, s1 = 0.0;
  const SEM_GLOBAL double* part = gl(a.partial);
  // thread t sums partials t, t+T, t+2T, ... into 4 interleaved accumulators
  // (independent loads in flight), then a fixed butterfly + wave-order sum
  constexpr int T4 = 4 * kFinThreads;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
  int64_t k = threadIdx.x;
  for (; k + 3 * kFinThreads < a.nblk; k += T4) {
    a0 += part[k];
    a1 += part[k + kFinThreads];
    a2 += part[k + 2 * kFinThreads];
    a3 += part[k + 3 * kFinThreads];
    b0 += part[a.stride + k];
    b1 += part[a.stride + k + kFinThreads];
    b2 += part[a.stride + k + 2 * kFinThreads];
    b3 += part[a.stride + k + 3 * kFinThreads];
  }
  for (; k < a.nblk; k += kFinThreads) {
    a0 += part[k];
    b0 += part[a.stride + k];
  }
  s0 = wave_sum((a0 + a1) + (a2 + a3));
  s1 = wave_sum((b0 + b1) + (b2 + b3));
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = s0;
    s_red[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s0 = 0.0;
    s1 = 0.0;
    for (int w = 0; w < kFinThreads / 64; ++w) {
      s0 += s_red[0][w];
      s1 += s_red[1][w];
    }
    s_red[0][0] = s0;
    s_red[1][0] = s1;
  }
  if (threadIdx.x != 0) return;
  s0 = s_red[0][0];
  s1 = s_red[1][0];
  SEM_GLOBAL double* sc = gl(a.scal);
  SEM_GLOBAL int* fl = gl(a.flags);
  switch (op) {
    case FIN_INIT:
      sc[S_BB] = s0;
      sc[S_RR] = s0;
      sc[S_BETA] = 0.0;
      sc[S_ALPHA] = 0.0;
      sc[S_RZ] = 0.0;
      fl[F_ITERS] = 0;
      fl[F_STATUS] = 1;
      fl[F_DONE] = 0;
      if (!isfinite(s0)) { fl[F_STATUS] = SEM_ENAN; fl[F_DONE] = 1; sc[S_RELRES] = s0; }
      else if (s0 == 0.0) { fl[F_STATUS] = SEM_OK; fl[F_DONE] = 1; sc[S_RELRES] = 0.0; }
      else sc[S_RELRES] = 1.0;
      break;
    case FIN_RZ:
      sc[S_RZ] = s0;
      sc[S_BETA] = 0.0;
      if (!isfinite(s0)) { fl[F_STATUS] = SEM_ENAN; fl[F_DONE] = 1; }
      break;
    case FIN_ALPHA: {
      sc[S_PW] = s0;
      const double al = sc[S_RZ] / s0;
      sc[S_ALPHA] = al;
      if (!isfinite(al)) { fl[F_STATUS] = SEM_ENAN; fl[F_DONE] = 1; sc[S_ALPHA] = 0.0; }
      break;
    }
    case FIN_CHECK:
    case FIN_CHECK_JACOBI: {
      sc[S_RR] = s0;
      const int it = ++fl[F_ITERS];
      if (a.total) ++(*gl(a.total));
      const double rel = sqrt(s0 / sc[S_BB]);
      sc[S_RELRES] = rel;
      if (!isfinite(s0)) { fl[F_STATUS] = SEM_ENAN; fl[F_DONE] = 1; }
      else if (a.fixed > 0) { if (it >= a.fixed) { fl[F_STATUS] = SEM_OK; fl[F_DONE] = 1; } }
      else if (rel <= a.rtol) { fl[F_STATUS] = SEM_OK; fl[F_DONE] = 1; }
      else if (it >= a.maxit) { fl[F_STATUS] = SEM_ENOCONV; fl[F_DONE] = 1; }
      if (op == FIN_CHECK_JACOBI && !fl[F_DONE]) {
        sc[S_BETA] = s1 / sc[S_RZ];
        sc[S_RZ] = s1;
      }
      break;
    }
    case FIN_BETA_FLEX:
      // (z_new, r_new - r_old) = -alpha (z_new, w) since r_new = r_old - alpha w
      sc[S_ZW] = s0;
      sc[S_RZ_NEW] = s1;
      sc[S_BETA] = fl[F_ITERS] == 0 ? 0.0 : -sc[S_ALPHA] * s0 / sc[S_RZ];
      sc[S_RZ] = s1;
      if (!isfinite(sc[S_BETA])) { fl[F_STATUS] = SEM_ENAN; fl[F_DONE] = 1; }
      break;
    case FIN_NORM:
      sc[S_TMP] = 1.0 / sqrt(s0);
      break;
    case FIN_STORE:
      sc[S_TMP] = s0;
      break;
    default:
      break;
  }
}

void launch_fin(FinOp op, const Table<FinArgs>& t, int nprob, hipStream_t s) {
  if (nprob <= 0) return;
  hipLaunchKernelGGL(k_fin, dim3(nprob), dim3(kFinThreads), 0, s, t, (int)op);
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// pMG transfers: out = (M x M x M) in per element, M is NO x NI
// ---------------------------------------------------------------------------
// one wave per block: an element's loads are all issued before its first
// LDS hand-off, and the hand-offs between the three passes stay inside a wave
constexpr int kXferThreads = 64;

template <int NI, int NO>
struct XferCfg {
  static constexpr int MAXC = (NI * NI * NI > NO * NO * NO) ? NI * NI * NI : NO * NO * NO;
  static constexpr int EPB = (kXferThreads / MAXC) > 0 ? (kXferThreads / MAXC) : 1;
  static constexpr int S0 = NI * NI * NI, S1 = NI * NI * NO, S2 = NI * NO * NO, S3 = NO * NO * NO;
};

// sum-factorised tensor apply on EPB elements staged in LDS
template <int NI, int NO, typename T>
__device__ __forceinline__ void tensor3(const T* sM, T (*s0)[XferCfg<NI, NO>::S0],
                                        T (*s1)[XferCfg<NI, NO>::S1], T (*s2)[XferCfg<NI, NO>::S2],
                                        T (*s3)[XferCfg<NI, NO>::S3]) {
  using C = XferCfg<NI, NO>;
  // along i: s1[k][j][a] = sum_i M[a][i] s0[k][j][i]
  for (int t = threadIdx.x; t < C::EPB * C::S1; t += kXferThreads) {
    const int el = t / C::S1, r = t - el * C::S1;
    const int aa = r % NO, kj = r / NO;
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NI; ++q) acc += sM[aa * NI + q] * s0[el][kj * NI + q];
    s1[el][r] = acc;
  }
  __syncthreads();
  // along j: s2[k][b][a] = sum_j M[b][j] s1[k][j][a]
  for (int t = threadIdx.x; t < C::EPB * C::S2; t += kXferThreads) {
    const int el = t / C::S2, r = t - el * C::S2;
    const int aa = r % NO, bb = (r / NO) % NO, k = r / (NO * NO);
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NI; ++q) acc += sM[bb * NI + q] * s1[el][(k * NI + q) * NO + aa];
    s2[el][r] = acc;
  }
  __syncthreads();
  // along k: s3[c][b][a] = sum_k M[c][k] s2[k][b][a]
  for (int t = threadIdx.x; t < C::EPB * C::S3; t += kXferThreads) {
    const int el = t / C::S3, r = t - el * C::S3;
    const int ba = r % (NO * NO), c = r / (NO * NO);
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NI; ++q) acc += sM[c * NI + q] * s2[el][q * NO * NO + ba];
    s3[el][r] = acc;
  }
  __syncthreads();
}

// DIR 0: prolong (NI = coarse, NO = fine): xf += M zc
// DIR 1: restrict (NI = fine, NO = coarse): out_c = M ((rf - tf) . owner)
template <int NI, int NO, typename Tf, typename Tc, int DIR>
__global__ __launch_bounds__(kXferThreads) void k_xfer(Table<XferArgs<Tf, Tc>> tab, const double* __restrict__ Mg) {
  using C = XferCfg<NI, NO>;
  __shared__ Tf sM[NO * NI];
  __shared__ Tf s0[C::EPB][C::S0];
  __shared__ Tf s1[C::EPB][C::S1];
  __shared__ Tf s2[C::EPB][C::S2];
  __shared__ Tf s3[C::EPB][C::S3];
  int lb;
  const XferArgs<Tf, Tc> a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  const int64_t e_first = (int64_t)lb * C::EPB;
  for (int t = threadIdx.x; t < NO * NI; t += kXferThreads) sM[t] = (Tf)Mg[t];
  // prolongation: the fine values that receive the correction are loaded up
  // front, so their latency overlaps the staging and the contraction
  constexpr int KO = (C::EPB * C::S3 + kXferThreads - 1) / kXferThreads;
  Tf xpre[KO];
  if constexpr (DIR == 0) {
#pragma unroll
    for (int k = 0; k < KO; ++k) {
      const int t = threadIdx.x + k * kXferThreads;
      const int el = t / C::S3, r = t - el * C::S3;
      const int64_t e = e_first + el;
      xpre[k] = (t < C::EPB * C::S3 && e < a.E) ? __builtin_nontemporal_load(gl(a.xf) + e * C::S3 + r) : Tf(0);
    }
  }
  // staging: every input of the thread's points loaded before any LDS store
  constexpr int KI = (C::EPB * C::S0 + kXferThreads - 1) / kXferThreads;
  Tf vin[KI], tin[KI];
  uint8_t oin[KI];
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int t = threadIdx.x + k * kXferThreads;
    const int el = t / C::S0, r = t - el * C::S0;
    const int64_t e = e_first + el;
    vin[k] = Tf(0);
    tin[k] = Tf(0);
    oin[k] = 0;
    if (t < C::EPB * C::S0 && e < a.E) {
      const int64_t g = e * C::S0 + r;
      if constexpr (DIR == 0) {
        vin[k] = (Tf)gl(a.zc)[a.umap_c ? (int64_t)gl(a.umap_c)[g] : g];
      } else {
        vin[k] = __builtin_nontemporal_load(gl(a.rf) + g);
        if (a.tf) tin[k] = __builtin_nontemporal_load(gl(a.tf) + g);
        oin[k] = __builtin_nontemporal_load(gl(a.owner_f) + g);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int t = threadIdx.x + k * kXferThreads;
    if (t >= C::EPB * C::S0) break;
    const int el = t / C::S0, r = t - el * C::S0;
    Tf v = vin[k];
    if constexpr (DIR == 1) v = oin[k] ? v - tin[k] : Tf(0);
    s0[el][r] = v;
  }
  __syncthreads();
  tensor3<NI, NO, Tf>(sM, s0, s1, s2, s3);
#pragma unroll
  for (int k = 0; k < KO; ++k) {
    const int t = threadIdx.x + k * kXferThreads;
    if (t >= C::EPB * C::S3) break;
    const int el = t / C::S3, r = t - el * C::S3;
    const int64_t e = e_first + el;
    if (e >= a.E) continue;
    const int64_t g = e * C::S3 + r;
    if constexpr (DIR == 0) __builtin_nontemporal_store(xpre[k] + s3[el][r], gl(a.xf) + g);
    else gl(a.out_c)[g] = (Tc)s3[el][r];
  }
}

template <int NI, int NO>
static int xfer_epb() { return XferCfg<NI, NO>::EPB; }

// supported level pairs (fine, coarse) with coarse < fine <= 15
// (the default schedules {N, (N-1)/2, 1}, every N -> 1, and the paper's
// 8-5-1 and 8-6-4-1 schedules)
#define SEM_FOR_PAIRS(X)                                                                      \
  X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(7, 1) X(8, 1) X(9, 1) X(10, 1) X(11, 1) X(12, 1)    \
  X(13, 1) X(14, 1) X(15, 1) X(5, 2) X(6, 2) X(7, 3) X(8, 3) X(9, 4) X(10, 4) X(11, 5)         \
  X(12, 5) X(13, 6) X(14, 6) X(15, 7) X(8, 5) X(8, 6) X(6, 4) X(7, 5) X(5, 3) X(9, 5) X(9, 7)

int xfer_blocks(int Nf, int Nc, int64_t E) {
  int epb = 0;
#define SEM_XB(f, c) if (Nf == f && Nc == c) epb = xfer_epb<c + 1, f + 1>();
  SEM_FOR_PAIRS(SEM_XB)
#undef SEM_XB
  if (epb == 0) fail(SEM_EINVAL, "pMG transfer %d->%d not supported", Nf, Nc);
  return (int)((E + epb - 1) / epb);
}

template <typename Tf, typename Tc>
void launch_xfer(int dir, int Nf, int Nc, const Table<XferArgs<Tf, Tc>>& t, int64_t total_blocks,
                 const double* M, hipStream_t s) {
  if (total_blocks <= 0) return;
  bool done = false;
#define SEM_XL(f, c)                                                                                    \
  if (!done && Nf == f && Nc == c) {                                                                    \
    done = true;                                                                                        \
    if (dir == 0)                                                                                       \
      hipLaunchKernelGGL((k_xfer<c + 1, f + 1, Tf, Tc, 0>), dim3((unsigned)total_blocks), dim3(kXferThreads), 0, s, t, M); \
    else                                                                                                \
      hipLaunchKernelGGL((k_xfer<f + 1, c + 1, Tf, Tc, 1>), dim3((unsigned)total_blocks), dim3(kXferThreads), 0, s, t, M); \
  }
  SEM_FOR_PAIRS(SEM_XL)
#undef SEM_XL
  if (!done) fail(SEM_EINVAL, "pMG transfer %d->%d not supported", Nf, Nc);
  SEM_HIP(hipGetLastError());
}
template void launch_xfer<float, float>(int, int, int, const Table<XferArgs<float, float>>&, int64_t, const double*, hipStream_t);
template void launch_xfer<float, double>(int, int, int, const Table<XferArgs<float, double>>&, int64_t, const double*, hipStream_t);
template void launch_xfer<double, double>(int, int, int, const Table<XferArgs<double, double>>&, int64_t, const double*, hipStream_t);

// ---------------------------------------------------------------------------
// unique-DOF operators of an assembled level
// ---------------------------------------------------------------------------
constexpr int kSpThreads = 256;

int64_t spmv_blocks(int64_t n) { return (n + kSpThreads - 1) / kSpThreads; }


// ---------------------------------------------------------------------------
// coarse-grid Jacobi-PCG, two launches per iteration (see CgArgs)
// ---------------------------------------------------------------------------
constexpr int kCgThreads = 256;
int64_t cg_update_blocks(int64_t n) { return (n + kCgThreads - 1) / kCgThreads; }

// sum of partial[0..nb) (and partial[stride..stride+nb) if two) in a fixed
// order; result valid in every thread
template <int THREADS>
__device__ __forceinline__ void block_sums2(const SEM_GLOBAL double* part, int64_t stride, int64_t nb, bool two,
                                            double& s0, double& s1, double (*red)[THREADS / 64]) {
  double a0 = 0.0, a1 = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += THREADS) {
    a0 += part[k];
    if (two) a1 += part[stride + k];
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a0;
    red[1][threadIdx.x >> 6] = a1;
  }
  __syncthreads();
  s0 = 0.0;
  s1 = 0.0;
  for (int q = 0; q < THREADS / 64; ++q) {
    s0 += red[0][q];
    s1 += red[1][q];
  }
}

// The p update fused into the SpMV. Every block decides convergence and beta
// (redundantly, from the same partials in the same order); then, with
// z = D^-1 r stored by the previous update, each row forms q_r = sum_k A_rk z_k
// and the new direction and its image row by row:
//   p_r = z_r + beta p_r,   w_r = q_r + beta w_r   (= (A p)_r),
// the block's partial of p . w included. Only z is gathered, and p and w are
// updated in place, so no block reads a value another block of the launch
// writes.
__global__ __launch_bounds__(kCgThreads) void k_cg_pspmv(Table<CgArgs> tab) {
  __shared__ double red[2][kCgThreads / 64];
  __shared__ int s_go;
  __shared__ double s_beta;
  int lb;
  const CgArgs a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  SEM_GLOBAL double* sc = gl(a.scal);
  SEM_GLOBAL int* fl = gl(a.flags);
  const int it = fl[a.par ? F_ITERS2 : F_ITERS];
  const bool first = it == 0;
  double rz_new = 0.0;
  if (!first) {
    double rr;
    block_sums2<kCgThreads>(gl(a.partial), a.stride, a.nblk_upd, true, rr, rz_new, red);
    if (threadIdx.x == 0) {
      const double rel = sqrt(rr / sc[S_BB]);
      int status = 1;
      if (!isfinite(rr) || !isfinite(rz_new)) status = SEM_ENAN;
      else if (a.fixed > 0) { if (it >= a.fixed) status = SEM_OK; }
      else if (rel <= a.rtol) status = SEM_OK;
      else if (it >= a.maxit) status = SEM_ENOCONV;
      s_go = status == 1;
      s_beta = rz_new / sc[a.par ? S_RZ_NEW : S_RZ];
      if (status != 1 && lb == 0) {
        sc[S_RR] = rr;
        sc[S_RELRES] = rel;
        fl[F_STATUS] = status;
        fl[F_DONE] = 1;
      }
    }
  } else if (threadIdx.x == 0) {
    s_go = 1;
    s_beta = 0.0;
  }
  __syncthreads();
  if (!s_go) return;
  const double beta = s_beta;
  if (lb == 0 && threadIdx.x == 0) {
    // ring slots the other parity reads: rz of the new p, iteration count
    sc[a.par ? S_RZ : S_RZ_NEW] = first ? sc[S_RZ] : rz_new;
    fl[a.par ? F_ITERS : F_ITERS2] = it + 1;
    if (a.total) ++(*gl(a.total));
  }
  const SEM_GLOBAL double* zv = gl(a.z);
  const int64_t i = (int64_t)lb * kCgThreads + threadIdx.x;
  double d = 0.0;
  if (i < a.n) {
    const SEM_GLOBAL int* col = gl(a.col) + i;
    const SEM_GLOBAL double* val = gl(a.val) + i;
    double q = 0.0;
    int k = 0;
    for (; k + 9 <= a.W; k += 9) {
      double v[9];
      int c[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) {  // the matrix is re-read every coarse iteration: keep it cached
        v[j] = val[(int64_t)(k + j) * a.n];
        c[j] = col[(int64_t)(k + j) * a.n];
      }
      double zc[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) zc[j] = zv[c[j]];
#pragma unroll
      for (int j = 0; j < 9; ++j) q += v[j] * zc[j];
    }
    for (; k < a.W; ++k) q += val[(int64_t)k * a.n] * zv[col[(int64_t)k * a.n]];
    SEM_GLOBAL double* P = gl(a.p);
    SEM_GLOBAL double* Wv = gl(a.w);
    const double pi = first ? zv[i] : zv[i] + beta * P[i];
    const double wi = first ? q : q + beta * Wv[i];
    P[i] = pi;
    Wv[i] = wi;
    d = pi * wi;
  }
  const double sblk = block_sum<kCgThreads>(d, red[0]);
  if (threadIdx.x == 0) gl(a.partial)[2 * a.stride + lb] = sblk;
}

__global__ __launch_bounds__(kCgThreads) void k_cg_update(Table<CgArgs> tab) {
  __shared__ double red[2][kCgThreads / 64];
  int lb;
  const CgArgs a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  double pw, unused;
  block_sums2<kCgThreads>(gl(a.partial) + 2 * a.stride, 0, a.nblk_sp, false, pw, unused, red);
  const double alpha = gl(a.scal)[a.par ? S_RZ : S_RZ_NEW] / pw;
  if (!isfinite(alpha)) {
    if (lb == 0 && threadIdx.x == 0) {
      gl(a.flags)[F_STATUS] = SEM_ENAN;
      gl(a.flags)[F_DONE] = 1;
    }
    return;
  }
  const int64_t i = (int64_t)lb * kCgThreads + threadIdx.x;
  double rr = 0.0, rz = 0.0;
  if (i < a.n) {
    const double pi = gl(a.p)[i];
    gl(a.x)[i] += alpha * pi;
    const double rn = gl(a.r)[i] - alpha * gl(a.w)[i];
    gl(a.r)[i] = rn;
    const double zn = gl(a.dinv)[i] * rn;
    gl(a.z)[i] = zn;  // the next iteration's SpMV gathers z
    rr = rn * rn;
    rz = zn * rn;
  }
  __syncthreads();  // red is reused
  double s0 = wave_sum(rr), s1 = wave_sum(rz);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s0;
    red[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < kCgThreads / 64; ++q) {
      t0 += red[0][q];
      t1 += red[1][q];
    }
    gl(a.partial)[lb] = t0;
    gl(a.partial)[a.stride + lb] = t1;
  }
}

void launch_cg_pspmv(const Table<CgArgs>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(k_cg_pspmv, dim3((unsigned)total_blocks), dim3(kCgThreads), 0, s, t);
  SEM_HIP(hipGetLastError());
}

void launch_cg_update(const Table<CgArgs>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(k_cg_update, dim3((unsigned)total_blocks), dim3(kCgThreads), 0, s, t);
  SEM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kSpThreads) void k_usum(Table<UsumArgs> tab) {
  int lb;
  const UsumArgs a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  const int64_t r = (int64_t)lb * kSpThreads + threadIdx.x;
  if (r >= a.n) return;
  double s = 0.0;
  if (!gl(a.udir)[r]) {
    const SEM_GLOBAL int* idx = gl(a.idx);
    const SEM_GLOBAL double* in = gl(a.in);
    const int q1 = gl(a.off)[r + 1];
    for (int q = gl(a.off)[r]; q < q1; ++q) s += in[idx[q]];
  }
  gl(a.out)[r] = s;
}

void launch_usum(const Table<UsumArgs>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(k_usum, dim3((unsigned)total_blocks), dim3(kSpThreads), 0, s, t);
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// projection space: multi-dot, per-component reduction, linear combination
// ---------------------------------------------------------------------------
constexpr int kMdotKC = 8;  // components per block (blockIdx.y picks the group)

__global__ __launch_bounds__(kVecThreads) void k_mdot(MdotArgs a) {
  __shared__ double s_red[kMdotKC][kVecThreads / 64];
  const int k0 = blockIdx.y * kMdotKC;
  const int per = vec_per(a.n);
  const int64_t base = (int64_t)blockIdx.x * kVecThreads * per + threadIdx.x;
  const SEM_GLOBAL double* Y = gl(a.y);
  const SEM_GLOBAL uint8_t* OWN = gl(a.owner);
  double acc[kMdotKC];
#pragma unroll
  for (int c = 0; c < kMdotKC; ++c) acc[c] = 0.0;
  for (int q = 0; q < per; ++q) {
    const int64_t l = base + (int64_t)q * kVecThreads;
    if (l >= a.n) break;
    if (!OWN[l]) continue;
    const double y = Y[l];
#pragma unroll
    for (int c = 0; c < kMdotKC; ++c)
      if (k0 + c < a.K) acc[c] += gl(gl(a.v)[k0 + c])[l] * y;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kMdotKC; ++c) {
    const double sc = wave_sum(acc[c]);
    if (lane == 0) s_red[c][wid] = sc;
  }
  __syncthreads();
  if (threadIdx.x < kMdotKC && k0 + (int)threadIdx.x < a.K) {
    double t = 0.0;
    for (int w = 0; w < kVecThreads / 64; ++w) t += s_red[threadIdx.x][w];
    gl(a.partial)[(int64_t)(k0 + threadIdx.x) * a.stride + blockIdx.x] = t;
  }
}

void launch_mdot(const MdotArgs& a, hipStream_t s) {
  if (a.K <= 0 || a.n <= 0) return;
  const dim3 g((unsigned)vec_blocks(a.n), (unsigned)((a.K + kMdotKC - 1) / kMdotKC));
  hipLaunchKernelGGL(k_mdot, g, dim3(kVecThreads), 0, s, a);
  SEM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kFinThreads) void k_mfin(const double* __restrict__ partial, int64_t stride,
                                                      int64_t nblk, double* out) {
  __shared__ double s_red[kFinThreads / 64];
  const SEM_GLOBAL double* part = gl(partial) + (int64_t)blockIdx.x * stride;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int64_t k = threadIdx.x;
  for (; k + 3 * kFinThreads < nblk; k += 4 * kFinThreads) {
    a0 += part[k];
    a1 += part[k + kFinThreads];
    a2 += part[k + 2 * kFinThreads];
    a3 += part[k + 3 * kFinThreads];
  }
  for (; k < nblk; k += kFinThreads) a0 += part[k];
  const double s = wave_sum((a0 + a1) + (a2 + a3));
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kFinThreads / 64; ++w) t += s_red[w];
    gl(out)[blockIdx.x] = t;
  }
}

void launch_mfin(const double* partial, int64_t stride, int64_t nblk, int K, double* out, hipStream_t s) {
  if (K <= 0) return;
  hipLaunchKernelGGL(k_mfin, dim3(K), dim3(kFinThreads), 0, s, partial, stride, nblk, out);
  SEM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kVecThreads) void k_lincomb(LincombArgs a) {
  const int64_t l = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (l >= a.n) return;
  double v = a.y ? a.a0 * gl(a.y)[l] : 0.0;
  double s = 0.0;
  for (int k = 0; k < a.K; ++k) s += gl(a.coef)[k] * gl(gl(a.v)[k])[l];
  gl(a.out)[l] = a.scale * (v + a.sign * s);
}

void launch_lincomb(const LincombArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((a.n + kVecThreads - 1) / kVecThreads)), dim3(kVecThreads), 0, s, a);
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// overlapping Schwarz smoother with fast-diagonalization local solves
// (Implementation, pMG smoothers, eq. fdm)
// ---------------------------------------------------------------------------
// One workgroup per element; (N+3)^2 threads, each owning one grid line of
// the extended box at a time (a c-column for the gather, the t transforms and
// the stores; a b, c row for the r transforms; an a, c line for the s
// transforms), with the box in LDS between directions.
template <int N>
struct SchCfg {
  static constexpr int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  static constexpr int NE = N + 3, NE2 = NE * NE, NE3 = NE2 * NE;
  static constexpr int THREADS = ((NE2 + 63) / 64) * 64;
};

int schwarz_blocks(int64_t E) { return (int)E; }

// value of v in lane `lane` of the wave (a scalar operand)
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int N, typename T, int MODE>
__global__ __launch_bounds__(SchCfg<N>::THREADS) void k_schwarz(Table<SchwarzArgs<T>> tab) {
  using C = SchCfg<N>;
  constexpr int NP = C::NP, NP2 = C::NP2, NP3 = C::NP3, NE = C::NE, NE2 = C::NE2;
  __shared__ T box[C::NE3];  // [c][b][a]
  __shared__ int sd[6][8];
  int lb;
  const SchwarzArgs<T> a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  const int64_t e = lb;
  const int tid = threadIdx.x;
  if (tid < 48) sd[tid >> 3][tid & 7] = gl(a.desc)[e * 48 + tid];
  __syncthreads();
  const int ia = tid % NE, ib = tid / NE;
  const bool live = ib < NE;
  const bool ca = ia >= 1 && ia <= N + 1, cb = ib >= 1 && ib <= N + 1;
  const SEM_GLOBAL T* in = gl(a.in);
  auto face = [&](int f, int u, int v) -> T {
    const int nb = sd[f][0];
    if (nb < 0) return T(0);
    return in[(int64_t)nb * NP3 + sd[f][1] + u * sd[f][2] + v * sd[f][3]];
  };
  T x[NE];
#pragma unroll
  for (int c = 0; c < NE; ++c) x[c] = T(0);
  if (live) {
    if (ca && cb) {
      const SEM_GLOBAL T* ue = in + e * NP3 + (ib - 1) * NP + (ia - 1);
#pragma unroll
      for (int c = 1; c <= N + 1; ++c) x[c] = ue[(c - 1) * NP2];
      x[0] = face(4, ia - 1, ib - 1);
      x[N + 2] = face(5, ia - 1, ib - 1);
    } else if (!ca && cb) {
      const int f = ia == 0 ? 0 : 1;
#pragma unroll
      for (int c = 1; c <= N + 1; ++c) x[c] = face(f, ib - 1, c - 1);
    } else if (ca && !cb) {
      const int f = ib == 0 ? 2 : 3;
#pragma unroll
      for (int c = 1; c <= N + 1; ++c) x[c] = face(f, ia - 1, c - 1);
    }
  }
  T o[NE];
  if constexpr (MODE == 1) {
    // identity on the active positions of the subdomain (edge columns hold zeros)
    auto lo = [](int k) { return k == 0 ? 0 : k == 1 ? 2 : 1; };
    auto hi = [](int k) { return k == 0 ? N + 2 : k == 1 ? N : N + 1; };
    const bool in_ab = ia >= lo(sd[0][7]) && ia <= hi(sd[1][7]) && ib >= lo(sd[2][7]) && ib <= hi(sd[3][7]);
#pragma unroll
    for (int c = 0; c < NE; ++c) o[c] = (in_ab && c >= lo(sd[4][7]) && c <= hi(sd[5][7])) ? x[c] : T(0);
  } else {
    // Every 1D transform is done by the thread that owns the whole grid line
    // in registers, so each LDS value feeds NE multiply-adds; the 1D
    // matrices and eigenvalues are uniform across the workgroup and are read
    // as scalar operands. Lines change direction through the LDS box.
    // The element's 1D data (3 NE^2 + 3 NE values) are loaded once per wave,
    // spread over the lanes (coalesced); each use broadcasts one lane's value
    // as a scalar operand, so no scalar-cache or LDS traffic per use.
    constexpr int NS = (3 * NE2 + 63) / 64, NL = (3 * NE + 63) / 64;
    const int lane = tid & 63;
    T sv[NS], lv[NL];
    {
      const SEM_GLOBAL T* Sg = gl(a.S) + e * 3 * NE2;  // [dir][ext index][mode]
      const SEM_GLOBAL T* Lg = gl(a.lam) + e * 3 * NE;
#pragma unroll
      for (int k = 0; k < NS; ++k) sv[k] = k * 64 + lane < 3 * NE2 ? Sg[k * 64 + lane] : T(0);
#pragma unroll
      for (int k = 0; k < NL; ++k) lv[k] = k * 64 + lane < 3 * NE ? Lg[k * 64 + lane] : T(0);
    }
    auto Sg = [&](int idx) -> T { return lane_value(sv[idx >> 6], idx & 63); };
    auto Lg = [&](int idx) -> T { return lane_value(lv[idx >> 6], idx & 63); };
    const int l1 = tid % NE, l2 = tid / NE;          // line coordinates (two of a, b, c)
    T y[NE];
    // t forward on the gathered column (a, b) = (ia, ib)
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < NE; ++c) acc += Sg(2 * NE2 + c * NE + m) * x[c];
      y[m] = acc;
    }
    if (live)
#pragma unroll
      for (int c = 0; c < NE; ++c) box[c * NE2 + ib * NE + ia] = y[c];
    __syncthreads();
    // r forward on the row (b, c) = (l1, l2)
    if (live) {
      T* row = box + l2 * NE2 + l1 * NE;
#pragma unroll
      for (int q = 0; q < NE; ++q) x[q] = row[q];
#pragma unroll
      for (int m = 0; m < NE; ++m) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) acc += Sg(q * NE + m) * x[q];
        row[m] = acc;
      }
    }
    __syncthreads();
    // s forward, divide by the eigenvalue sums, s backward on the line (a, c) = (l1, l2).
    // The eigenvalue shuffle runs with every lane active: a lane outside the
    // grid may be the source another lane reads.
    static_assert(NL == 1, "eigenvalues fit in one register per lane");
    const T lac = __shfl(lv[0], l1 < NE ? l1 : 0, 64) + __shfl(lv[0], 2 * NE + (l2 < NE ? l2 : 0), 64);
    if (live) {
      T* ln = box + l2 * NE2 + l1;
#pragma unroll
      for (int q = 0; q < NE; ++q) x[q] = ln[q * NE];
#pragma unroll
      for (int m = 0; m < NE; ++m) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) acc += Sg(NE2 + q * NE + m) * x[q];
        const T lam = lac + Lg(NE + m);
        T inv;
        if constexpr (sizeof(T) == 4) inv = lam > T(0) ? __builtin_amdgcn_rcpf(lam) : T(0);
        else inv = lam > T(0) ? T(1) / lam : T(0);
        y[m] = acc * inv;
      }
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        T acc = 0;
#pragma unroll
        for (int m = 0; m < NE; ++m) acc += Sg(NE2 + q * NE + m) * y[m];
        ln[q * NE] = acc;
      }
    }
    __syncthreads();
    // r backward on the row (b, c) = (l1, l2)
    if (live) {
      T* row = box + l2 * NE2 + l1 * NE;
#pragma unroll
      for (int m = 0; m < NE; ++m) y[m] = row[m];
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        T acc = 0;
#pragma unroll
        for (int m = 0; m < NE; ++m) acc += Sg(q * NE + m) * y[m];
        row[q] = acc;
      }
    }
    __syncthreads();
    // t backward on the column (a, b) = (ia, ib)
    if (live)
#pragma unroll
      for (int m = 0; m < NE; ++m) y[m] = box[m * NE2 + ib * NE + ia];
#pragma unroll
    for (int c = 0; c < NE; ++c) {
      T acc = 0;
#pragma unroll
      for (int m = 0; m < NE; ++m) acc += Sg(2 * NE2 + c * NE + m) * y[m];
      o[c] = acc;
    }
  }
  if (!live) return;
  SEM_GLOBAL T* ovl = a.ovl ? gl(a.ovl) + e * 6 * NP2 : nullptr;
  if (ca && cb) {
    SEM_GLOBAL T* oe = gl(a.out) + e * NP3 + (ib - 1) * NP + (ia - 1);
#pragma unroll
    for (int c = 1; c <= N + 1; ++c) oe[(c - 1) * NP2] = o[c];
    if (ovl) {
      ovl[4 * NP2 + (ib - 1) * NP + (ia - 1)] = o[0];
      ovl[5 * NP2 + (ib - 1) * NP + (ia - 1)] = o[N + 2];
    }
  } else if (ovl && !ca && cb) {
    const int f = ia == 0 ? 0 : 1;
#pragma unroll
    for (int c = 1; c <= N + 1; ++c) ovl[f * NP2 + (c - 1) * NP + (ib - 1)] = o[c];
  } else if (ovl && ca && !cb) {
    const int f = ib == 0 ? 2 : 3;
#pragma unroll
    for (int c = 1; c <= N + 1; ++c) ovl[f * NP2 + (c - 1) * NP + (ia - 1)] = o[c];
  }
}

// Fast-diagonalization solve on the matrix cores: one 64-lane wave per
// element. The solve is six 1D transforms (S^T along a, b, c, the division
// by the eigenvalue sums, then S along a, b, c). Each transform is a small
// GEMM  out[line][m] = sum_q in[line][q] S[q][m]  over the NE^2 grid lines
// of the contracted direction, done as 16x16x4 MFMA tiles (16 lines x 16
// modes x 4 ext indices, zero-padded). Operand layout (both precisions):
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; D[i][j] sits in
// lane j + 16 (i / 4), register i % 4 for f32, and in lane j + 16 (i % 4),
// register i / 4 for f64.
//
// The box lives in one LDS buffer whose layout rotates with every
// transform: a transform reads line-major (address line NE + q, the
// contracted index fastest) and writes mode-major (address line + m NE^2).
// With the lines of a transform numbered (slow, fast) = (first, second)
// remaining index, the mode-major output is exactly the line-major input of
// the next direction: [c][b][a] -> [m_a][c][b] -> [m_b][m_a][c] ->
// [m_c][m_b][m_a] -> [a][m_c][m_b] -> [b][a][m_c] -> [c][b][a]. Every LDS
// address is a per-lane base plus a compile-time offset, and the four rows a
// lane holds in FP32 are consecutive (one 16-byte store). A transform reads
// all of its operands into registers before it writes, so it runs in place;
// a wave-scope fence separates the transforms (every transform reads the
// same per-lane addresses).
// Rows beyond the NE^2 lines and padded ext indices read the zero tail of
// the buffer or the next line's values, which meet zero rows of B.
template <typename T>
struct Mfma4 {
  typedef T v __attribute__((ext_vector_type(4)));
};
__device__ __forceinline__ Mfma4<float>::v mfma16x16x4(float a, float b, Mfma4<float>::v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ Mfma4<double>::v mfma16x16x4(double a, double b, Mfma4<double>::v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int N>
struct SchMfma {
  static constexpr int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  static constexpr int NE = N + 3, NE2 = NE * NE, NE3 = NE2 * NE;
  static constexpr int MT = (NE2 + 15) / 16, KS = (NE + 3) / 4;
  // largest line-major read: row 16 MT - 1, ext index 4 KS - 1
  static constexpr int RMAX = (16 * MT - 1) * NE + 4 * KS;
  static constexpr int BUF = ((RMAX > NE3 ? RMAX : NE3) + 3) / 4 * 4;
};

template <int N, typename T>
// FP32: at least five waves per SIMD (the register budget that allows);
// FP64 keeps the compiler's choice, which holds the MFMA results in
// accumulation registers.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1, 8)))
void k_schwarz_mfma(Table<SchwarzArgs<T>> tab, int total) {
  using C = SchMfma<N>;
  constexpr int NP = C::NP, NP2 = C::NP2, NP3 = C::NP3, NE = C::NE, NE2 = C::NE2, NE3 = C::NE3;
  constexpr int MT = C::MT, KS = C::KS, BUF = C::BUF;
  constexpr int OWN_IT = (NP3 + 63) / 64, FACE_IT = (NP2 + 63) / 64, S_IT = (3 * NE2 + 63) / 64;
  static_assert(NE <= 16, "one MFMA tile spans the modes");
  __shared__ __attribute__((aligned(16))) T box[BUF];
  __shared__ __attribute__((aligned(16))) T sab[16 * MT];  // lambda_b + lambda_a per line of the scaled transform
  __shared__ T sL[3 * NE];
  __shared__ T sS[3 * NE2];
  // lane indices are redefined opaquely in every element iteration, so the
  // per-lane LDS and global addresses are recomputed where they are used
  // instead of being hoisted out of the loop and held in registers
  int lane = threadIdx.x;
  int kq = lane >> 4, jm = lane & 15;

  // An element's inputs, held in registers between their load and their
  // store to LDS: the own block, the six face layers (zero where there is no
  // neighbour), the 1D matrices and the 1D eigenvalues.
  struct Staged {
    T own[OWN_IT];
    T face[6][FACE_IT];
    T s[S_IT];
    T lam;
    int faces;  // bit f set: face f has a neighbour (its staged values are valid)
  };
  // Loads inside the element loop may follow this kernel's own stores, so
  // the compiler cannot use scalar loads for them; uniform values (problem
  // arguments, face descriptors) are therefore loaded one word per lane and
  // broadcast with readlane.
  // The descriptor load is issued first so that waiting for it (loads
  // complete in order) leaves the element's other loads in flight. Absent
  // faces have zero descriptors and load element 0's first value, which the
  // staging step skips (the box there stays zero). The skip flags are read
  // once per problem.
  int last_prob = -1;
  bool last_skip = false;
  auto fetch = [&](int vb, SchwarzArgs<T>& a, int64_t& e, bool& skip, Staged& st) {
    int lb, prob = 0;
    if (tab.many == nullptr) {
      lb = vb;
      a = tab.one;
    } else {
      const SEM_GLOBAL int* stt = gl(tab.starts);
      int lo = 0, hi = tab.n;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (__builtin_amdgcn_readfirstlane(stt[mid]) <= vb) lo = mid; else hi = mid;
      }
      prob = lo;
      lb = vb - __builtin_amdgcn_readfirstlane(stt[lo]);
      constexpr int W = sizeof(SchwarzArgs<T>) / 4;
      static_assert(sizeof(SchwarzArgs<T>) % 4 == 0 && W <= 64, "arguments fit one word per lane");
      const SEM_GLOBAL int* src = (const SEM_GLOBAL int*)gl(tab.many + lo);
      const int w = lane < W ? src[lane] : 0;
      int words[W];
#pragma unroll
      for (int k = 0; k < W; ++k) words[k] = __builtin_amdgcn_readlane(w, k);
      __builtin_memcpy(&a, words, sizeof(a));
    }
    e = lb;
    if (prob != last_prob) {
      last_prob = prob;
      last_skip = skipped(a.skip);
    }
    skip = last_skip;
    if (skip) return;
    const SEM_GLOBAL T* in = gl(a.in);
    const SEM_GLOBAL int* dsc = gl(a.desc) + e * 48;
    const int dw = dsc[lane < 24 ? (lane >> 2) * 8 + (lane & 3) : 0];
    const SEM_GLOBAL T* ue = in + e * NP3;
#pragma unroll
    for (int it = 0; it < OWN_IT; ++it) {
      const int p = lane + 64 * it;
      if (64 * (it + 1) <= NP3) st.own[it] = ue[p];
      else st.own[it] = p < NP3 ? ue[p] : T(0);
    }
    const SEM_GLOBAL T* Sg = gl(a.S) + e * 3 * NE2;
#pragma unroll
    for (int it = 0; it < S_IT; ++it) {
      const int p = lane + 64 * it;
      if (64 * (it + 1) <= 3 * NE2) st.s[it] = Sg[p];
      else st.s[it] = p < 3 * NE2 ? Sg[p] : T(0);
    }
    st.lam = gl(a.lam)[e * 3 * NE + (lane < 3 * NE ? lane : 0)];
    st.faces = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int nb = __builtin_amdgcn_readlane(dw, 4 * f);
      const int off = __builtin_amdgcn_readlane(dw, 4 * f + 1);
      const int su = __builtin_amdgcn_readlane(dw, 4 * f + 2);
      const int sv = __builtin_amdgcn_readlane(dw, 4 * f + 3);
      const SEM_GLOBAL T* src = in + (int64_t)(nb < 0 ? 0 : nb) * NP3 + off;
#pragma unroll
      for (int it = 0; it < FACE_IT; ++it) {
        const int p = lane + 64 * it;
        const int pc = 64 * (it + 1) <= NP2 || p < NP2 ? p : 0;
        st.face[f][it] = src[(pc % NP) * su + (pc / NP) * sv];
      }
      if (nb >= 0) st.faces |= 1 << f;
    }
  };
  // ext-box position of face f's node (u, v): a = 0 / N+2 (f = 0, 1),
  // b = 0 / N+2 (2, 3), c = 0 / N+2 (4, 5); (u, v) run over the other two
  auto face_pos = [](int f, int u, int v) {
    const int base = f == 0 ? NE2 + NE : f == 1 ? NE2 + NE + (N + 2) : f == 2 ? NE2 + 1 : f == 3 ? NE2 + 1 + (N + 2) * NE
                   : f == 4 ? NE + 1 : NE + 1 + (N + 2) * NE2;
    return base + u * (f < 2 ? NE : 1) + v * (f < 4 ? NE2 : NE);
  };
  auto own_pos = [](int p) {
    const int i = p % NP, j = (p / NP) % NP, k = p / NP2;
    return (k + 1) * NE2 + (j + 1) * NE + (i + 1);
  };

  // one transform: line-major in, mode-major out, in place. The fence makes
  // the previous transform's stores (by other lanes) visible: without it the
  // compiler may reuse values a lane loaded from the same addresses before.
  auto transform = [&](int d, bool fwd, bool scale) {
    lds_sync<64>();
    T B[KS];  // lane holds B[k][j], k = 4 ks + kq, j = jm: S[k][j] forward, S[j][k] backward
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int q = 4 * ks + kq;
      const bool ok = q < NE && jm < NE;
      const int ad = d * NE2 + (fwd ? q * NE + jm : jm * NE + q);
      B[ks] = ok ? sS[ok ? ad : 0] : T(0);
    }
    T av[MT][KS];
    const T* rd = box + jm * NE + kq;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[mt][ks] = rd[mt * 16 * NE + 4 * ks];
    typename Mfma4<T>::v acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      acc[mt] = typename Mfma4<T>::v{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) acc[mt] = mfma16x16x4(av[mt][ks], B[ks], acc[mt]);
    }
    // rows held by this lane: 4 kq + r (f32) or 4 r + kq (f64)
    constexpr bool F32 = sizeof(T) == 4;
    const int rb = F32 ? 4 * kq : kq;
    constexpr int rs = F32 ? 1 : 4;
    if (scale) {
      const T lc = sL[2 * NE + (jm < NE ? jm : 0)];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T lam = sab[mt * 16 + rb + r * rs] + lc;
          T v = acc[mt][r];
          if constexpr (F32) v = lam > T(0) ? v * __builtin_amdgcn_rcpf(lam) : T(0);
          else v = lam > T(0) ? v / lam : T(0);
          acc[mt][r] = v;
        }
    }
    if (jm < NE) {
      T* wr = box + jm * NE2 + rb;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        if (mt + 1 < MT || 16 * MT == NE2) {
#pragma unroll
          for (int r = 0; r < 4; ++r) wr[mt * 16 + r * rs] = acc[mt][r];
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (mt * 16 + rb + r * rs < NE2) wr[mt * 16 + r * rs] = acc[mt][r];
        }
      }
    }
  };

  // Small elements keep the next element's inputs in flight during the
  // current element's transforms; large ones (or FP64 at N = 7 and up) would
  // need too many registers for that and load at the top of each iteration.
  constexpr bool PRE = sizeof(T) * (OWN_IT + 6 * FACE_IT + S_IT + 1) <= 4 * 24;
  int vb = blockIdx.x;
  if (vb >= total) return;
  SchwarzArgs<T> a;
  int64_t e = 0;
  bool skip = true;
  Staged st;
  if constexpr (PRE) fetch(vb, a, e, skip, st);
  // the tail beyond the box is read as padding and never written
  for (int k = NE3 + lane; k < BUF; k += 64) box[k] = T(0);
  for (;;) {
    asm volatile("" : "+v"(lane));
    lane &= 63;  // keeps the known range (small-integer address arithmetic)
    kq = lane >> 4;
    jm = lane & 15;
    if constexpr (!PRE) fetch(vb, a, e, skip, st);
    if (!skip) {
      // stage the element into LDS: zero box (edges and absent faces), own
      // block, faces, 1D data; the fence orders these stores after the
      // previous element's final reads
      lds_sync<64>();
      for (int k = lane; k < NE3; k += 64) box[k] = T(0);
      lds_sync<64>();
#pragma unroll
      for (int it = 0; it < OWN_IT; ++it) {
        const int p = lane + 64 * it;
        if (64 * (it + 1) <= NP3 || p < NP3) box[own_pos(p)] = st.own[it];
      }
#pragma unroll
      for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int it = 0; it < FACE_IT; ++it) {
          const int p = lane + 64 * it;
          if ((64 * (it + 1) <= NP2 || p < NP2) && (st.faces >> f & 1)) box[face_pos(f, p % NP, p / NP)] = st.face[f][it];
        }
#pragma unroll
      for (int it = 0; it < S_IT; ++it) {
        const int p = lane + 64 * it;
        if (64 * (it + 1) <= 3 * NE2 || p < 3 * NE2) sS[p] = st.s[it];
      }
      if (lane < 3 * NE) sL[lane] = st.lam;
      lds_sync<64>();
      for (int l = lane; l < 16 * MT; l += 64) sab[l] = l < NE2 ? sL[NE + l / NE] + sL[l % NE] : T(1);
    }
    // issue the next element's loads; they stay in flight during this
    // element's transforms
    const int vn = vb + (int)gridDim.x;
    SchwarzArgs<T> an;
    int64_t en = 0;
    bool skn = true;
    Staged sn;
    if constexpr (PRE)
      if (vn < total) fetch(vn, an, en, skn, sn);
    if (!skip) {
      transform(0, true, false);   // [c][b][a]     -> [m_a][c][b]
      transform(1, true, false);   // [m_a][c][b]   -> [m_b][m_a][c]
      transform(2, true, true);    // [m_b][m_a][c] -> [m_c][m_b][m_a], divided by the eigenvalue sums
      transform(0, false, false);  // -> [a][m_c][m_b]
      transform(1, false, false);  // -> [b][a][m_c]
      transform(2, false, false);  // -> [c][b][a]
      lds_sync<64>();
      // own block and, for the additive variant, the face layers of the local solution
      SEM_GLOBAL T* oe = gl(a.out) + e * NP3;
#pragma unroll
      for (int it = 0; it < OWN_IT; ++it) {
        const int p = lane + 64 * it;
        if (64 * (it + 1) <= NP3 || p < NP3) oe[p] = box[own_pos(p)];
      }
      if (a.ovl) {
        SEM_GLOBAL T* ovl = gl(a.ovl) + e * 6 * NP2;
#pragma unroll
        for (int f = 0; f < 6; ++f)
#pragma unroll
          for (int it = 0; it < FACE_IT; ++it) {
            const int p = lane + 64 * it;
            if (64 * (it + 1) <= NP2 || p < NP2) ovl[f * NP2 + p] = box[face_pos(f, p % NP, p / NP)];
          }
      }
    }
    if (vn >= total) break;
    vb = vn;
    if constexpr (PRE) {
      a = an;
      e = en;
      skip = skn;
      st = sn;
    }
  }
}

// One 64-lane wave per element and pass: pass d adds the overlaps across the
// two faces normal to direction d. A node at depth 1 behind faces of two
// directions is updated in two passes, so the passes are ordered by barriers.
constexpr int kPullThreads = 64;

template <int N, typename T>
__global__ __launch_bounds__(kPullThreads) void k_schwarz_pull(Table<SchwarzPullArgs<T>> tab) {
  constexpr int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  __shared__ int sd[6][8];
  int lb;
  const SchwarzPullArgs<T> a = fetch_args(tab, blockIdx.x, lb);
  if (skipped(a.skip)) return;
  const int64_t e = lb;
  if (threadIdx.x < 48) sd[threadIdx.x >> 3][threadIdx.x & 7] = gl(a.desc)[e * 48 + threadIdx.x];
  __syncthreads();
  const SEM_GLOBAL T* ovl = gl(a.ovl);
  SEM_GLOBAL T* out = gl(a.out) + e * NP3;
  auto pull = [&](int f, int u, int v) -> T {
    const int nb = sd[f][0];
    if (nb < 0) return T(0);
    return ovl[(int64_t)nb * 6 * NP2 + sd[f][4] + u * sd[f][5] + v * sd[f][6]];
  };
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    const int f0 = 2 * axis, f1 = f0 + 1;
    const bool any = sd[f0][0] >= 0 || sd[f1][0] >= 0;  // uniform
    if (any) {
      for (int t = threadIdx.x; t < NP2; t += kPullThreads) {
        const int u = t % NP, v = t / NP;
        // local index of (u, v) at depth 1 behind face f0 (low side) and f1 (high side)
        int p0, p1;
        if (axis == 0) { p0 = 1 + NP * u + NP2 * v; p1 = (N - 1) + NP * u + NP2 * v; }
        else if (axis == 1) { p0 = u + NP + NP2 * v; p1 = u + NP * (N - 1) + NP2 * v; }
        else { p0 = u + NP * v + NP2; p1 = u + NP * v + NP2 * (N - 1); }
        const T a0 = pull(f0, u, v), a1 = pull(f1, u, v);
        if (p0 == p1) {
          out[p0] += a0 + a1;
        } else {
          out[p0] += a0;
          out[p1] += a1;
        }
      }
    }
    __syncthreads();
  }
}

// The matrix-core kernel is persistent: as many one-wave workgroups as fit on
// the device at once, each walking the elements with a stride of the grid.
template <int N, typename T>
void launch_schwarz_mfma(const Table<SchwarzArgs<T>>& t, int64_t total, hipStream_t s) {
  static const int64_t cap = [] {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_schwarz_mfma<N, T>, 64, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
      return (int64_t)1 << 30;
    return (int64_t)cus * per_cu;
  }();
  if (total > INT32_MAX) fail(SEM_EINVAL, "Schwarz smoother: %lld elements exceed the launch limit", (long long)total);
  const int64_t g = total < cap ? total : cap;
  hipLaunchKernelGGL((k_schwarz_mfma<N, T>), dim3((unsigned)g), dim3(64), 0, s, t, (int)total);
}

template <typename T>
void launch_schwarz(int N, int mode, const Table<SchwarzArgs<T>>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  const dim3 g((unsigned)total_blocks);
  switch (N) {
#define SEM_SCH_CASE(n) case n: if (mode == 0 && n + 3 <= 16) launch_schwarz_mfma<(n + 3 <= 16 ? n : 2), T>(t, total_blocks, s); else if (mode == 0) hipLaunchKernelGGL((k_schwarz<n, T, 0>), g, dim3(SchCfg<n>::THREADS), 0, s, t); else hipLaunchKernelGGL((k_schwarz<n, T, 1>), g, dim3(SchCfg<n>::THREADS), 0, s, t); break;
    SEM_SCH_CASE(2) SEM_SCH_CASE(3) SEM_SCH_CASE(4) SEM_SCH_CASE(5) SEM_SCH_CASE(6) SEM_SCH_CASE(7)
    SEM_SCH_CASE(8) SEM_SCH_CASE(9) SEM_SCH_CASE(10) SEM_SCH_CASE(11) SEM_SCH_CASE(12) SEM_SCH_CASE(13)
    SEM_SCH_CASE(14) SEM_SCH_CASE(15)
#undef SEM_SCH_CASE
    default:
      fail(SEM_EINVAL, "Schwarz smoother: unsupported order N=%d", N);
  }
  SEM_HIP(hipGetLastError());
}
template void launch_schwarz<double>(int, int, const Table<SchwarzArgs<double>>&, int64_t, hipStream_t);
template void launch_schwarz<float>(int, int, const Table<SchwarzArgs<float>>&, int64_t, hipStream_t);

template <typename T>
void launch_schwarz_pull(int N, const Table<SchwarzPullArgs<T>>& t, int64_t total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  const dim3 g((unsigned)total_blocks), b(kPullThreads);
  switch (N) {
#define SEM_PULL_CASE(n) case n: hipLaunchKernelGGL((k_schwarz_pull<n, T>), g, b, 0, s, t); break;
    SEM_PULL_CASE(2) SEM_PULL_CASE(3) SEM_PULL_CASE(4) SEM_PULL_CASE(5) SEM_PULL_CASE(6) SEM_PULL_CASE(7)
    SEM_PULL_CASE(8) SEM_PULL_CASE(9) SEM_PULL_CASE(10) SEM_PULL_CASE(11) SEM_PULL_CASE(12) SEM_PULL_CASE(13)
    SEM_PULL_CASE(14) SEM_PULL_CASE(15)
#undef SEM_PULL_CASE
    default:
      fail(SEM_EINVAL, "Schwarz smoother: unsupported order N=%d", N);
  }
  SEM_HIP(hipGetLastError());
}
template void launch_schwarz_pull<double>(int, const Table<SchwarzPullArgs<double>>&, int64_t, hipStream_t);
template void launch_schwarz_pull<float>(int, const Table<SchwarzPullArgs<float>>&, int64_t, hipStream_t);

// per element: corner IDs, all-Dirichlet face flags, mean lengths (one thread per element)
__global__ __launch_bounds__(64) void k_schwarz_info(SchwarzInfoArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (e >= a.E) return;
  const int N = a.N, NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  const int64_t b = e * NP3;
  const SEM_GLOBAL int64_t* gid = gl(a.gid);
  const SEM_GLOBAL uint8_t* dm = gl(a.dmask);
  const SEM_GLOBAL double* X = gl(a.x);
  const SEM_GLOBAL double* Y = gl(a.y);
  const SEM_GLOBAL double* Z = gl(a.z);
  for (int q = 0; q < 8; ++q) {
    const int i = (q & 1) ? N : 0, j = (q & 2) ? N : 0, k = (q & 4) ? N : 0;
    gl(a.corners)[e * 8 + q] = gid[b + i + NP * j + NP2 * k];
  }
  for (int f = 0; f < 6; ++f) {
    const int axis = f >> 1, d = (f & 1) ? N : 0;
    int all = 1;
    for (int u = 0; u < NP; ++u)
      for (int v = 0; v < NP; ++v) {
        const int p = axis == 0 ? d + NP * u + NP2 * v : axis == 1 ? u + NP * d + NP2 * v : u + NP * v + NP2 * d;
        all &= dm[b + p] != 0;
      }
    gl(a.face_dir)[e * 6 + f] = (uint8_t)all;
  }
  for (int axis = 0; axis < 3; ++axis) {
    double sum = 0.0;
    for (int u = 0; u < NP; ++u)
      for (int v = 0; v < NP; ++v) {
        int p0, p1;
        if (axis == 0) { p0 = NP * u + NP2 * v; p1 = p0 + N; }
        else if (axis == 1) { p0 = u + NP2 * v; p1 = p0 + N * NP; }
        else { p0 = u + NP * v; p1 = p0 + N * NP2; }
        const double dx = X[b + p1] - X[b + p0], dy = Y[b + p1] - Y[b + p0], dz = Z[b + p1] - Z[b + p0];
        sum += sqrt(dx * dx + dy * dy + dz * dz);
      }
    gl(a.lengths)[e * 3 + axis] = sum / NP2;
  }
}

void launch_schwarz_info(const SchwarzInfoArgs& a, hipStream_t s) {
  if (a.E <= 0) return;
  hipLaunchKernelGGL(k_schwarz_info, dim3((unsigned)((a.E + 63) / 64)), dim3(64), 0, s, a);
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

// Geometric factors at every GLL point (one thread per point).
// Jm[l][m] = d x_l / d r_m by Dhat along i, j, k; cof_m = det * grad r_m;
// G_mn = W cof_m . cof_n / det; B = W det.
constexpr int kGeoThreads = 256;

__global__ __launch_bounds__(kGeoThreads) void k_geometry(int N, int64_t nloc, const double* __restrict__ X,
                                                          const double* __restrict__ Y, const double* __restrict__ Z,
                                                          const double* __restrict__ Dg, const double* __restrict__ wg,
                                                          double* G64, float* G32, double* B64, float* B32,
                                                          double* detmin_partial, double* vol_partial,
                                                          unsigned long long* bad) {
  __shared__ double s_min[kGeoThreads / 64], s_vol[kGeoThreads / 64];
  const int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  const int64_t l = (int64_t)blockIdx.x * kGeoThreads + threadIdx.x;
  double detv = INFINITY, volv = 0.0;
  if (l < nloc) {
    const int64_t e = l / NP3;
    const int p = (int)(l - e * NP3);
    const int i = p % NP, j = (p / NP) % NP, k = p / NP2;
    const double* xs[3] = {X + e * NP3, Y + e * NP3, Z + e * NP3};
    double Jm[3][3];
    for (int c = 0; c < 3; ++c) {
      double dr = 0, ds = 0, dt = 0;
      for (int q = 0; q < NP; ++q) {
        dr += Dg[i * NP + q] * xs[c][k * NP2 + j * NP + q];
        ds += Dg[j * NP + q] * xs[c][k * NP2 + q * NP + i];
        dt += Dg[k * NP + q] * xs[c][q * NP2 + j * NP + i];
      }
      Jm[c][0] = dr;
      Jm[c][1] = ds;
      Jm[c][2] = dt;
    }
    const double xr = Jm[0][0], xs_ = Jm[0][1], xt = Jm[0][2];
    const double yr = Jm[1][0], ys = Jm[1][1], yt = Jm[1][2];
    const double zr = Jm[2][0], zs = Jm[2][1], zt = Jm[2][2];
    // cofactor rows: cof_m[l] = det * d r_m / d x_l
    const double a0[3] = {ys * zt - yt * zs, xt * zs - xs_ * zt, xs_ * yt - xt * ys};
    const double a1[3] = {yt * zr - yr * zt, xr * zt - xt * zr, xt * yr - xr * yt};
    const double a2[3] = {yr * zs - ys * zr, xs_ * zr - xr * zs, xr * ys - xs_ * yr};
    const double det = xr * a0[0] + yr * a0[1] + zr * a0[2];
    const double W = wg[i] * wg[j] * wg[k];
    if (!(det > 0.0)) atomicMin(bad, (unsigned long long)l);
    const double f = W / det;
    const double g[6] = {f * (a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2]),
                         f * (a0[0] * a1[0] + a0[1] * a1[1] + a0[2] * a1[2]),
                         f * (a0[0] * a2[0] + a0[1] * a2[1] + a0[2] * a2[2]),
                         f * (a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]),
                         f * (a1[0] * a2[0] + a1[1] * a2[1] + a1[2] * a2[2]),
                         f * (a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2])};
    for (int c = 0; c < 6; ++c) {
      G64[(e * 6 + c) * NP3 + p] = g[c];
      G32[(e * 6 + c) * NP3 + p] = (float)g[c];
    }
    B64[l] = W * det;
    B32[l] = (float)(W * det);
    detv = det;
    volv = W * det;
  }
  // fixed-order block reductions (min and sum)
  double m = detv, v = volv;
  for (int off = 32; off > 0; off >>= 1) {
    m = fmin(m, __shfl_xor(m, off, 64));
    v += __shfl_xor(v, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { s_min[wid] = m; s_vol[wid] = v; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = s_min[0], vv = s_vol[0];
    for (int k2 = 1; k2 < kGeoThreads / 64; ++k2) { mm = fmin(mm, s_min[k2]); vv += s_vol[k2]; }
    detmin_partial[blockIdx.x] = mm;
    vol_partial[blockIdx.x] = vv;
  }
}

void launch_geometry(const MeshData& m, double* detmin_partial, double* vol_partial, int64_t* bad_index,
                     hipStream_t s) {
  const int64_t nb = (m.nloc + kGeoThreads - 1) / kGeoThreads;
  hipLaunchKernelGGL(k_geometry, dim3((unsigned)nb), dim3(kGeoThreads), 0, s, m.N, m.nloc,
                     m.x.as<double>(), m.y.as<double>(), m.z.as<double>(), m.Dg64.as<double>(),
                     m.wg.as<double>(), m.G64.as<double>(), m.G32.as<float>(), m.B64.as<double>(),
                     m.B32.as<float>(), detmin_partial, vol_partial, (unsigned long long*)bad_index);
  SEM_HIP(hipGetLastError());
}

// Local diagonal of A^e = sum_mn D_m^T diag(G_mn) D_n at (i,j,k).
__global__ __launch_bounds__(256) void k_diag(int N, int64_t nloc, const double* __restrict__ G,
                                              const double* __restrict__ Dg, double* dl) {
  const int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= nloc) return;
  const int64_t e = l / NP3;
  const int p = (int)(l - e * NP3);
  const int i = p % NP, j = (p / NP) % NP, k = p / NP2;
  const double* g = G + e * 6 * NP3;
  double d = 0.0;
  for (int q = 0; q < NP; ++q) {
    const double a = Dg[q * NP + i], b = Dg[q * NP + j], c = Dg[q * NP + k];
    d += a * a * g[0 * NP3 + k * NP2 + j * NP + q];
    d += b * b * g[3 * NP3 + k * NP2 + q * NP + i];
    d += c * c * g[5 * NP3 + q * NP2 + j * NP + i];
  }
  const double di = Dg[i * NP + i], dj = Dg[j * NP + j], dk = Dg[k * NP + k];
  d += 2.0 * di * dj * g[1 * NP3 + p] + 2.0 * di * dk * g[2 * NP3 + p] + 2.0 * dj * dk * g[4 * NP3 + p];
  dl[l] = d;
}

void launch_diag_local(const MeshData& m, double* dl, hipStream_t s) {
  const int64_t nb = (m.nloc + 255) / 256;
  hipLaunchKernelGGL(k_diag, dim3((unsigned)nb), dim3(256), 0, s, m.N, m.nloc, m.G64.as<double>(),
                     m.Dg64.as<double>(), dl);
  SEM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_dinv(int64_t nloc, const double* __restrict__ d,
                                              const uint8_t* __restrict__ dmask, double* inv64, float* inv32) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= nloc) return;
  const double v = dmask[l] ? 0.0 : 1.0 / d[l];
  inv64[l] = v;
  inv32[l] = (float)v;
}

__global__ __launch_bounds__(256) void k_dinv_to(int64_t nloc, const double* __restrict__ d,
                                                 const uint8_t* __restrict__ dmask, double* out) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l < nloc) out[l] = dmask[l] ? 0.0 : 1.0 / d[l];
}

void launch_dinv_to(const MeshData& m, const double* d_assembled, double* out, hipStream_t s) {
  const int64_t nb = (m.nloc + 255) / 256;
  hipLaunchKernelGGL(k_dinv_to, dim3((unsigned)nb), dim3(256), 0, s, m.nloc, d_assembled, m.dmask.as<uint8_t>(), out);
  SEM_HIP(hipGetLastError());
}

void launch_dinv_finish(const MeshData& m, const double* d_assembled, hipStream_t s) {
  const int64_t nb = (m.nloc + 255) / 256;
  hipLaunchKernelGGL(k_dinv, dim3((unsigned)nb), dim3(256), 0, s, m.nloc, d_assembled, m.dmask.as<uint8_t>(),
                     m.dinv64.as<double>(), m.dinv32.as<float>());
  SEM_HIP(hipGetLastError());
}

// out[e] = (M x M x M) in[e], M is (Nc+1) x (Nf+1): coarse nodal coordinates
// as the fine isoparametric map evaluated at the coarse GLL points.
__global__ __launch_bounds__(256) void k_tensor_coords(int NI, int NO, int64_t E, const double* __restrict__ in,
                                                       double* out, const double* __restrict__ M) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int NO3 = NO * NO * NO, NI3 = NI * NI * NI;
  if (t >= E * NO3) return;
  const int64_t e = t / NO3;
  const int r = (int)(t - e * NO3);
  const int a = r % NO, b = (r / NO) % NO, c = r / (NO * NO);
  const double* u = in + e * NI3;
  double acc = 0.0;
  for (int k = 0; k < NI; ++k)
    for (int j = 0; j < NI; ++j) {
      double row = 0.0;
      for (int i = 0; i < NI; ++i) row += M[a * NI + i] * u[(k * NI + j) * NI + i];
      acc += M[c * NI + k] * M[b * NI + j] * row;
    }
  out[t] = acc;
}

void launch_tensor_coords(int Nf, int Nc, int64_t E, const double* in, double* out, const double* Mcf,
                          hipStream_t s) {
  const int NO3 = (Nc + 1) * (Nc + 1) * (Nc + 1);
  const int64_t nb = (E * NO3 + 255) / 256;
  hipLaunchKernelGGL(k_tensor_coords, dim3((unsigned)nb), dim3(256), 0, s, Nf + 1, Nc + 1, E, in, out, Mcf);
  SEM_HIP(hipGetLastError());
}

// splitmix64 (Steele, Lea & Flood 2014) keyed by global ID -> [-1, 1), 0 on Dirichlet copies
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_start(int64_t n, const int64_t* __restrict__ gid,
                                               const uint8_t* __restrict__ dmask, double* v) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= n) return;
  const double u = (double)(splitmix64((uint64_t)gid[l]) >> 11) * 0x1.0p-53;
  v[l] = dmask[l] ? 0.0 : 2.0 * u - 1.0;
}

void launch_start_vector(int64_t n, const int64_t* gid, const uint8_t* dmask, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_start, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, gid, dmask, v);
  SEM_HIP(hipGetLastError());
}

template <typename T>
__global__ __launch_bounds__(256) void k_mass(int64_t n, const T* __restrict__ B, const T* __restrict__ u, T* Bu) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l < n) Bu[l] = B[l] * u[l];
}

void launch_mass(int N, int64_t nloc, int is_f32, const void* B, const void* u, void* Bu, hipStream_t s) {
  (void)N;
  const dim3 g((unsigned)((nloc + 255) / 256)), b(256);
  if (is_f32)
    hipLaunchKernelGGL(k_mass<float>, g, b, 0, s, nloc, (const float*)B, (const float*)u, (float*)Bu);
  else
    hipLaunchKernelGGL(k_mass<double>, g, b, 0, s, nloc, (const double*)B, (const double*)u, (double*)Bu);
  SEM_HIP(hipGetLastError());
}

}  // namespace sem
