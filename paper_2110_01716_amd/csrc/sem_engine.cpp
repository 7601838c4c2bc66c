// Solver engine: Jacobi-PCG and pMG-preconditioned flexible CG for one or
// many independent problems.
//
// Paper: the pressure solve runs flexible CG (a short recurrence tolerant of
// the nonsymmetric pMG preconditioner, Implementation, FlexCG/GMRES paragraph)
// around a p-multigrid V-cycle whose smoothers are Chebyshev-accelerated point
// Jacobi, all pMG steps in 32-bit (Implementation, pMG paragraph); the coarse
// level is solved approximately (the paper uses AMG on the CPU; here FP64
// Jacobi-PCG to a loose tolerance on the GPU). Velocity-type solves use
// Jacobi-PCG (Implementation, Helmholtz paragraph).
//
// Execution model:
//   * every solve occupies a Slot: its workspace vectors, partial-sum buffer and
//     a block of device scalars/flags (alpha, beta, norms, done, status, iters);
//   * an iteration is a fixed sequence of phases (Ax, gs, fused vector updates,
//     finalize reductions, transfers); each phase is ONE launch covering every
//     active slot of a group (per-problem argument tables, block offsets);
//   * all scalar recurrences stay on the device; the host only polls done
//     flags (every check_every outer iterations, every coarse_check_every
//     coarse iterations); finished problems skip via their flags, so a
//     problem's arithmetic never depends on the other problems in the batch;
//   * reductions are per block in a fixed order, then per problem in a fixed
//     order: a solve gives bitwise the same result alone or in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "sem_internal.h"

namespace sem {

using Fn = std::function<void(hipStream_t)>;
using Clock = std::chrono::steady_clock;

// ---------------------------------------------------------------------------
// workspace pool: reuse freed solve workspaces (no allocation on the hot path).
// Blocks are kept per device: a block is handed out again only on the device
// it was allocated on (the device current at pool_get).
// ---------------------------------------------------------------------------
static std::mutex g_pool_mu;
static std::multimap<std::pair<int, size_t>, void*> g_pool;  // (device, bytes) -> free block
static std::map<void*, int> g_pool_dev;                      // device of every block the pool allocated

void* pool_get(size_t bytes) {
  int dev = 0;
  SEM_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool.lower_bound({dev, bytes});
    if (it != g_pool.end() && it->first.first == dev && it->first.second <= bytes + bytes / 8) {
      void* p = it->second;
      g_pool.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    // give this device's free blocks back and try once more
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto it = g_pool.lower_bound({dev, 0}); it != g_pool.end() && it->first.first == dev;) {
      (void)hipFree(it->second);
      g_pool_dev.erase(it->second);
      it = g_pool.erase(it);
    }
    e = hipMalloc(&p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? SEM_ENOMEM : SEM_EHIP, "workspace allocation of %zu bytes failed: %s", bytes,
         hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pool_dev[p] = dev;
  return p;
}

void pool_put(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto d = g_pool_dev.find(p);
  if (d == g_pool_dev.end()) return;  // not a pool block
  g_pool.emplace(std::make_pair(d->second, bytes), p);
}

// ---------------------------------------------------------------------------
// slots
// ---------------------------------------------------------------------------
struct Slot {
  sem_mesh_s* mesh = nullptr;
  sem_pmg_s* pmg = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  sem_solve_opts o{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *w = nullptr;
  void *lr[kMaxLevels] = {}, *lx[kMaxLevels] = {}, *lres[kMaxLevels] = {}, *ld[kMaxLevels] = {},
       *lt[kMaxLevels] = {};
  void *ls[kMaxLevels] = {}, *lovl[kMaxLevels] = {};  // Schwarz smoother: output and face overlaps
  double *cr = nullptr, *cx = nullptr, *cp = nullptr, *cw = nullptr;
  double* cz = nullptr;   // D^-1 r of the assembled coarse CG
  double* clocal = nullptr;  // restriction output on coarse element storage (assembled coarse level)
  double* dinv_h = nullptr;  // Jacobi-PCG: inverse diagonal of A + lambda B (Helmholtz solves)
  double* partial = nullptr;
  int64_t stride = 0;
  int idx = -1;
  int state = 0;  // 0 free, 1 admitted, 2 running, 3 finished
  int64_t launches0 = 0;  // the batch's launch count when this solve was admitted
  bool ctrl_clean = false;  // its scalars and flags are still zero from the batch's initialisation
  Clock::time_point t0;
  sem_solve_info info{};
  double* scal[2] = {nullptr, nullptr};  // device: outer, coarse
  int* flags[2] = {nullptr, nullptr};

  const MeshData& level(int l) const { return pmg ? pmg->lv[l].mesh->d : mesh->d; }
  double lam() const { return pmg ? 0.0 : o.lambda; }
  const double* dinv0() const { return lam() != 0.0 ? dinv_h : level(0).dinv64.as<double>(); }
  int nlev() const { return pmg ? pmg->n_levels : 1; }
  bool f32() const { return pmg && pmg->o.smoother_dtype == SEM_F32; }
};

namespace {

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

// layout of a slot workspace; with base == nullptr only computes the size
size_t layout(Slot& s, uint8_t* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const MeshData& f = s.level(0);
  const int64_t n0 = f.nloc;
  int64_t stride = std::max<int64_t>(ax_blocks(f.N, f.E), vec_blocks(n0));
  s.r = (double*)take(8 * n0);
  s.z = (double*)take(8 * n0);
  s.p = (double*)take(8 * n0);
  s.w = (double*)take(8 * n0);
  if (!s.pmg) s.dinv_h = (double*)take(8 * n0);
  if (s.pmg) {
    const int L = s.pmg->n_levels;
    const size_t ts = s.f32() ? 4 : 8;
    for (int l = 0; l + 1 < L; ++l) {
      const int64_t nl = s.level(l).nloc;
      s.lr[l] = take(ts * nl);
      s.lx[l] = take(ts * nl);
      s.lres[l] = take(ts * nl);
      s.ld[l] = take(ts * nl);
      s.lt[l] = take(ts * nl);
      if (s.pmg->lv[l].sw.on) {
        const MeshData& m = s.level(l);
        s.ls[l] = take(ts * nl);
        s.lovl[l] = take(ts * 6 * (m.N + 1) * (m.N + 1) * m.E);
      }
    }
    const MeshData& c = s.level(L - 1);
    const int64_t nc = c.assembled ? c.n_unique : c.nloc;
    s.cr = (double*)take(8 * nc);
    s.cx = (double*)take(8 * nc);
    s.cp = (double*)take(8 * nc);
    s.cw = (double*)take(8 * nc);
    if (c.assembled) {
      s.cz = (double*)take(8 * nc);
      s.clocal = (double*)take(8 * c.nloc);
      stride = std::max<int64_t>(stride, std::max<int64_t>(std::max<int64_t>(spmv_blocks(nc), cg_update_blocks(nc)),
                                                          vec_blocks(nc)));
    } else {
      stride = std::max<int64_t>(stride, std::max<int64_t>(ax_blocks(c.N, c.E), vec_blocks(c.nloc)));
    }
  }
  s.stride = stride;
  s.partial = (double*)take(8 * 3 * stride);  // [0], [1]: vector-kernel sums; [2]: Ax/SpMV sums read redundantly
  return off;
}

template <typename T>
const T* G_of(const MeshData& m) {
  if constexpr (sizeof(T) == 8) return m.G64.as<double>(); else return m.G32.as<float>();
}
template <typename T>
const T* D_of(const MeshData& m) {
  if constexpr (sizeof(T) == 8) return m.Dg64.as<double>(); else return m.Dg32.as<float>();
}
template <typename T>
const T* dinv_of(const MeshData& m) {
  if constexpr (sizeof(T) == 8) return m.dinv64.as<double>(); else return m.dinv32.as<float>();
}

}  // namespace

// ---------------------------------------------------------------------------
// plans: launch sequences over a set of slots
// ---------------------------------------------------------------------------
struct Group {
  std::vector<Slot*> S;
  bool pmg = false;
  bool vcycle_only = false;
  int L = 1;
  std::vector<Fn> init, head, cinit, citer, tail;
  int coarse_limit = 0, coarse_fixed = 0, coarse_check = 8;
};

class Plan {
 public:
  std::vector<uint8_t> host;
  DevBuf dev;
  std::vector<Group> groups;

  size_t push(const void* p, size_t n) {
    const size_t off = align_up(host.size());
    host.resize(off + n);
    std::memcpy(host.data() + off, p, n);
    return off;
  }
  const uint8_t* base() const { return dev.as<uint8_t>(); }

  void upload(hipStream_t s) {
    if (host.empty()) return;
    dev.alloc(host.size());
    SEM_HIP(hipMemcpyAsync(dev.p, host.data(), host.size(), hipMemcpyHostToDevice, s));
  }

  template <typename A, typename L>
  void add(std::vector<Fn>& seq, const std::vector<A>& args, const std::vector<int>& starts, L launch) {
    const int n = (int)args.size();
    if (n == 0) return;
    if (n == 1) {
      A one = args[0];
      seq.push_back([one, launch](hipStream_t s) {
        Table<A> t;
        t.one = one;
        launch(t, s);
      });
      return;
    }
    const size_t oa = push(args.data(), sizeof(A) * n);
    const size_t os = push(starts.data(), sizeof(int) * (n + 1));
    seq.push_back([this, oa, os, n, launch](hipStream_t s) {
      Table<A> t;
      t.many = reinterpret_cast<const A*>(base() + oa);
      t.starts = reinterpret_cast<const int*>(base() + os);
      t.n = n;
      launch(t, s);
    });
  }

  // A(u -> t) at level l: local Ax (optionally with the fused u.Au partial) then gs + mask
  template <typename T, typename FU, typename FT>
  void apply_A(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, FU u_of, FT t_of, bool with_partial,
               int skip_mode) {
    std::map<int, std::vector<Slot*>> by;
    for (Slot* s : S) by[s->level(l).N].push_back(s);
    for (auto& kv : by) {
      const int N = kv.first;
      std::vector<AxArgs<T>> args;
      std::vector<int> starts{0};
      for (Slot* s : kv.second) {
        const MeshData& m = s->level(l);
        AxArgs<T> a;
        a.G = G_of<T>(m);
        if constexpr (sizeof(T) == 8) {
          if (l == 0 && s->lam() != 0.0) {
            a.B = m.B64.as<double>();
            a.lambda = s->lam();
          }
        }
        a.u = u_of(*s);
        a.Au = t_of(*s);
        a.e0 = 0;
        a.ne = m.E;
        a.partial = with_partial ? s->partial : nullptr;
        a.skip = skip(*s, skip_mode);
        args.push_back(a);
        starts.push_back(starts.back() + ax_blocks(N, m.E, sizeof(T) == 4));
      }
      const T* D = D_of<T>(kv.second[0]->level(l));
      const int64_t total = starts.back();
      const bool helm = args[0].B != nullptr;  // groups never mix Poisson and Helmholtz
      add(seq, args, starts, [N, D, total, helm](const Table<AxArgs<T>>& t, hipStream_t st) {
        launch_ax<T>(N, t, total, D, st, helm);
      });
    }
    gs<T>(seq, S, l, t_of, skip_mode);
  }

  template <typename T, typename FV>
  void gs(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, FV v_of, int skip_mode) {
    std::vector<GsArgs<T>> args;
    std::vector<int> starts{0};
    for (Slot* s : S) {
      const MeshData& m = s->level(l);
      GsArgs<T> a;
      a.v = v_of(*s);
      a.off = m.gs_off.as<int>();
      a.idx = m.gs_idx.as<int>();
      a.sdir = m.gs_dir.as<uint8_t>();
      a.dir_idx = m.dir_idx.as<int>();
      a.n_shared = m.n_shared;
      a.n_dir = m.n_dir_single;
      a.mask = 1;
      a.skip = skip(*s, skip_mode);
      args.push_back(a);
      starts.push_back(starts.back() + (int)gs_blocks(m.n_shared, m.n_dir_single));
    }
    const int64_t total = starts.back();
    add(seq, args, starts, [total](const Table<GsArgs<T>>& t, hipStream_t st) { launch_gs<T>(t, total, st); });
  }

  // uniq: the vectors live on the unique DOFs of an assembled level
  template <typename T, typename F>
  void vec(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, VecOp op, F fill, int skip_mode,
           bool uniq = false) {
    std::vector<VecArgs<T>> args;
    std::vector<int> starts{0};
    for (Slot* s : S) {
      const MeshData& m = s->level(l);
      VecArgs<T> a;
      a.n = uniq ? m.n_unique : m.nloc;
      a.owner = uniq ? nullptr : m.owner.as<uint8_t>();
      a.partial = s->partial;
      a.stride = s->stride;
      a.skip = skip(*s, skip_mode);
      fill(*s, a);
      args.push_back(a);
      starts.push_back(starts.back() + (int)vec_blocks(a.n));
    }
    const int64_t total = starts.back();
    add(seq, args, starts, [op, total](const Table<VecArgs<T>>& t, hipStream_t st) { launch_vec<T>(op, t, total, st); });
  }

  // out (unique DOFs) = masked sum of the element-storage copies in `in`
  template <typename FI, typename FO>
  void usum(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, FI in_of, FO out_of, int skip_mode) {
    std::vector<UsumArgs> args;
    std::vector<int> starts{0};
    for (Slot* s : S) {
      const MeshData& m = s->level(l);
      UsumArgs a;
      a.n = m.n_unique;
      a.off = m.u2l_off.as<int>();
      a.idx = m.u2l_idx.as<int>();
      a.udir = m.udir.as<uint8_t>();
      a.in = in_of(*s);
      a.out = out_of(*s);
      a.skip = skip(*s, skip_mode);
      args.push_back(a);
      starts.push_back(starts.back() + (int)spmv_blocks(a.n));
    }
    const int64_t total = starts.back();
    add(seq, args, starts, [total](const Table<UsumArgs>& t, hipStream_t st) { launch_usum(t, total, st); });
  }

  template <typename Tin, typename Tout, typename F>
  void cast(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, F fill, int skip_mode) {
    std::vector<CastArgs<Tin, Tout>> args;
    std::vector<int> starts{0};
    for (Slot* s : S) {
      CastArgs<Tin, Tout> a;
      a.n = s->level(l).nloc;
      a.skip = skip(*s, skip_mode);
      fill(*s, a);
      args.push_back(a);
      starts.push_back(starts.back() + (int)vec_blocks(a.n));
    }
    const int64_t total = starts.back();
    add(seq, args, starts, [total](const Table<CastArgs<Tin, Tout>>& t, hipStream_t st) {
      launch_cast<Tin, Tout>(t, total, st);
    });
  }

  // stage 0 = outer, 1 = coarse; nblk from the producing kernel's blocks
  template <typename F>
  void fin(std::vector<Fn>& seq, const std::vector<Slot*>& S, FinOp op, int stage, F nblk_of, int skip_mode,
           double rtol = 0, int maxit = 0, int fixed = 0, bool count_total = false) {
    std::vector<FinArgs> args;
    std::vector<int> starts{0};
    for (Slot* s : S) {
      FinArgs a;
      a.partial = s->partial;
      a.stride = s->stride;
      a.nblk = nblk_of(*s);
      a.scal = s->scal[stage];
      a.flags = s->flags[stage];
      a.rtol = rtol;
      a.maxit = maxit;
      a.fixed = fixed;
      a.total = count_total ? s->flags[0] + F_TOTAL : nullptr;
      a.skip = skip(*s, skip_mode);
      if (stage == 0) {
        a.rtol = s->o.rtol;
        a.maxit = s->o.maxit;
        a.fixed = s->o.fixed_iters;
      }
      args.push_back(a);
      starts.push_back(starts.back() + 1);
    }
    const int n = (int)args.size();
    add(seq, args, starts, [op, n](const Table<FinArgs>& t, hipStream_t st) { launch_fin(op, t, n, st); });
  }

  template <typename Tf, typename Tc, typename F>
  void xfer(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, int dir, F fill, int skip_mode) {
    std::map<std::pair<int, int>, std::vector<Slot*>> by;
    for (Slot* s : S) by[{s->level(l).N, s->level(l + 1).N}].push_back(s);
    for (auto& kv : by) {
      const int Nf = kv.first.first, Nc = kv.first.second;
      std::vector<XferArgs<Tf, Tc>> args;
      std::vector<int> starts{0};
      for (Slot* s : kv.second) {
        XferArgs<Tf, Tc> a;
        a.E = s->level(l).E;
        a.skip = skip(*s, skip_mode);
        fill(*s, a);
        args.push_back(a);
        starts.push_back(starts.back() + xfer_blocks(Nf, Nc, a.E));
      }
      const PmgLevel& lv = kv.second[0]->pmg->lv[l];
      const double* M = dir == 0 ? lv.J.as<double>() : lv.JT.as<double>();
      const int64_t total = starts.back();
      add(seq, args, starts, [dir, Nf, Nc, total, M](const Table<XferArgs<Tf, Tc>>& t, hipStream_t st) {
        launch_xfer<Tf, Tc>(dir, Nf, Nc, t, total, M, st);
      });
    }
  }

  // out = QQ^T-summed, masked Schwarz sum of local FDM solves of in (weights applied by the caller)
  template <typename T, typename FI, typename FO>
  void schwarz(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, FI in_of, FO out_of, int skip_mode) {
    std::map<int, std::vector<Slot*>> by;
    for (Slot* s : S) by[s->level(l).N].push_back(s);
    for (auto& kv : by) {
      const int N = kv.first;
      std::vector<SchwarzArgs<T>> args;
      std::vector<SchwarzPullArgs<T>> pargs;
      std::vector<int> starts{0};
      bool ras = false;
      for (Slot* s : kv.second) {
        const MeshData& m = s->level(l);
        const SchwarzData& sw = s->pmg->lv[l].sw;
        ras = sw.ras;
        SchwarzArgs<T> a;
        a.E = m.E;
        a.in = in_of(*s);
        a.out = out_of(*s);
        a.ovl = sw.ras ? nullptr : (T*)s->lovl[l];
        a.desc = sw.desc.as<int>();
        if constexpr (sizeof(T) == 8) {
          a.S = sw.S64.as<double>();
          a.lam = sw.L64.as<double>();
        } else {
          a.S = sw.S32.as<float>();
          a.lam = sw.L32.as<float>();
        }
        a.skip = skip(*s, skip_mode);
        args.push_back(a);
        SchwarzPullArgs<T> p;
        p.E = m.E;
        p.out = a.out;
        p.ovl = a.ovl;
        p.desc = a.desc;
        p.skip = a.skip;
        pargs.push_back(p);
        starts.push_back(starts.back() + schwarz_blocks(m.E));
      }
      const int64_t total = starts.back();
      add(seq, args, starts, [N, total](const Table<SchwarzArgs<T>>& t, hipStream_t st) {
        launch_schwarz<T>(N, 0, t, total, st);
      });
      if (!ras)  // one variant per group: the smoother is part of the plan signature
        add(seq, pargs, starts, [N, total](const Table<SchwarzPullArgs<T>>& t, hipStream_t st) {
          launch_schwarz_pull<T>(N, t, total, st);
        });
    }
    gs<T>(seq, S, l, out_of, skip_mode);
  }

  // one coarse CG iteration on unique DOFs of level l (parity par): p update fused
  // with the SpMV, then the x/r update
  void cg_iteration(std::vector<Fn>& seq, const std::vector<Slot*>& S, int l, int par, const sem_pmg_opts& o) {
    std::vector<CgArgs> args;
    std::vector<int> st_up{0};
    for (Slot* s : S) {
      const MeshData& m = s->level(l);
      CgArgs a;
      a.n = m.n_unique;
      a.W = m.ell_w;
      a.col = m.ell_col.as<int>();
      a.val = m.ell_val.as<double>();
      a.dinv = m.dinv_u.as<double>();
      a.x = s->cx;
      a.r = s->cr;
      a.w = s->cw;
      a.p = s->cp;
      a.z = s->cz;
      a.partial = s->partial;
      a.stride = s->stride;
      a.nblk_upd = cg_update_blocks(a.n);
      a.nblk_sp = cg_update_blocks(a.n);  // the SpMV launch runs on the same grid as the update
      a.scal = s->scal[1];
      a.flags = s->flags[1];
      a.total = s->flags[0] + F_TOTAL;
      a.par = par;
      a.rtol = o.coarse_rtol;
      a.maxit = o.coarse_fixed_iters > 0 ? (1 << 30) : o.coarse_maxit;
      a.fixed = o.coarse_fixed_iters;
      a.skip = skip(*s, 2);
      args.push_back(a);
      st_up.push_back(st_up.back() + (int)a.nblk_upd);
    }
    const int64_t tup = st_up.back();
    add(seq, args, st_up, [tup](const Table<CgArgs>& t, hipStream_t st) { launch_cg_pspmv(t, tup, st); });
    add(seq, args, st_up, [tup](const Table<CgArgs>& t, hipStream_t st) { launch_cg_update(t, tup, st); });
  }

  // skip modes: 0 none, 1 outer done, 2 outer or coarse done
  static Skip skip(const Slot& s, int mode) {
    Skip k;
    if (mode >= 1) k.f0 = s.flags[0] + F_DONE;
    if (mode >= 2) k.f1 = s.flags[1] + F_DONE;
    return k;
  }

  template <typename T>
  void build_vcycle(Group& g);
  void build_flex(Group& g);
  void build_jacobi(Group& g);
  void build_init(Group& g);
};

// ---------------------------------------------------------------------------
// V-cycle: r (FP64, slot.r) -> z (FP64, slot.z)
// ---------------------------------------------------------------------------
template <typename T>
void Plan::build_vcycle(Group& g) {
  auto& S = g.S;
  const int L = g.L;
  const sem_pmg_opts& o = S[0]->pmg->o;
  const int K = o.cheb_degree;
  constexpr int SK = 1;  // skip when the outer solve is done
  // with Chebyshev-Jacobi on the fine level, the entry precision conversion
  // is folded into the first smoothing step; with any smoother, the exit
  // conversion (and the outer solver's two dot products) into the last one
  const bool jac0 = !S[0]->pmg->lv[0].sw.on;
  const bool fold_in = jac0 && o.pre > 0 && K >= 2;
  const bool fold_out = o.post > 0;

  if (!fold_in) {
    if constexpr (sizeof(T) == 4)
      cast<double, float>(g.head, S, 0, [](Slot& s, CastArgs<double, float>& a) {
        a.in = s.r;
        a.out = (float*)s.lr[0];
      }, SK);
    else
      vec<double>(g.head, S, 0, V_COPY, [](Slot& s, VecArgs<double>& a) {
        a.x = (double*)s.lr[0];
        a.r = s.r;
      }, SK);
  }

  auto Tp = [](void* p) { return (T*)p; };

  // one Chebyshev-accelerated Schwarz sweep: D^-1 res of the Jacobi sweep
  // becomes W S(res), computed into ls before each update
  auto sweep_schwarz = [&](std::vector<Fn>& seq, int l, bool from_zero, bool out64) {
    const auto wts = [l](Slot& s) -> const T* {
      if constexpr (sizeof(T) == 8) return s.pmg->lv[l].sw.w64.template as<double>();
      else return s.pmg->lv[l].sw.w32.template as<float>();
    };
    const auto setv = [l, Tp, wts](Slot& s, VecArgs<T>& a) {
      a.r = Tp(s.ls[l]);
      a.x = Tp(s.lx[l]);
      a.res = Tp(s.lres[l]);
      a.d = Tp(s.ld[l]);
      a.t = Tp(s.lt[l]);
      a.dinv = wts(s);
      a.in64 = s.r;
      a.out64 = s.z;
      a.w64 = s.w;
    };
    const auto out_s = [l, Tp](Slot& s) { return Tp(s.ls[l]); };
    if (from_zero) {
      schwarz<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.lr[l]); }, out_s, SK);
      vec<T>(seq, S, l, V_CHEB_INIT0, [l, setv](Slot& s, VecArgs<T>& a) {
        setv(s, a);
        a.c0 = 1.0 / s.pmg->lv[l].theta;
      }, SK);
    } else {
      apply_A<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.lx[l]); }, [l, Tp](Slot& s) { return Tp(s.lt[l]); },
                 false, SK);
      vec<T>(seq, S, l, V_RES0, [l, Tp](Slot& s, VecArgs<T>& a) {
        a.r = Tp(s.lr[l]);
        a.res = Tp(s.lres[l]);
        a.t = Tp(s.lt[l]);
      }, SK);
      schwarz<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.lres[l]); }, out_s, SK);
      vec<T>(seq, S, l, out64 && K == 1 ? V_CHEB_UPD0_OUT64 : V_CHEB_UPD0, [l, setv](Slot& s, VecArgs<T>& a) {
        setv(s, a);
        a.c2 = 1.0 / s.pmg->lv[l].theta;
      }, SK);
    }
    for (int j = 1; j < K; ++j) {
      apply_A<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.ld[l]); }, [l, Tp](Slot& s) { return Tp(s.lt[l]); },
                 false, SK);
      const VecOp rop = (from_zero && j == 1) ? V_RES0 : V_RES;
      vec<T>(seq, S, l, rop, [l, Tp](Slot& s, VecArgs<T>& a) {
        a.r = Tp(s.lr[l]);
        a.res = Tp(s.lres[l]);
        a.t = Tp(s.lt[l]);
      }, SK);
      schwarz<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.lres[l]); }, out_s, SK);
      vec<T>(seq, S, l, out64 && j == K - 1 ? V_CHEB_UPD_OUT64 : V_CHEB_UPD, [l, j, setv](Slot& s, VecArgs<T>& a) {
        setv(s, a);
        a.c1 = s.pmg->lv[l].c1[j - 1];
        a.c2 = s.pmg->lv[l].c2[j - 1];
      }, SK);
    }
  };

  // one Chebyshev sweep at level l; from_zero: x0 = 0
  // One Chebyshev-Jacobi sweep at level l; from_zero: x0 = 0. Writes that no
  // later step reads are left out: the last step updates x only, a sweep from
  // zero keeps x = d implicit until its second step. in64: the sweep starts
  // from the FP64 outer residual (V-cycle entry cast folded into the first
  // step); out64: its last step writes the FP64 V-cycle output instead of x.
  auto sweep = [&](std::vector<Fn>& seq, int l, bool from_zero, bool in64 = false, bool out64 = false) {
    if (S[0]->pmg->lv[l].sw.on) {
      sweep_schwarz(seq, l, from_zero, out64);
      return;
    }
    const auto setv = [l, Tp](Slot& s, VecArgs<T>& a) {
      a.r = Tp(s.lr[l]);
      a.x = Tp(s.lx[l]);
      a.res = Tp(s.lres[l]);
      a.d = Tp(s.ld[l]);
      a.t = Tp(s.lt[l]);
      a.dinv = dinv_of<T>(s.level(l));
      a.in64 = s.r;
      a.out64 = s.z;
      a.w64 = s.w;
    };
    if (from_zero) {
      const VecOp op = K == 1 ? V_CHEB_INIT0 : (in64 ? V_CHEB_INIT0D_IN64 : V_CHEB_INIT0D);
      vec<T>(seq, S, l, op, [l, setv](Slot& s, VecArgs<T>& a) {
        setv(s, a);
        a.c0 = 1.0 / s.pmg->lv[l].theta;
      }, SK);
    } else {
      apply_A<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.lx[l]); }, [l, Tp](Slot& s) { return Tp(s.lt[l]); },
                 false, SK);
      const VecOp op = K > 1 ? V_CHEB_INITX : (out64 ? V_CHEB_INITX_OUT64 : V_CHEB_INITX_LAST);
      vec<T>(seq, S, l, op, [l, setv](Slot& s, VecArgs<T>& a) {
        setv(s, a);
        a.c0 = 1.0 / s.pmg->lv[l].theta;
      }, SK);
    }
    for (int j = 1; j < K; ++j) {
      apply_A<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.ld[l]); }, [l, Tp](Slot& s) { return Tp(s.lt[l]); },
                 false, SK);
      const bool last = j == K - 1;
      VecOp op;
      if (from_zero && j == 1) op = last ? V_CHEB_LAST0X : V_CHEB_STEP0X;
      else op = last ? (out64 ? V_CHEB_LAST_OUT64 : V_CHEB_LAST) : V_CHEB_STEP;
      vec<T>(seq, S, l, op, [l, j, setv](Slot& s, VecArgs<T>& a) {
        setv(s, a);
        a.c1 = s.pmg->lv[l].c1[j - 1];
        a.c2 = s.pmg->lv[l].c2[j - 1];
      }, SK);
    }
  };

  // down-sweep
  for (int l = 0; l + 1 < L; ++l) {
    auto& seq = g.head;
    if (o.pre > 0) {
      sweep(seq, l, true, l == 0 && fold_in);
      for (int q = 1; q < o.pre; ++q) sweep(seq, l, false);
      apply_A<T>(seq, S, l, [l, Tp](Slot& s) { return (const T*)Tp(s.lx[l]); }, [l, Tp](Slot& s) { return Tp(s.lt[l]); },
                 false, SK);
    } else {
      vec<T>(seq, S, l, V_ZERO, [l, Tp](Slot& s, VecArgs<T>& a) { a.x = Tp(s.lx[l]); }, SK);
    }
    const bool pre = o.pre > 0;
    if (l + 2 == L) {
      const bool asmb = S[0]->level(L - 1).assembled;
      xfer<T, double>(seq, S, l, 1, [l, Tp, pre, asmb](Slot& s, XferArgs<T, double>& a) {
        a.rf = Tp(s.lr[l]);
        a.tf = pre ? Tp(s.lt[l]) : nullptr;
        a.owner_f = s.level(l).owner.as<uint8_t>();
        a.out_c = asmb ? s.clocal : s.cr;
      }, SK);
      if (asmb)
        usum(seq, S, l + 1, [](Slot& s) { return (const double*)s.clocal; }, [](Slot& s) { return s.cr; }, SK);
      else
        gs<double>(seq, S, l + 1, [](Slot& s) { return s.cr; }, SK);
    } else {
      xfer<T, T>(seq, S, l, 1, [l, Tp, pre](Slot& s, XferArgs<T, T>& a) {
        a.rf = Tp(s.lr[l]);
        a.tf = pre ? Tp(s.lt[l]) : nullptr;
        a.owner_f = s.level(l).owner.as<uint8_t>();
        a.out_c = Tp(s.lr[l + 1]);
      }, SK);
      gs<T>(seq, S, l + 1, [l, Tp](Slot& s) { return Tp(s.lr[l + 1]); }, SK);
    }
  }

  // coarse Jacobi-PCG, FP64 (on unique DOFs when the level is assembled)
  {
    const int c = L - 1;
    const bool U = S[0]->level(c).assembled;
    g.coarse_limit = o.coarse_fixed_iters > 0 ? o.coarse_fixed_iters : o.coarse_maxit;
    g.coarse_fixed = o.coarse_fixed_iters;
    g.coarse_check = o.coarse_check_every;
    if (U) {
      // a pass of the loop body is two iterations (both parities)
      g.coarse_limit = (g.coarse_limit + 1) / 2;
      g.coarse_fixed = g.coarse_fixed > 0 ? g.coarse_limit : 0;
      g.coarse_check = std::max(1, g.coarse_check / 2);
    }
    auto nvec = [c, U](Slot& s) { return vec_blocks(U ? s.level(c).n_unique : s.level(c).nloc); };
    auto cdinv = [c, U](Slot& s) { return U ? s.level(c).dinv_u.as<double>() : s.level(c).dinv64.as<double>(); };
    vec<double>(g.cinit, S, c, V_ZERO, [](Slot& s, VecArgs<double>& a) { a.x = s.cx; }, SK, U);
    vec<double>(g.cinit, S, c, V_DOT1, [](Slot& s, VecArgs<double>& a) { a.r = s.cr; }, SK, U);
    fin(g.cinit, S, FIN_INIT, 1, nvec, SK);
    vec<double>(g.cinit, S, c, V_RZ_JACOBI, [cdinv, U](Slot& s, VecArgs<double>& a) {
      a.r = s.cr;
      a.p = U ? s.cz : s.cp;  // assembled: z = D^-1 r, which the first SpMV gathers
      a.dinv = cdinv(s);
    }, SK, U);
    fin(g.cinit, S, FIN_RZ, 1, nvec, SK);

    if (U) {
      cg_iteration(g.citer, S, c, 0, o);
      cg_iteration(g.citer, S, c, 1, o);
    } else {
      apply_A<double>(g.citer, S, c, [](Slot& s) { return (const double*)s.cp; }, [](Slot& s) { return s.cw; }, true, 2);
      fin(g.citer, S, FIN_ALPHA, 1, [c](Slot& s) { return (int64_t)ax_blocks(s.level(c).N, s.level(c).E); }, 2);
      vec<double>(g.citer, S, c, V_PCG_UPDATE, [cdinv](Slot& s, VecArgs<double>& a) {
        a.x = s.cx;
        a.p = s.cp;
        a.r = s.cr;
        a.w = s.cw;
        a.dinv = cdinv(s);
        a.scal = s.scal[1];
      }, 2);
      fin(g.citer, S, FIN_CHECK_JACOBI, 1, nvec, 2, o.coarse_rtol,
          o.coarse_fixed_iters > 0 ? (1 << 30) : o.coarse_maxit, o.coarse_fixed_iters, true);
      vec<double>(g.citer, S, c, V_P_JACOBI, [cdinv](Slot& s, VecArgs<double>& a) {
        a.p = s.cp;
        a.r = s.cr;
        a.dinv = cdinv(s);
        a.scal = s.scal[1];
      }, 2);
    }
  }

  // up-sweep
  for (int l = L - 2; l >= 0; --l) {
    auto& seq = g.tail;
    if (l + 2 == L) {
      xfer<T, double>(seq, S, l, 0, [l, L, Tp](Slot& s, XferArgs<T, double>& a) {
        a.zc = s.cx;
        a.umap_c = s.level(L - 1).assembled ? s.level(L - 1).umap.as<int>() : nullptr;
        a.xf = Tp(s.lx[l]);
      }, SK);
    } else {
      xfer<T, T>(seq, S, l, 0, [l, Tp](Slot& s, XferArgs<T, T>& a) {
        a.zc = Tp(s.lx[l + 1]);
        a.xf = Tp(s.lx[l]);
      }, SK);
    }
    for (int q = 0; q < o.post; ++q) sweep(seq, l, false, false, l == 0 && fold_out && q + 1 == o.post);
  }

  if (!fold_out) {
    if constexpr (sizeof(T) == 4)
      cast<float, double>(g.tail, S, 0, [](Slot& s, CastArgs<float, double>& a) {
        a.in = (const float*)s.lx[0];
        a.out = s.z;
      }, SK);
    else
      vec<double>(g.tail, S, 0, V_COPY, [](Slot& s, VecArgs<double>& a) {
        a.x = s.z;
        a.r = (double*)s.lx[0];
      }, SK);
  }
}

// outer flexible CG body (after the V-cycle has produced z from r)
void Plan::build_flex(Group& g) {
  auto& S = g.S;
  if (S[0]->f32()) build_vcycle<float>(g); else build_vcycle<double>(g);
  if (g.vcycle_only) return;
  auto& t = g.tail;
  // with post-smoothing on the fine level, the V-cycle's last step already
  // left the partials of (z, w) and (z, r)
  const sem_pmg_opts& o = S[0]->pmg->o;
  if (o.post == 0)
    vec<double>(t, S, 0, V_DOT2, [](Slot& s, VecArgs<double>& a) {
      a.z = s.z;
      a.w = s.w;
      a.r = s.r;
    }, 1);
  fin(t, S, FIN_BETA_FLEX, 0, [](Slot& s) { return vec_blocks(s.level(0).nloc); }, 1);
  vec<double>(t, S, 0, V_P_FLEX, [](Slot& s, VecArgs<double>& a) {
    a.p = s.p;
    a.z = s.z;
    a.scal = s.scal[0];
  }, 1);
  apply_A<double>(t, S, 0, [](Slot& s) { return (const double*)s.p; }, [](Slot& s) { return s.w; }, true, 1);
  fin(t, S, FIN_ALPHA, 0, [](Slot& s) { return (int64_t)ax_blocks(s.level(0).N, s.level(0).E); }, 1);
  vec<double>(t, S, 0, V_PCG_UPDATE, [](Slot& s, VecArgs<double>& a) {
    a.x = s.x;
    a.p = s.p;
    a.r = s.r;
    a.w = s.w;
    a.scal = s.scal[0];
  }, 1);
  fin(t, S, FIN_CHECK, 0, [](Slot& s) { return vec_blocks(s.level(0).nloc); }, 1);
}

void Plan::build_jacobi(Group& g) {
  auto& S = g.S;
  auto& h = g.head;
  apply_A<double>(h, S, 0, [](Slot& s) { return (const double*)s.p; }, [](Slot& s) { return s.w; }, true, 1);
  fin(h, S, FIN_ALPHA, 0, [](Slot& s) { return (int64_t)ax_blocks(s.level(0).N, s.level(0).E); }, 1);
  vec<double>(h, S, 0, V_PCG_UPDATE, [](Slot& s, VecArgs<double>& a) {
    a.x = s.x;
    a.p = s.p;
    a.r = s.r;
    a.w = s.w;
    a.dinv = s.dinv0();
    a.scal = s.scal[0];
  }, 1);
  fin(h, S, FIN_CHECK_JACOBI, 0, [](Slot& s) { return vec_blocks(s.level(0).nloc); }, 1);
  vec<double>(h, S, 0, V_P_JACOBI, [](Slot& s, VecArgs<double>& a) {
    a.p = s.p;
    a.r = s.r;
    a.dinv = s.dinv0();
    a.scal = s.scal[0];
  }, 1);
}

// x = 0, r = b, ||b||; Jacobi: p = D^-1 r and (r, p); flexible CG: p = w = 0
void Plan::build_init(Group& g) {
  auto& S = g.S;
  auto& q = g.init;
  vec<double>(q, S, 0, V_ZERO, [](Slot& s, VecArgs<double>& a) { a.x = s.x; }, 0);
  vec<double>(q, S, 0, V_COPY, [](Slot& s, VecArgs<double>& a) {
    a.x = s.r;
    a.r = const_cast<double*>(s.b);
  }, 0);
  vec<double>(q, S, 0, V_DOT1, [](Slot& s, VecArgs<double>& a) { a.r = s.r; }, 0);
  fin(q, S, FIN_INIT, 0, [](Slot& s) { return vec_blocks(s.level(0).nloc); }, 0);
  if (g.pmg) {
    vec<double>(q, S, 0, V_ZERO, [](Slot& s, VecArgs<double>& a) { a.x = s.p; }, 0);
    vec<double>(q, S, 0, V_ZERO, [](Slot& s, VecArgs<double>& a) { a.x = s.w; }, 0);
  } else {
    vec<double>(q, S, 0, V_RZ_JACOBI, [](Slot& s, VecArgs<double>& a) {
      a.r = s.r;
      a.p = s.p;
      a.dinv = s.dinv0();
    }, 1);
    fin(q, S, FIN_RZ, 0, [](Slot& s) { return vec_blocks(s.level(0).nloc); }, 1);
  }
}

// group slots by solver structure
static std::string signature(const Slot& s) {
  if (!s.pmg) return s.lam() != 0.0 ? "jacobi-helmholtz" : "jacobi";
  const sem_pmg_opts& o = s.pmg->o;
  // every option a group reads from its first problem (the per-level data,
  // rho and the Chebyshev coefficients, are read per problem)
  char buf[160];
  snprintf(buf, sizeof(buf), "pmg L%d t%d k%d pre%d post%d cf%d cm%d cc%d sm%d cr%.17g", s.pmg->n_levels,
           (int)o.smoother_dtype, o.cheb_degree, o.pre, o.post, o.coarse_fixed_iters, o.coarse_maxit,
           o.coarse_check_every, o.smoother, o.coarse_rtol);
  return buf;
}

static std::unique_ptr<Plan> make_plan(const std::vector<Slot*>& slots, bool init, bool vcycle_only,
                                       hipStream_t s) {
  auto P = std::make_unique<Plan>();
  std::map<std::string, std::vector<Slot*>> by;
  for (Slot* sl : slots) by[signature(*sl)].push_back(sl);
  P->groups.reserve(by.size());
  for (auto& kv : by) {
    P->groups.emplace_back();
    Group& g = P->groups.back();
    g.S = kv.second;
    g.pmg = g.S[0]->pmg != nullptr;
    g.L = g.S[0]->nlev();
    g.vcycle_only = vcycle_only;
    if (init) P->build_init(g);
    else if (g.pmg) P->build_flex(g);
    else P->build_jacobi(g);
  }
  P->upload(s);
  return P;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
}  // namespace sem

// An asynchronous look at the slots' flags: a copy of the flag block into
// pinned memory queued behind the work so far, and an event after it. The
// host queues more work before waiting on the event, so the device never
// drains while the host reads convergence flags.
struct sem_probe {
  void* host = nullptr;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

struct sem_batch_s {
  hipStream_t stream = nullptr;
  int max_slots = 0;
  std::vector<sem::Slot> slots;
  sem::DevBuf ctrl;             // per slot: 2 x S_COUNT doubles, then 2 x F_COUNT ints
  void* host_ctrl = nullptr;    // pinned mirror
  size_t ctrl_bytes = 0;
  std::unique_ptr<sem::Plan> plan;
  bool dirty = true;
  sem_probe probe_outer, probe_coarse;  // separate channels: a coarse loop runs while an outer probe is pending
  int64_t launches = 0;                 // kernels queued through plans so far

  size_t scal_bytes() const { return sizeof(double) * 2 * sem::S_COUNT * max_slots; }
  size_t flag_bytes() const { return sizeof(int) * 2 * sem::F_COUNT * max_slots; }
  ~sem_batch_s() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& s : slots) sem::pool_put(s.ws, s.ws_bytes);
    if (host_ctrl) (void)hipHostFree(host_ctrl);
    for (sem_probe* p : {&probe_outer, &probe_coarse}) {
      if (p->host) (void)hipHostFree(p->host);
      if (p->ev) (void)hipEventDestroy(p->ev);
    }
  }
};

namespace sem {

static void batch_init(sem_batch_s* B, int max_slots, hipStream_t s) {
  B->stream = s;
  B->max_slots = max_slots;
  B->slots.resize(max_slots);
  B->ctrl_bytes = B->scal_bytes() + sizeof(int) * 2 * F_COUNT * max_slots;
  B->ctrl.alloc(B->ctrl_bytes);
  SEM_HIP(hipMemsetAsync(B->ctrl.p, 0, B->ctrl_bytes, s));
  SEM_HIP(hipHostMalloc(&B->host_ctrl, B->ctrl_bytes, hipHostMallocDefault));
  for (sem_probe* p : {&B->probe_outer, &B->probe_coarse}) {
    SEM_HIP(hipHostMalloc(&p->host, B->flag_bytes(), hipHostMallocDefault));
    SEM_HIP(hipEventCreateWithFlags(&p->ev, hipEventDisableTiming));
  }
  for (int k = 0; k < max_slots; ++k) {
    Slot& sl = B->slots[k];
    sl.idx = k;
    double* sc = B->ctrl.as<double>() + (size_t)2 * S_COUNT * k;
    int* fl = reinterpret_cast<int*>(B->ctrl.as<uint8_t>() + B->scal_bytes()) + (size_t)2 * F_COUNT * k;
    sl.scal[0] = sc;
    sl.scal[1] = sc + S_COUNT;
    sl.flags[0] = fl;
    sl.flags[1] = fl + F_COUNT;
    sl.ctrl_clean = true;  // cleared above
  }
}

static void fetch_ctrl(sem_batch_s* B) {
  SEM_HIP(hipMemcpyAsync(B->host_ctrl, B->ctrl.p, B->ctrl_bytes, hipMemcpyDeviceToHost, B->stream));
  SEM_HIP(hipStreamSynchronize(B->stream));
}
static const double* host_scal(sem_batch_s* B, int k, int stage) {
  return static_cast<const double*>(B->host_ctrl) + (size_t)2 * S_COUNT * k + (size_t)stage * S_COUNT;
}
static const int* host_flags(sem_batch_s* B, int k, int stage) {
  return reinterpret_cast<const int*>(static_cast<const uint8_t*>(B->host_ctrl) + B->scal_bytes()) +
         (size_t)2 * F_COUNT * k + (size_t)stage * F_COUNT;
}

static void probe_post(sem_batch_s* B, sem_probe& p) {
  if (p.pending) fail(SEM_EHIP, "internal: a probe is already pending");
  SEM_HIP(hipMemcpyAsync(p.host, B->ctrl.as<uint8_t>() + B->scal_bytes(), B->flag_bytes(), hipMemcpyDeviceToHost,
                         B->stream));
  SEM_HIP(hipEventRecord(p.ev, B->stream));
  p.pending = true;
}
// waits for the pending probe; returns its flag block
static const int* probe_wait(sem_probe& p) {
  SEM_HIP(hipEventSynchronize(p.ev));
  p.pending = false;
  return static_cast<const int*>(p.host);
}
static const int* probe_flags(const int* block, int k, int stage) {
  return block + (size_t)2 * F_COUNT * k + (size_t)stage * F_COUNT;
}

// queues one plan sequence (one kernel per entry) and counts its launches
static void run(sem_batch_s* B, const std::vector<Fn>& seq) {
  for (const Fn& f : seq) f(B->stream);
  B->launches += (int64_t)seq.size();
}

// one pass of every group's body. The coarse loop is queued in chunks; after
// queuing chunk k+1 the host reads the flags probed after chunk k, so it is
// always one chunk ahead of the device (a chunk queued after the last problem
// finished runs as no-ops: its launches skip finished problems).
static void run_body(sem_batch_s* B, Plan& P) {
  for (Group& g : P.groups) {
    run(B, g.head);
    if (!g.cinit.empty()) {
      run(B, g.cinit);
      sem_probe& pr = B->probe_coarse;
      int ran = 0;
      while (ran < g.coarse_limit) {
        const int chunk = g.coarse_fixed > 0 ? g.coarse_limit : std::min(g.coarse_check, g.coarse_limit - ran);
        for (int k = 0; k < chunk; ++k) run(B, g.citer);
        ran += chunk;
        if (pr.pending) {
          const int* fl = probe_wait(pr);
          bool all = true;
          for (Slot* s : g.S)
            if (!probe_flags(fl, s->idx, 0)[F_DONE] && !probe_flags(fl, s->idx, 1)[F_DONE]) all = false;
          if (all) break;
        }
        if (ran >= g.coarse_limit) break;
        probe_post(B, pr);
      }
      if (pr.pending) (void)probe_wait(pr);
    }
    run(B, g.tail);
  }
}

static void batch_add(sem_batch_s* B, sem_mesh m, sem_pmg p, const double* b, double* x, const sem_solve_opts* oin,
                      int* slot_out) {
  if (!m || !b || !x) fail(SEM_EINVAL, "batch add: NULL argument");
  if (p && p->base != m) fail(SEM_EINVAL, "batch add: the pMG hierarchy was built on another mesh");
  int k = -1;
  for (int q = 0; q < B->max_slots; ++q)
    if (B->slots[q].state == 0) { k = q; break; }
  if (k < 0) fail(SEM_EBUSY, "batch add: all %d slots are in use", B->max_slots);
  Slot& s = B->slots[k];
  s.mesh = m;
  s.pmg = p;
  s.b = b;
  s.x = x;
  sem_solve_opts_default(&s.o);
  if (oin) s.o = *oin;
  if (!(s.o.rtol >= 0)) fail(SEM_EINVAL, "batch add: rtol must be >= 0");
  if (p && s.o.lambda != 0.0)
    fail(SEM_EINVAL, "batch add: Helmholtz (lambda != 0) is solved by Jacobi-PCG; pass no pMG hierarchy");
  if (!std::isfinite(s.o.lambda) || s.o.lambda < 0.0) fail(SEM_EINVAL, "batch add: lambda must be finite and >= 0");
  if (s.o.maxit < 1) s.o.maxit = 1;
  if (s.o.check_every < 1) s.o.check_every = 1;
  const size_t bytes = layout(s, nullptr);
  s.ws = pool_get(bytes);
  s.ws_bytes = bytes;
  layout(s, static_cast<uint8_t*>(s.ws));
  if (s.lam() != 0.0) helmholtz_dinv(s.level(0), s.lam(), s.dinv_h, s.w, B->stream);
  s.state = 1;
  s.info = sem_solve_info{};
  s.info.status = 1;
  s.info.relres_initial = 1.0;  // x0 = 0
  s.t0 = Clock::now();
  s.launches0 = B->launches;
  if (!s.ctrl_clean) {  // a reused slot: clear what the previous solve left
    SEM_HIP(hipMemsetAsync(s.scal[0], 0, sizeof(double) * 2 * S_COUNT, B->stream));
    SEM_HIP(hipMemsetAsync(s.flags[0], 0, sizeof(int) * 2 * F_COUNT, B->stream));
  }
  s.ctrl_clean = false;
  B->dirty = true;
  if (slot_out) *slot_out = k;
}

static void batch_release(sem_batch_s* B, int k) {
  if (k < 0 || k >= B->max_slots) fail(SEM_EINVAL, "batch release: slot %d out of range", k);
  Slot& s = B->slots[k];
  if (s.state == 0) return;
  SEM_HIP(hipStreamSynchronize(B->stream));
  pool_put(s.ws, s.ws_bytes);
  s.ws = nullptr;
  s.ws_bytes = 0;
  if (s.state == 1 || s.state == 2) B->dirty = true;
  s.state = 0;
  s.mesh = nullptr;
  s.pmg = nullptr;
}

// Retire finished solves: their info from the fetched flags, and the true
// residual ||b - H x|| of all of them in one pass (one launch per kernel over
// every slot, one reduction per slot, one copy back) instead of one
// synchronised pass per slot. The caller has fetched the control block.
static void finish_slots(sem_batch_s* B, const std::vector<Slot*>& S) {
  std::vector<Slot*> need;
  for (Slot* s : S) {
    const double* sc = host_scal(B, s->idx, 0);
    const int* fl = host_flags(B, s->idx, 0);
    s->info.iters = fl[F_ITERS];
    s->info.status = fl[F_STATUS];
    s->info.relres = sc[S_RELRES];
    s->info.coarse_iters = fl[F_TOTAL];
    const double bb = sc[S_BB];
    if (bb > 0 && std::isfinite(bb) && s->info.status != SEM_ENAN) need.push_back(s);
    else s->info.relres_true = (bb == 0) ? 0.0 : NAN;
  }
  if (!need.empty()) {
    Plan P;
    std::vector<Fn> seq;
    P.apply_A<double>(seq, need, 0, [](Slot& s) { return (const double*)s.x; }, [](Slot& s) { return s.w; }, false, 0);
    P.vec<double>(seq, need, 0, V_TRUE_RES, [](Slot& s, VecArgs<double>& a) {
      a.r = const_cast<double*>(s.b);
      a.t = s.w;
    }, 0);
    P.fin(seq, need, FIN_STORE, 0, [](Slot& s) { return vec_blocks(s.level(0).nloc); }, 0);
    P.upload(B->stream);
    run(B, seq);
    fetch_ctrl(B);  // also waits before P's tables are freed
    for (Slot* s : need)
      s->info.relres_true = std::sqrt(host_scal(B, s->idx, 0)[S_TMP] / host_scal(B, s->idx, 0)[S_BB]);
  }
  const auto now = Clock::now();
  for (Slot* s : S) {
    s->info.seconds = std::chrono::duration<double>(now - s->t0).count();
    s->info.launches = B->launches - s->launches0;
    s->state = 3;
  }
}

static int batch_step(sem_batch_s* B, int iters) {
  // initialise newly admitted solves
  std::vector<Slot*> fresh;
  for (Slot& s : B->slots)
    if (s.state == 1) fresh.push_back(&s);
  if (!fresh.empty()) {
    auto P = make_plan(fresh, true, false, B->stream);
    for (Group& g : P->groups) run(B, g.init);
    SEM_HIP(hipStreamSynchronize(B->stream));
    for (Slot* s : fresh) s->state = 2;
    B->dirty = true;
  }
  std::vector<Slot*> act;
  for (Slot& s : B->slots)
    if (s.state == 2) act.push_back(&s);
  if (act.empty()) return 0;
  // problems that are already done after init (zero or NaN rhs) retire now
  fetch_ctrl(B);
  {
    std::vector<Slot*> still, done;
    for (Slot* s : act) (host_flags(B, s->idx, 0)[F_DONE] ? done : still).push_back(s);
    if (!done.empty()) {
      finish_slots(B, done);
      B->dirty = true;
    }
    act.swap(still);
  }
  if (act.empty()) return 0;
  if (B->dirty || !B->plan) {
    SEM_HIP(hipStreamSynchronize(B->stream));
    B->plan = make_plan(act, false, false, B->stream);
    B->dirty = false;
  }
  for (int it = 0; it < iters; ++it) run_body(B, *B->plan);
  fetch_ctrl(B);
  std::vector<Slot*> done;
  for (Slot* s : act)
    if (host_flags(B, s->idx, 0)[F_DONE]) done.push_back(s);
  if (!done.empty()) {
    finish_slots(B, done);
    B->dirty = true;
  }
  return (int)(act.size() - done.size());
}

}  // namespace sem

using namespace sem;

extern "C" void sem_solve_opts_default(sem_solve_opts* o) {
  if (!o) return;
  *o = sem_solve_opts{};
  o->rtol = 1e-8;
  o->maxit = 10000;
  o->check_every = 1;
  o->fixed_iters = 0;
  o->lambda = 0.0;
}

extern "C" size_t sem_solve_workspace_bytes(sem_mesh m, sem_pmg p) {
  if (!m) return 0;
  try {
    Slot s;
    s.mesh = m;
    s.pmg = p;
    return layout(s, nullptr);
  } catch (...) {
    return 0;
  }
}

extern "C" int sem_batch_create(int max_slots, void* stream, sem_batch* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out || max_slots < 1) fail(SEM_EINVAL, "sem_batch_create: bad argument");
    auto B = std::make_unique<sem_batch_s>();
    batch_init(B.get(), max_slots, (hipStream_t)stream);
    *out = B.release();
  });
}

extern "C" int sem_batch_destroy(sem_batch b) {
  return guarded([&] { delete b; });
}

extern "C" int sem_batch_add(sem_batch b, sem_mesh m, sem_pmg p, const double* rhs, double* x,
                             const sem_solve_opts* o, int* slot) {
  return guarded([&] {
    if (!b) fail(SEM_EINVAL, "sem_batch_add: NULL batch");
    batch_add(b, m, p, rhs, x, o, slot);
  });
}

extern "C" int sem_batch_step(sem_batch b, int iters, int* n_active) {
  return guarded([&] {
    if (!b) fail(SEM_EINVAL, "sem_batch_step: NULL batch");
    const int n = batch_step(b, iters < 1 ? 1 : iters);
    if (n_active) *n_active = n;
  });
}

extern "C" int sem_batch_poll(sem_batch b, int slot, sem_solve_info* info) {
  return guarded([&] {
    if (!b || !info) fail(SEM_EINVAL, "sem_batch_poll: NULL argument");
    if (slot < 0 || slot >= b->max_slots) fail(SEM_EINVAL, "sem_batch_poll: slot %d out of range", slot);
    const Slot& s = b->slots[slot];
    *info = s.info;
    if (s.state == 1 || s.state == 2) info->status = 1;
    if (s.state == 0) fail(SEM_EINVAL, "sem_batch_poll: slot %d is free", slot);
  });
}

extern "C" int sem_batch_release(sem_batch b, int slot) {
  return guarded([&] {
    if (!b) fail(SEM_EINVAL, "sem_batch_release: NULL batch");
    batch_release(b, slot);
  });
}

static int solve_many(int n, const sem_mesh* m, const sem_pmg* p, const double* const* b, double* const* x,
                      const sem_solve_opts* o, sem_solve_info* info, void* stream) {
  sem_batch_s B;
  batch_init(&B, n, (hipStream_t)stream);
  const auto t0 = Clock::now();
  for (int k = 0; k < n; ++k) batch_add(&B, m[k], p ? p[k] : nullptr, b[k], x[k], o, nullptr);
  const int every = (o && o->check_every > 0) ? o->check_every : 1;
  int64_t cap = 0;
  for (int k = 0; k < n; ++k) cap = std::max<int64_t>(cap, std::max(B.slots[k].o.maxit, B.slots[k].o.fixed_iters));
  int64_t ran = 0;
  // the first step initialises every problem (and retires those done at once);
  // after it the host stays one step ahead: it queues step k+1 before reading
  // the flags probed after step k, and a step queued after the last problem
  // finished runs as no-ops. The device marks every problem done by maxit;
  // the host bound is a backstop.
  if (batch_step(&B, every) > 0) {
    sem_probe& pr = B.probe_outer;
    while (true) {
      for (int it = 0; it < every; ++it) run_body(&B, *B.plan);
      ran += every;
      if (pr.pending) {
        const int* fl = probe_wait(pr);
        bool all = true;
        for (const Slot& s : B.slots)
          if (s.state == 2 && !probe_flags(fl, s.idx, 0)[F_DONE]) all = false;
        if (all) break;
      }
      if (ran > cap + 2 * every + 8) fail(SEM_EHIP, "solve: device convergence flags did not settle");
      probe_post(&B, pr);
    }
    if (pr.pending) (void)probe_wait(pr);
    fetch_ctrl(&B);
    std::vector<Slot*> done;
    for (Slot& s : B.slots)
      if (s.state == 2) done.push_back(&s);
    finish_slots(&B, done);
  }
  int worst = SEM_OK;
  const double secs = std::chrono::duration<double>(Clock::now() - t0).count();
  for (int k = 0; k < n; ++k) {
    Slot& s = B.slots[k];
    if (info) {
      info[k] = s.info;
      info[k].seconds = secs;
    }
    if (s.info.status < 0 && worst == SEM_OK) worst = s.info.status;
  }
  if (worst == SEM_ENOCONV) set_error("solve: iteration limit reached");
  if (worst == SEM_ENAN) set_error("solve: NaN or Inf in the right-hand side or an iterate");
  return worst;
}

extern "C" int sem_pcg_solve(sem_mesh m, sem_pmg p, const double* b, double* x, const sem_solve_opts* o,
                             sem_solve_info* info, void* stream) {
  int rc = SEM_OK;
  int g = guarded([&] {
    if (!m || !b || !x) fail(SEM_EINVAL, "sem_pcg_solve: NULL argument");
    rc = solve_many(1, &m, p ? &p : nullptr, &b, &x, o, info, stream);
  });
  return g != SEM_OK ? g : rc;
}

extern "C" int sem_pcg_solve_batched(int n, const sem_mesh* m, const sem_pmg* p, const double* const* b,
                                     double* const* x, const sem_solve_opts* o, sem_solve_info* info, void* stream) {
  int rc = SEM_OK;
  int g = guarded([&] {
    if (n < 1 || !m || !b || !x) fail(SEM_EINVAL, "sem_pcg_solve_batched: bad argument");
    rc = solve_many(n, m, p, b, x, o, info, stream);
  });
  return g != SEM_OK ? g : rc;
}

namespace sem {

// a one-slot batch whose plan is the V-cycle alone
struct VcycleRunner {
  sem_batch_s B;
  std::unique_ptr<Plan> P;
  sem_pmg p = nullptr;
};

VcycleRunner* vcycle_runner_create(sem_pmg p, hipStream_t st) {
  auto v = std::make_unique<VcycleRunner>();
  v->p = p;
  batch_init(&v->B, 1, st);
  Slot& s = v->B.slots[0];
  s.mesh = p->base;
  s.pmg = p;
  const size_t bytes = layout(s, nullptr);
  s.ws = pool_get(bytes);
  s.ws_bytes = bytes;
  layout(s, static_cast<uint8_t*>(s.ws));
  s.state = 2;
  std::vector<Slot*> one{&s};
  v->P = make_plan(one, false, true, st);
  return v.release();
}

// the V-cycle reads slot.r and writes slot.z: copy r in, z out
void vcycle_runner_apply(VcycleRunner* v, const double* r, double* z) {
  Slot& s = v->B.slots[0];
  const size_t bytes = sizeof(double) * v->p->base->d.nloc;
  SEM_HIP(hipMemcpyAsync(s.r, r, bytes, hipMemcpyDeviceToDevice, v->B.stream));
  run_body(&v->B, *v->P);
  SEM_HIP(hipMemcpyAsync(z, s.z, bytes, hipMemcpyDeviceToDevice, v->B.stream));
}

int64_t vcycle_runner_coarse_iters(VcycleRunner* v) {
  fetch_ctrl(&v->B);
  return host_flags(&v->B, 0, 0)[F_TOTAL];
}

void vcycle_runner_destroy(VcycleRunner* v) { delete v; }

}  // namespace sem

extern "C" int sem_pmg_apply(sem_pmg p, const double* r, double* z, void* stream) {
  return guarded([&] {
    if (!p || !r || !z) fail(SEM_EINVAL, "sem_pmg_apply: NULL argument");
    std::unique_ptr<VcycleRunner, void (*)(VcycleRunner*)> v(vcycle_runner_create(p, (hipStream_t)stream),
                                                              vcycle_runner_destroy);
    vcycle_runner_apply(v.get(), r, z);
    SEM_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

extern "C" int sem_pmg_transfer(sem_pmg p, int level, int direction, const void* in, void* out, void* stream) {
  return guarded([&] {
    if (!p || !in || !out) fail(SEM_EINVAL, "sem_pmg_transfer: NULL argument");
    if (level < 0 || level + 1 >= p->n_levels) fail(SEM_EINVAL, "sem_pmg_transfer: level %d out of range", level);
    if (direction != 0 && direction != 1) fail(SEM_EINVAL, "sem_pmg_transfer: direction must be 0 or 1");
    hipStream_t s = (hipStream_t)stream;
    const MeshData& f = p->lv[level].mesh->d;
    const MeshData& c = p->lv[level + 1].mesh->d;
    const bool f32 = p->o.smoother_dtype == SEM_F32;
    const bool coarse_is_last = (level + 2 == p->n_levels);
    const int64_t nb = xfer_blocks(f.N, c.N, f.E);
    const double* M = direction == 0 ? p->lv[level].J.as<double>() : p->lv[level].JT.as<double>();
    auto gs_c = [&](auto* v) {
      using T = std::remove_pointer_t<decltype(v)>;
      Table<GsArgs<T>> t;
      t.one.v = v;
      t.one.off = c.gs_off.as<int>();
      t.one.idx = c.gs_idx.as<int>();
      t.one.sdir = c.gs_dir.as<uint8_t>();
      t.one.dir_idx = c.dir_idx.as<int>();
      t.one.n_shared = c.n_shared;
      t.one.n_dir = c.n_dir_single;
      t.one.mask = 1;
      launch_gs<T>(t, gs_blocks(c.n_shared, c.n_dir_single), s);
    };
    auto go = [&](auto tf, auto tc) {
      using Tf = decltype(tf);
      using Tc = decltype(tc);
      Table<XferArgs<Tf, Tc>> t;
      t.one.E = f.E;
      if (direction == 0) {
        t.one.zc = (const Tc*)in;
        t.one.xf = (Tf*)out;
      } else {
        t.one.rf = (const Tf*)in;
        t.one.owner_f = f.owner.as<uint8_t>();
        t.one.out_c = (Tc*)out;
      }
      launch_xfer<Tf, Tc>(direction, f.N, c.N, t, nb, M, s);
      if (direction == 1) gs_c((Tc*)out);
    };
    if (f32 && coarse_is_last) go(float{}, double{});
    else if (f32) go(float{}, float{});
    else go(double{}, double{});
  });
}
