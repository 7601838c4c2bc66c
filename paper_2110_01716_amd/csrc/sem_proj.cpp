// Projection onto prior solutions (Implementation, "Projection Is Key").
//
// The pressure evolves smoothly in time, so the solution for a new right-hand
// side is mostly a combination of earlier solutions. With an A-orthonormal
// basis P = [p_1 .. p_L] (and AP kept alongside), the best approximation of
// x = A^-1 b in the A-norm is xbar = P P^T b: one multi-dot of length L. The
// Krylov solver then only has to remove the residual b - A xbar = b - AP P^T b.
// The correction dx is A-orthogonalised against P by one round of classical
// Gram-Schmidt (coefficients beta_i = (p_i, A dx) from one multi-dot, norm
// from Pythagoras: |dx - P beta|_A^2 = (dx, A dx) - |beta|^2) and appended.
// With L_max vectors the space restarts from the newest solution alone.
//
// Storage: L_max + 1 slots for p and for Ap (FP64 E-vectors). The correction
// of a solve is computed directly in slot L (and A dx in Ap slot L), so the
// Gram-Schmidt multi-dot runs over the contiguous slots 0..L and the new basis
// vector is formed in place. The device arrays of slot pointers never change
// after creation. The few Gram-Schmidt scalars come back to the host once per
// solve.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "sem_internal.h"

struct sem_proj_s {
  sem_mesh m = nullptr;
  int Lmax = 0;
  int L = 0;
  int gmres_K = 0;                   // inner solver: 0 = CG family, K > 0 = flexible GMRES(K)
  std::vector<sem::DevBuf> P, AP;    // L_max + 1 slots each
  sem::DevBuf ptrP, ptrAP;           // device arrays of the slot pointers
  sem::DevBuf coef;                  // device: alpha [L_max+1], beta [L_max+1]
  sem::DevBuf partial;               // [L_max+1][stride]
  sem::DevBuf r;                     // projected residual, later A x at restart
  int64_t stride = 0;
  std::vector<double> hbeta;         // host copy of beta
};

namespace {

void multidot(sem_proj_s* pr, const sem::DevBuf& ptrs, int K, const double* y, double* out, hipStream_t s) {
  sem::mesh_multidot(pr->m->d, ptrs.as<const double*>(), K, y, pr->partial.as<double>(), pr->stride, out, s);
}

void lincomb(sem_proj_s* pr, const sem::DevBuf& ptrs, int K, const double* coef, const double* y, double a0,
             double sign, double scale, double* out, hipStream_t s) {
  sem::mesh_lincomb(pr->m->d, ptrs.as<const double*>(), K, coef, y, a0, sign, scale, out, s);
}

void vec1(sem::VecOp op, int64_t n, double* x, const double* r, double c0, hipStream_t s) {
  sem::vec_op1(op, n, x, r, c0, nullptr, s);
}

}  // namespace

using namespace sem;

extern "C" int sem_proj_create(sem_mesh m, int L_max, sem_proj* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!m || !out) fail(SEM_EINVAL, "sem_proj_create: NULL argument");
    if (L_max < 1 || L_max > 64) fail(SEM_EINVAL, "sem_proj_create: L_max=%d outside [1,64]", L_max);
    auto pr = std::make_unique<sem_proj_s>();
    pr->m = m;
    pr->Lmax = L_max;
    const int64_t n = m->d.nloc;
    pr->P.resize(L_max + 1);
    pr->AP.resize(L_max + 1);
    std::vector<const double*> hp, hap;
    for (int i = 0; i <= L_max; ++i) {
      pr->P[i].alloc(sizeof(double) * n);
      pr->AP[i].alloc(sizeof(double) * n);
      hp.push_back(pr->P[i].as<double>());
      hap.push_back(pr->AP[i].as<double>());
    }
    pr->ptrP.alloc(sizeof(double*) * (L_max + 1));
    pr->ptrAP.alloc(sizeof(double*) * (L_max + 1));
    SEM_HIP(hipMemcpy(pr->ptrP.p, hp.data(), sizeof(double*) * hp.size(), hipMemcpyHostToDevice));
    SEM_HIP(hipMemcpy(pr->ptrAP.p, hap.data(), sizeof(double*) * hap.size(), hipMemcpyHostToDevice));
    pr->coef.alloc(sizeof(double) * 2 * (L_max + 1));
    pr->stride = vec_blocks(n);
    pr->partial.alloc(sizeof(double) * pr->stride * (L_max + 1));
    pr->r.alloc(sizeof(double) * n);
    pr->hbeta.resize(L_max + 1);
    *out = pr.release();
  });
}

extern "C" int sem_proj_destroy(sem_proj pr) {
  return guarded([&] {
    if (pr) (void)hipDeviceSynchronize();
    delete pr;
  });
}

extern "C" int sem_proj_size(sem_proj pr, int* L) {
  return guarded([&] {
    if (!pr || !L) fail(SEM_EINVAL, "sem_proj_size: NULL argument");
    *L = pr->L;
  });
}

extern "C" int sem_proj_reset(sem_proj pr) {
  return guarded([&] {
    if (!pr) fail(SEM_EINVAL, "sem_proj_reset: NULL argument");
    pr->L = 0;
  });
}

extern "C" int sem_proj_set_gmres(sem_proj pr, int K) {
  return guarded([&] {
    if (!pr) fail(SEM_EINVAL, "sem_proj_set_gmres: NULL argument");
    if (K < 0 || K > 64) fail(SEM_EINVAL, "sem_proj_set_gmres: K=%d outside [0,64]", K);
    pr->gmres_K = K;
  });
}

extern "C" int sem_proj_export(sem_proj pr, int i, double* p, double* Ap, void* stream) {
  return guarded([&] {
    if (!pr) fail(SEM_EINVAL, "sem_proj_export: NULL argument");
    if (i < 0 || i >= pr->L) fail(SEM_EINVAL, "sem_proj_export: vector %d of %d", i, pr->L);
    const size_t bytes = sizeof(double) * pr->m->d.nloc;
    hipStream_t s = (hipStream_t)stream;
    if (p) SEM_HIP(hipMemcpyAsync(p, pr->P[i].p, bytes, hipMemcpyDeviceToDevice, s));
    if (Ap) SEM_HIP(hipMemcpyAsync(Ap, pr->AP[i].p, bytes, hipMemcpyDeviceToDevice, s));
  });
}

extern "C" int sem_pcg_solve_projected(sem_proj pr, sem_pmg pm, const double* b, double* x, const sem_solve_opts* oin,
                                       sem_solve_info* info, void* stream) {
  int rc = SEM_OK;
  const int g = guarded([&] {
    if (!pr || !b || !x) fail(SEM_EINVAL, "sem_pcg_solve_projected: NULL argument");
    if (pm && pm->base != pr->m) fail(SEM_EINVAL, "sem_pcg_solve_projected: pMG hierarchy of another mesh");
    hipStream_t s = (hipStream_t)stream;
    const MeshData& m = pr->m->d;
    const int64_t n = m.nloc;
    sem_solve_opts o;
    sem_solve_opts_default(&o);
    if (oin) o = *oin;
    if (o.lambda != 0.0) fail(SEM_EINVAL, "sem_pcg_solve_projected: Poisson solves only (lambda = 0)");
    const int L = pr->L;
    double* dx = pr->P[L].as<double>();   // the correction is built in slot L
    double* w = pr->AP[L].as<double>();
    double* alpha = pr->coef.as<double>();
    double* beta = alpha + pr->Lmax + 1;
    double* r = pr->r.as<double>();
    const double bb = mesh_dot_ws(m, b, b, pr->partial.as<double>(), s);
    // starting guess xbar = P (P^T b), residual r = b - AP (P^T b)
    if (L > 0) {
      multidot(pr, pr->ptrP, L, b, alpha, s);
      lincomb(pr, pr->ptrP, L, alpha, nullptr, 0.0, 1.0, 1.0, x, s);
      lincomb(pr, pr->ptrAP, L, alpha, b, 1.0, -1.0, 1.0, r, s);
    } else {
      SEM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
      SEM_HIP(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    const double rr = mesh_dot_ws(m, r, r, pr->partial.as<double>(), s);
    const double rel0 = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    sem_solve_info inner{};
    bool solved = false;
    if (!std::isfinite(bb) || !std::isfinite(rr)) {
      rc = SEM_ENAN;
      inner.status = SEM_ENAN;
      set_error("sem_pcg_solve_projected: NaN or Inf in the right-hand side or the space");
    } else if (bb == 0.0 || rel0 <= o.rtol) {
      inner.status = SEM_OK;
      inner.relres = rel0;
      inner.relres_true = rel0;
    } else {
      sem_solve_opts oi = o;
      oi.rtol = o.rtol / rel0;  // |r - A dx| <= rtol |b|
      rc = pr->gmres_K > 0 ? sem_gmres_solve(pr->m, pm, pr->gmres_K, r, dx, &oi, &inner, stream)
                           : sem_pcg_solve(pr->m, pm, r, dx, &oi, &inner, stream);
      inner.relres *= rel0;
      inner.relres_true *= rel0;
      solved = true;
      vec1(V_AXPY, n, x, dx, 1.0, s);  // x = xbar + dx
    }
    // augment the space with dx, A-orthogonalised against P (one multi-dot)
    if (solved && inner.status == SEM_OK) {
      apply_A(m, SEM_F64, dx, w, s);
      multidot(pr, pr->ptrP, L + 1, w, beta, s);  // beta_i = (p_i, A dx), beta_L = (dx, A dx)
      std::vector<double>& hb = pr->hbeta;
      SEM_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * (L + 1), hipMemcpyDeviceToHost, s));
      SEM_HIP(hipStreamSynchronize(s));
      const double dAd = hb[L];
      double g2 = dAd;
      for (int i = 0; i < L; ++i) g2 -= hb[i] * hb[i];
      if (L == pr->Lmax) {
        // restart from the newest solution alone: A x = (b - r) + A dx
        vec1(V_SCALE, n, r, r, -1.0, s);
        vec1(V_AXPY, n, r, b, 1.0, s);
        vec1(V_AXPY, n, r, w, 1.0, s);
        const double xAx = mesh_dot_ws(m, x, r, pr->partial.as<double>(), s);
        if (xAx > 0 && std::isfinite(xAx)) {
          const double inv = 1.0 / std::sqrt(xAx);
          vec1(V_SCALE, n, pr->P[0].as<double>(), x, inv, s);
          vec1(V_SCALE, n, pr->AP[0].as<double>(), r, inv, s);
          pr->L = 1;
        } else {
          pr->L = 0;
        }
      } else if (dAd > 0 && std::isfinite(g2) && g2 > 1e-12 * dAd) {
        // p_L = (dx - P beta) / gamma, in place; likewise Ap_L
        const double inv = 1.0 / std::sqrt(g2);
        lincomb(pr, pr->ptrP, L, beta, dx, 1.0, -1.0, inv, dx, s);
        lincomb(pr, pr->ptrAP, L, beta, w, 1.0, -1.0, inv, w, s);
        pr->L = L + 1;
      }
    }
    SEM_HIP(hipStreamSynchronize(s));
    if (info) {
      *info = inner;
      info->relres_initial = rel0;
    }
  });
  return g != SEM_OK ? g : rc;
}
