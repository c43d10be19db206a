// Native ADAPT-VQE driver (paper, "Numerical performance": grow the ansatz
// one pool operator at a time, choosing the operator with the largest energy
// gradient, then re-optimise every parameter; "General Framework for
// Variational Algorithms": E(theta) = <psi_0|U(theta)^T H U(theta)|psi_0>).
//
// One energy+gradient evaluation of the inner optimiser is
//   phi = |HF>, phi <- U_j..U_1 phi            (j rotations, theta on device)
//   [FP32 storage: phi <- phi / ||phi||]
//   lam = H phi, E = <phi|lam>
//   for i = j..1:  dE/dtheta_i = 2 <lam|A_i phi>, phi <- U_i^T phi, lam <- U_i^T lam
// (the adjoint recursion: 1 H psi + 3j pair passes), captured once per ADAPT
// iteration into a hipGraph and replayed for every BFGS evaluation.  The
// host only exchanges E and the j gradient entries with the device.
#include "hyp_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace hyp {

__global__ void k_fill_hf_f64(double* v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (i == 0) ? 1.0 : 0.0;  // the HF determinant has sector index 0
}
__global__ void k_fill_hf_f32(float* v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (i == 0) ? 1.0f : 0.0f;
}
template <typename T>
__global__ void k_scale_inv_sqrt(T* v, int64_t n, const double* nrm2) {
  const double s = 1.0 / sqrt(*nrm2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (T)((double)v[i] * s);
}
template <typename T>
__global__ void k_copy(const T* a, T* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

static unsigned grid_for(int64_t n) {
  return (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
}

hyp_status fill_hf(Sector* S, hyp_dtype dt, void* v, hipStream_t st) {
  unsigned g = (unsigned)((S->dim + 255) / 256);
  if (dt == HYP_F64)
    HYP_LAUNCH("k_fill_hf", k_fill_hf_f64, dim3(g), dim3(256), 0, st, (double*)v, S->dim);
  else
    HYP_LAUNCH("k_fill_hf", k_fill_hf_f32, dim3(g), dim3(256), 0, st, (float*)v, S->dim);
  return HYP_OK;
}

hyp_status renormalise(Sector* S, hyp_dtype dt, void* v, double* nrm2, hipStream_t st) {
  hyp_status r = launch_dot(S, dt, v, v, nrm2, st);
  if (r != HYP_OK) return r;
  if (dt == HYP_F64)
    HYP_LAUNCH("k_scale", k_scale_inv_sqrt<double>, dim3(grid_for(S->dim)), dim3(256), 0, st,
               (double*)v, S->dim, nrm2);
  else
    HYP_LAUNCH("k_scale", k_scale_inv_sqrt<float>, dim3(grid_for(S->dim)), dim3(256), 0, st,
               (float*)v, S->dim, nrm2);
  return HYP_OK;
}

hyp_status copy_vec(Sector* S, hyp_dtype dt, const void* a, void* b, hipStream_t st) {
  if (dt == HYP_F64)
    HYP_LAUNCH("k_copy", k_copy<double>, dim3(grid_for(S->dim)), dim3(256), 0, st, (const double*)a,
               (double*)b, S->dim);
  else
    HYP_LAUNCH("k_copy", k_copy<float>, dim3(grid_for(S->dim)), dim3(256), 0, st, (const float*)a,
               (float*)b, S->dim);
  return HYP_OK;
}

struct Adapt {
  hyp_ham ham = nullptr;
  Sector* S = nullptr;
  hyp_dtype dt = HYP_F64;
  hyp_adapt_opts o{};
  std::vector<hyp_exc> pool;
  hyp_exc* d_pool = nullptr;
  hyp_exc* d_sub = nullptr;        // candidate subset (screened iterations)
  size_t esz = 8;
  void *psi = nullptr, *sig = nullptr, *phi = nullptr, *lam = nullptr;
  double* d_theta = nullptr;       // [max_iter]
  double* d_grad = nullptr;        // [max_iter]
  double* d_scal = nullptr;        // [0] E, [1] norm^2
  double* d_part = nullptr;        // [max_iter][max_rot_chunks]
  double* d_pgrad = nullptr;       // [n_pool]
  double* h_pin = nullptr;         // pinned: [0] E, [1..] gradient / theta staging
  hipStream_t st = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_j = -1;
  std::vector<int32_t> ops;
  std::vector<double> theta;
  std::vector<double> last_grad;   // pool gradient of the last iteration (NaN = not computed)
  int n_evals = 0;
  // inverse-Hessian estimate left by the last optimisation (n_rec x n_rec),
  // the start of the next one when the ansatz has grown by one parameter
  std::vector<double> h_rec;
  size_t n_rec = 0;
};

static hyp_status enqueue_eval(Adapt* A, int j) {
  Sector* S = A->S;
  hipStream_t st = A->st;
  hyp_status r = fill_hf(S, A->dt, A->phi, st);
  if (r != HYP_OK) return r;
  for (int i = 0; i < j; ++i) {
    r = launch_rotate(S, A->dt, A->pool[A->ops[i]], 0.0, A->d_theta + i, A->phi, st);
    if (r != HYP_OK) return r;
  }
  if (A->dt == HYP_F32) {
    r = renormalise(S, A->dt, A->phi, A->d_scal + 1, st);
    if (r != HYP_OK) return r;
  }
  r = apply_h_internal(A->ham, A->dt, A->phi, A->lam, st);
  if (r != HYP_OK) return r;
  r = launch_dot(S, A->dt, A->phi, A->lam, A->d_scal, st);
  if (r != HYP_OK) return r;
  const int nch = max_rot_chunks();
  for (int i = j - 1; i >= 0; --i) {
    r = launch_adjoint_step(S, A->dt, A->pool[A->ops[i]], A->d_theta + i, A->phi, A->lam,
                            A->d_part + (size_t)i * nch, A->d_grad + i, st);
    if (r != HYP_OK) return r;
  }
  return HYP_OK;
}

static void drop_graph(Adapt* A) {
  if (A->exec) (void)hipGraphExecDestroy(A->exec);
  if (A->graph) (void)hipGraphDestroy(A->graph);
  A->exec = nullptr;
  A->graph = nullptr;
  A->graph_j = -1;
}

// E(theta) and dE/dtheta (host), one replay of the captured evaluation.
static hyp_status evaluate(Adapt* A, const double* th, double* E, double* g) {
  const int j = (int)A->ops.size();
  std::memcpy(A->h_pin + 1, th, sizeof(double) * j);
  if (j) HYP_HIP(hipMemcpyAsync(A->d_theta, A->h_pin + 1, sizeof(double) * j, hipMemcpyHostToDevice, A->st));
  if (A->o.use_graph) {
    if (A->graph_j != j) {
      drop_graph(A);
      HYP_HIP(hipStreamBeginCapture(A->st, hipStreamCaptureModeThreadLocal));
      hyp_status r = enqueue_eval(A, j);
      hipGraph_t gph = nullptr;
      hipError_t e = hipStreamEndCapture(A->st, &gph);
      if (r != HYP_OK) {
        if (gph) (void)hipGraphDestroy(gph);
        return r;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      A->graph = gph;
      HYP_HIP(hipGraphInstantiate(&A->exec, A->graph, nullptr, nullptr, 0));
      A->graph_j = j;
    }
    HYP_HIP(hipGraphLaunch(A->exec, A->st));
  } else {
    hyp_status r = enqueue_eval(A, j);
    if (r != HYP_OK) return r;
  }
  HYP_HIP(hipMemcpyAsync(A->h_pin, A->d_scal, sizeof(double), hipMemcpyDeviceToHost, A->st));
  if (j) HYP_HIP(hipMemcpyAsync(A->h_pin + 1, A->d_grad, sizeof(double) * j, hipMemcpyDeviceToHost, A->st));
  HYP_HIP(hipStreamSynchronize(A->st));
  *E = A->h_pin[0];
  std::memcpy(g, A->h_pin + 1, sizeof(double) * j);
  A->n_evals++;
  return HYP_OK;
}

// ---------------------------------------------------------------- BFGS

static double dotv(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}
static double infnorm(const std::vector<double>& a) {
  double m = 0.0;
  for (double v : a) m = std::max(m, std::fabs(v));
  return m;
}

struct LineResult {
  bool ok;
  double alpha, f;
  std::vector<double> g;
};

// Energy noise of the evaluation: FP32 storage rounds the state and every
// product to FP32 (relative error about 1e-7 of E, measured), so sufficient
// decrease is tested against that floor, the zoom is capped and steps that
// gain less than it count as stalls.
static double energy_noise(const Adapt* A, double f) {
  return A->dt == HYP_F32 ? 2e-7 * std::fabs(f) : 0.0;
}

// Slack of the sufficient-decrease test: the FP32 noise above, and in FP64
// the rounding floor of the energy (a dot product over dim terms of sigma,
// itself a sum of thousands of products per amplitude, about 1e-14 of E).
// Near a minimum the decrease a step can make, |g|^2 / (2 lambda), falls
// below that floor while the adjoint gradient is still exact to about 1e-14,
// so the search relies on the curvature test there (the approximate Wolfe
// conditions of Hager and Zhang, 2005).
static double armijo_slack(const Adapt* A, double f) {
  return A->dt == HYP_F32 ? energy_noise(A, f) : 1e-14 * std::fabs(f);
}

// Strong-Wolfe line search (bracketing + zoom with safeguarded cubic
// interpolation), c1 = 1e-4, c2 = 0.9; the sufficient-decrease test is
// relaxed by the energy's rounding or noise floor (armijo_slack); with noisy
// (FP32) energies the zoom is capped, the best decreasing point being
// accepted when the curvature test never holds.
static hyp_status wolfe(Adapt* A, const std::vector<double>& x, double f0,
                        const std::vector<double>& g0, const std::vector<double>& p,
                        LineResult* out) {
  const double c1 = 1e-4, c2 = 0.9;
  const double eps = armijo_slack(A, f0);
  const int max_zoom = energy_noise(A, f0) > 0.0 ? 10 : 40;
  const size_t n = x.size();
  const double d0 = dotv(g0, p);
  std::vector<double> xt(n), gt(n);
  auto phi = [&](double a, double* f, double* d) -> hyp_status {
    for (size_t i = 0; i < n; ++i) xt[i] = x[i] + a * p[i];
    hyp_status r = evaluate(A, xt.data(), f, gt.data());
    *d = dotv(gt, p);
    return r;
  };
  double a_prev = 0.0, f_prev = f0, d_prev = d0;
  double a = 1.0;
  out->ok = false;
  for (int it = 0; it < 30; ++it) {
    double f, d;
    hyp_status r = phi(a, &f, &d);
    if (r != HYP_OK) return r;
    bool lo_is_prev = true;
    double alo, ahi, flo, fhi, dlo, dhi;
    if (f > f0 + c1 * a * d0 + eps || (it > 0 && f >= f_prev)) {
      alo = a_prev; flo = f_prev; dlo = d_prev; ahi = a; fhi = f; dhi = d;
    } else if (std::fabs(d) <= -c2 * d0) {
      out->ok = true; out->alpha = a; out->f = f; out->g = gt;
      return HYP_OK;
    } else if (d >= 0) {
      alo = a; flo = f; dlo = d; ahi = a_prev; fhi = f_prev; dhi = d_prev;
      lo_is_prev = false;
    } else {
      a_prev = a; f_prev = f; d_prev = d;
      a = std::min(2.0 * a, 1e6);
      continue;
    }
    (void)lo_is_prev;
    // zoom
    for (int z = 0; z < max_zoom; ++z) {
      // cubic interpolation between (alo, flo, dlo) and (ahi, fhi, dhi)
      double aj;
      {
        double d1 = dlo + dhi - 3.0 * (flo - fhi) / (alo - ahi);
        double disc = d1 * d1 - dlo * dhi;
        double lo = std::min(alo, ahi), hi = std::max(alo, ahi);
        if (disc >= 0.0) {
          double d2 = std::copysign(std::sqrt(disc), ahi - alo);
          aj = ahi - (ahi - alo) * (dhi + d2 - d1) / (dhi - dlo + 2.0 * d2);
        } else {
          aj = 0.5 * (alo + ahi);
        }
        double w = hi - lo;
        if (!(aj > lo + 0.1 * w && aj < hi - 0.1 * w)) aj = 0.5 * (alo + ahi);
      }
      double fj, dj;
      hyp_status r2 = phi(aj, &fj, &dj);
      if (r2 != HYP_OK) return r2;
      if (fj > f0 + c1 * aj * d0 + eps || fj >= flo) {
        ahi = aj; fhi = fj; dhi = dj;
      } else {
        if (std::fabs(dj) <= -c2 * d0) {
          out->ok = true; out->alpha = aj; out->f = fj; out->g = gt;
          return HYP_OK;
        }
        if (dj * (ahi - alo) >= 0) {
          ahi = alo; fhi = flo; dhi = dlo;
        }
        alo = aj; flo = fj; dlo = dj;
      }
      if (std::fabs(ahi - alo) < 1e-14 * std::max(1.0, std::fabs(alo))) break;
    }
    // accept the best sufficient-decrease point if the curvature test never held
    if (alo > 0.0 && (flo < f0 + c1 * alo * d0 || (eps > 0.0 && flo < f0))) {
      double ff, dd;
      hyp_status r3 = phi(alo, &ff, &dd);
      if (r3 != HYP_OK) return r3;
      out->ok = true; out->alpha = alo; out->f = ff; out->g = gt;
    }
    return HYP_OK;
  }
  return HYP_OK;
}

static hyp_status bfgs(Adapt* A, std::vector<double>& x, double* fout, int* iters, int* conv,
                       double* ginf) {
  const size_t n = x.size();
  std::vector<double> g(n), p(n), s(n), y(n), Hy(n);
  double f;
  hyp_status r = evaluate(A, x.data(), &f, g.data());
  if (r != HYP_OK) return r;
  std::vector<double> Hi(n * n, 0.0);
  for (size_t i = 0; i < n; ++i) Hi[i * n + i] = 1.0;
  if (A->o.recycle_hessian && n > 1 && A->n_rec + 1 == n && A->h_rec.size() == A->n_rec * A->n_rec) {
    // the previous optimisation's estimate for the old parameters, identity
    // for the appended one (the old parameters keep their order)
    for (size_t i = 0; i + 1 < n; ++i)
      for (size_t k = 0; k + 1 < n; ++k) Hi[i * n + k] = A->h_rec[i * (n - 1) + k];
  }
  int it = 0, stall = 0;
  *conv = 0;
  for (; it < A->o.max_bfgs; ++it) {
    if (infnorm(g) <= A->o.gtol) {
      *conv = 1;
      break;
    }
    for (size_t i = 0; i < n; ++i) {
      double v = 0.0;
      for (size_t k = 0; k < n; ++k) v += Hi[i * n + k] * g[k];
      p[i] = -v;
    }
    if (dotv(p, g) >= 0.0) {  // not a descent direction: restart from steepest descent
      for (size_t i = 0; i < n; ++i) {
        p[i] = -g[i];
        for (size_t k = 0; k < n; ++k) Hi[i * n + k] = (i == k);
      }
    }
    LineResult lr;
    r = wolfe(A, x, f, g, p, &lr);
    if (r != HYP_OK) return r;
    if (!lr.ok) break;
    for (size_t i = 0; i < n; ++i) {
      s[i] = lr.alpha * p[i];
      y[i] = lr.g[i] - g[i];
      x[i] += s[i];
    }
    const double fprev = f;
    f = lr.f;
    g = lr.g;
    const double ys = dotv(y, s);
    if (ys > 1e-300) {
      // H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T
      const double rho = 1.0 / ys;
      for (size_t i = 0; i < n; ++i) {
        double v = 0.0;
        for (size_t k = 0; k < n; ++k) v += Hi[i * n + k] * y[k];
        Hy[i] = v;
      }
      const double yHy = dotv(y, Hy);
      for (size_t i = 0; i < n; ++i)
        for (size_t k = 0; k < n; ++k)
          Hi[i * n + k] += -rho * (Hy[i] * s[k] + s[i] * Hy[k]) + (rho * rho * yHy + rho) * s[i] * s[k];
    }
    if (std::fabs(fprev - f) <= 1e-16 * std::max(1.0, std::fabs(f)) && infnorm(g) <= 10 * A->o.gtol) {
      *conv = 1;
      ++it;
      break;
    }
    // noisy energies: three steps in a row that gain less than the noise
    // floor end the optimisation
    const double eps = energy_noise(A, f);
    stall = (eps > 0.0 && fprev - f <= eps) ? stall + 1 : 0;
    if (stall >= 3) {
      ++it;
      break;
    }
  }
  *fout = f;
  *iters = it;
  *ginf = infnorm(g);
  A->h_rec = Hi;
  A->n_rec = n;
  // converged: the gradient test held, the energy stopped changing with the
  // gradient within 10 gtol (*conv set in the loop), or the optimisation
  // ended at a point whose gradient is at the precision floor (100 gtol)
  *conv = (*ginf <= A->o.gtol || *conv == 1 || *ginf <= 100.0 * A->o.gtol) ? 1 : 0;
  return HYP_OK;
}

// state, sigma and energy of the current ansatz into psi / sig (on A->st)
static hyp_status prepare_state(Adapt* A) {
  const int j = (int)A->ops.size();
  if (j) {
    std::memcpy(A->h_pin + 1, A->theta.data(), sizeof(double) * j);
    HYP_HIP(hipMemcpyAsync(A->d_theta, A->h_pin + 1, sizeof(double) * j, hipMemcpyHostToDevice, A->st));
  }
  hyp_status r = fill_hf(A->S, A->dt, A->psi, A->st);
  for (int i = 0; i < j && r == HYP_OK; ++i)
    r = launch_rotate(A->S, A->dt, A->pool[A->ops[i]], 0.0, A->d_theta + i, A->psi, A->st);
  if (r == HYP_OK && A->dt == HYP_F32) r = renormalise(A->S, A->dt, A->psi, A->d_scal + 1, A->st);
  if (r == HYP_OK) r = apply_h_internal(A->ham, A->dt, A->psi, A->sig, A->st);
  if (r == HYP_OK) r = launch_dot(A->S, A->dt, A->psi, A->sig, A->d_scal, A->st);
  return r;
}

}  // namespace hyp

using namespace hyp;

struct hyp_adapt_s {
  Adapt a;
};

extern "C" {

hyp_status hyp_adapt_destroy(hyp_adapt h) {
  if (!h) return HYP_OK;
  Adapt& A = h->a;
  if (A.st) (void)hipStreamSynchronize(A.st);
  drop_graph(&A);
  (void)hipFree(A.d_pool);
  (void)hipFree(A.d_sub);
  (void)hipFree(A.psi);
  (void)hipFree(A.sig);
  (void)hipFree(A.phi);
  (void)hipFree(A.lam);
  (void)hipFree(A.d_theta);
  (void)hipFree(A.d_grad);
  (void)hipFree(A.d_scal);
  (void)hipFree(A.d_part);
  (void)hipFree(A.d_pgrad);
  if (A.h_pin) (void)hipHostFree(A.h_pin);
  if (A.st) (void)hipStreamDestroy(A.st);
  delete h;
  return HYP_OK;
}

hyp_status hyp_adapt_create(hyp_ham ham, hyp_dtype dtype, const hyp_exc* pool, int64_t n_pool,
                            const hyp_adapt_opts* opts, hyp_adapt* out) {
  Ham* H = ham_of(ham);
  if (!H || !pool || !opts || !out) return fail(HYP_ERR_ARG, "hyp_adapt_create: NULL argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_adapt_create: bad dtype");
  if (n_pool < 1 || n_pool > (1 << 24)) return fail(HYP_ERR_ARG, "hyp_adapt_create: n_pool out of range");
  if (opts->max_iter < 1 || opts->max_iter > 4096 || opts->max_bfgs < 0 || !(opts->gtol > 0) ||
      !(opts->tie_tol >= 0) || opts->tie_tol >= 1 || (opts->recycle_hessian != 0 && opts->recycle_hessian != 1))
    return fail(HYP_ERR_ARG, "hyp_adapt_create: bad options");
  Sector* S = H->sec;
  for (int64_t k = 0; k < n_pool; ++k) {
    hyp_status r = validate_exc(S, pool[k]);
    if (r != HYP_OK) return r;
  }
  hyp_status rb = ensure_binom();
  if (rb != HYP_OK) return rb;
  hyp_adapt_s* h = new (std::nothrow) hyp_adapt_s();
  if (!h) return fail(HYP_ERR_NOMEM, "hyp_adapt_create: host allocation");
  Adapt& A = h->a;
  A.ham = ham;
  A.S = S;
  A.dt = dtype;
  A.o = *opts;
  A.pool.assign(pool, pool + n_pool);
  A.esz = dtype == HYP_F64 ? 8 : 4;
  A.last_grad.assign((size_t)n_pool, NAN);
  const size_t vb = (size_t)S->dim * A.esz;
  hipError_t e = hipStreamCreateWithFlags(&A.st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&A.d_pool, sizeof(hyp_exc) * n_pool);
  if (e == hipSuccess) e = hipMalloc(&A.d_sub, sizeof(hyp_exc) * n_pool);
  if (e == hipSuccess) e = hipMalloc(&A.psi, vb);
  if (e == hipSuccess) e = hipMalloc(&A.sig, vb);
  if (e == hipSuccess) e = hipMalloc(&A.phi, vb);
  if (e == hipSuccess) e = hipMalloc(&A.lam, vb);
  if (e == hipSuccess) e = hipMalloc(&A.d_theta, sizeof(double) * opts->max_iter);
  if (e == hipSuccess) e = hipMalloc(&A.d_grad, sizeof(double) * opts->max_iter);
  if (e == hipSuccess) e = hipMalloc(&A.d_scal, sizeof(double) * 4);
  if (e == hipSuccess) e = hipMalloc(&A.d_part, sizeof(double) * opts->max_iter * (size_t)max_rot_chunks());
  if (e == hipSuccess) e = hipMalloc(&A.d_pgrad, sizeof(double) * n_pool);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&A.h_pin, sizeof(double) * (2 + std::max<int64_t>(opts->max_iter, n_pool)), 0);
  if (e == hipSuccess)
    e = hipMemcpy(A.d_pool, pool, sizeof(hyp_exc) * n_pool, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hyp_adapt_destroy(h);
    return hip_fail(e, "hyp_adapt_create: allocation");
  }
  // the pool-gradient partial buffer must exist before any graph capture
  double* dummy;
  hyp_status r = pair_scratch(S, (size_t)n_pool * 16, &dummy);
  if (r != HYP_OK) {
    hyp_adapt_destroy(h);
    return r;
  }
  *out = h;
  return HYP_OK;
}

// Exact pool gradients of the current state.  cand == NULL: the whole pool;
// otherwise only the n_cand pool indices in cand (host array).  Stores them
// (NaN elsewhere) for the selection and fills energy_before, gmax, grad_ms.
hyp_status hyp_adapt_gradients(hyp_adapt h, const int32_t* cand, int64_t n_cand, hyp_adapt_record* rec) {
  if (!h || !rec) return fail(HYP_ERR_ARG, "hyp_adapt_gradients: NULL argument");
  Adapt& A = h->a;
  const int64_t np = (int64_t)A.pool.size();
  if (cand && (n_cand < 1 || n_cand > np)) return fail(HYP_ERR_ARG, "hyp_adapt_gradients: bad candidate count");
  if (cand)
    for (int64_t i = 0; i < n_cand; ++i)
      if (cand[i] < 0 || cand[i] >= np) return fail(HYP_ERR_ARG, "hyp_adapt_gradients: candidate index out of range");
  std::memset(rec, 0, sizeof(*rec));
  auto t0 = std::chrono::steady_clock::now();
  hyp_status r = prepare_state(&A);
  if (r != HYP_OK) return r;
  const int64_t ng = cand ? n_cand : np;
  if (cand) {
    std::vector<hyp_exc> sub((size_t)n_cand);
    for (int64_t i = 0; i < n_cand; ++i) sub[(size_t)i] = A.pool[(size_t)cand[i]];
    HYP_HIP(hipMemcpyAsync(A.d_sub, sub.data(), sizeof(hyp_exc) * n_cand, hipMemcpyHostToDevice, A.st));
    HYP_HIP(hipStreamSynchronize(A.st));  // sub is a host temporary
    r = launch_pool_gradients(A.S, A.dt, A.d_sub, n_cand, A.psi, A.sig, A.d_pgrad, A.st);
  } else {
    r = launch_pool_gradients(A.S, A.dt, A.d_pool, np, A.psi, A.sig, A.d_pgrad, A.st);
  }
  if (r != HYP_OK) return r;
  HYP_HIP(hipMemcpyAsync(A.h_pin + 1, A.d_pgrad, sizeof(double) * ng, hipMemcpyDeviceToHost, A.st));
  HYP_HIP(hipMemcpyAsync(A.h_pin, A.d_scal, sizeof(double), hipMemcpyDeviceToHost, A.st));
  HYP_HIP(hipStreamSynchronize(A.st));
  rec->energy_before = A.h_pin[0];
  std::fill(A.last_grad.begin(), A.last_grad.end(), NAN);
  double gmax = 0.0;
  for (int64_t i = 0; i < ng; ++i) {
    const int64_t k = cand ? cand[i] : i;
    A.last_grad[(size_t)k] = A.h_pin[1 + i];
    gmax = std::max(gmax, std::fabs(A.h_pin[1 + i]));
  }
  rec->gmax = gmax;
  rec->grad_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HYP_OK;
}

// Selection over the stored gradients (tie rule: lowest pool index among
// |g| >= max|g| (1 - tie_tol)), then BFGS over all parameters.  Keeps the
// gradient fields of rec; selected = -1 (nothing appended) if max|g| <
// gmax_stop.
hyp_status hyp_adapt_select_optimize(hyp_adapt h, hyp_adapt_record* rec) {
  if (!h || !rec) return fail(HYP_ERR_ARG, "hyp_adapt_select_optimize: NULL argument");
  Adapt& A = h->a;
  const int64_t np = (int64_t)A.pool.size();
  if ((int)A.ops.size() >= A.o.max_iter) return fail(HYP_ERR_ARG, "hyp_adapt_select_optimize: ansatz at max_iter");
  double gmax = 0.0;
  for (int64_t k = 0; k < np; ++k)
    if (!std::isnan(A.last_grad[(size_t)k])) gmax = std::max(gmax, std::fabs(A.last_grad[(size_t)k]));
  rec->gmax = gmax;
  if (gmax < A.o.gmax_stop) {
    rec->selected = -1;
    rec->energy = rec->energy_before;
    return HYP_OK;
  }
  int32_t best = -1, ties = 0;
  for (int64_t k = 0; k < np; ++k) {
    const double v = A.last_grad[(size_t)k];
    if (std::isnan(v)) continue;
    if (std::fabs(v) >= gmax * (1.0 - A.o.tie_tol)) {
      ++ties;
      if (best < 0) best = (int32_t)k;
    }
  }
  rec->selected = best;
  rec->tie_count = ties;
  auto t1 = std::chrono::steady_clock::now();
  A.ops.push_back(best);
  A.theta.push_back(0.0);
  A.n_evals = 0;
  double f = 0.0;
  int iters = 0, conv = 0;
  double ginf = 0.0;
  std::vector<double> x = A.theta;
  hyp_status r = bfgs(&A, x, &f, &iters, &conv, &ginf);
  if (r != HYP_OK) {
    A.ops.pop_back();
    A.theta.pop_back();
    drop_graph(&A);
    return r;
  }
  A.theta = x;
  rec->energy = f;
  rec->n_evals = A.n_evals;
  rec->bfgs_iters = iters;
  rec->converged = conv;
  rec->grad_inf = ginf;
  rec->opt_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  return HYP_OK;
}

// One ADAPT iteration: gradients (cand as in hyp_adapt_gradients), then
// selection and optimisation.
hyp_status hyp_adapt_iterate(hyp_adapt h, const int32_t* cand, int64_t n_cand, hyp_adapt_record* rec) {
  if (h && (int)h->a.ops.size() >= h->a.o.max_iter)
    return fail(HYP_ERR_ARG, "hyp_adapt_iterate: ansatz at max_iter");
  hyp_status r = hyp_adapt_gradients(h, cand, n_cand, rec);
  if (r != HYP_OK) return r;
  return hyp_adapt_select_optimize(h, rec);
}

hyp_status hyp_adapt_optimize(hyp_adapt h, hyp_adapt_record* rec) {
  if (!h || !rec) return fail(HYP_ERR_ARG, "hyp_adapt_optimize: NULL argument");
  Adapt& A = h->a;
  std::memset(rec, 0, sizeof(*rec));
  rec->selected = -1;
  auto t1 = std::chrono::steady_clock::now();
  if (A.ops.empty()) {
    hyp_status r = prepare_state(&A);
    if (r != HYP_OK) return r;
    HYP_HIP(hipMemcpyAsync(A.h_pin, A.d_scal, sizeof(double), hipMemcpyDeviceToHost, A.st));
    HYP_HIP(hipStreamSynchronize(A.st));
    rec->energy = rec->energy_before = A.h_pin[0];
    rec->converged = 1;
    return HYP_OK;
  }
  A.n_evals = 0;
  std::vector<double> x = A.theta;
  std::vector<double> g0(x.size());
  double f0 = 0.0;
  hyp_status r = evaluate(&A, x.data(), &f0, g0.data());
  if (r != HYP_OK) return r;
  rec->energy_before = f0;
  double f = 0.0, ginf = 0.0;
  int iters = 0, conv = 0;
  r = bfgs(&A, x, &f, &iters, &conv, &ginf);
  if (r != HYP_OK) return r;
  A.theta = x;
  rec->energy = f;
  rec->n_evals = A.n_evals;
  rec->bfgs_iters = iters;
  rec->converged = conv;
  rec->grad_inf = ginf;
  rec->opt_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  return HYP_OK;
}

hyp_status hyp_adapt_last_gradients(hyp_adapt h, double* out, int64_t n) {
  if (!h || !out) return fail(HYP_ERR_ARG, "hyp_adapt_last_gradients: NULL argument");
  Adapt& A = h->a;
  if (n != (int64_t)A.pool.size()) return fail(HYP_ERR_ARG, "hyp_adapt_last_gradients: n != pool size");
  std::memcpy(out, A.last_grad.data(), sizeof(double) * n);
  return HYP_OK;
}

hyp_status hyp_adapt_ansatz(hyp_adapt h, int32_t* ops, double* theta, int64_t cap, int64_t* n) {
  if (!h || !n) return fail(HYP_ERR_ARG, "hyp_adapt_ansatz: NULL argument");
  Adapt& A = h->a;
  *n = (int64_t)A.ops.size();
  if (cap < *n) return HYP_OK;  // size query
  if (*n && (!ops || !theta)) return fail(HYP_ERR_ARG, "hyp_adapt_ansatz: NULL output");
  for (int64_t i = 0; i < *n; ++i) {
    ops[i] = A.ops[(size_t)i];
    theta[i] = A.theta[(size_t)i];
  }
  return HYP_OK;
}

hyp_status hyp_adapt_set_ansatz(hyp_adapt h, const int32_t* ops, const double* theta, int64_t n) {
  if (!h || (n && (!ops || !theta))) return fail(HYP_ERR_ARG, "hyp_adapt_set_ansatz: NULL argument");
  Adapt& A = h->a;
  if (n < 0 || n > A.o.max_iter) return fail(HYP_ERR_ARG, "hyp_adapt_set_ansatz: length out of range");
  for (int64_t i = 0; i < n; ++i)
    if (ops[i] < 0 || ops[i] >= (int64_t)A.pool.size() || !std::isfinite(theta[i]))
      return fail(HYP_ERR_ARG, "hyp_adapt_set_ansatz: bad entry");
  A.ops.assign(ops, ops + n);
  A.theta.assign(theta, theta + n);
  A.h_rec.clear();
  A.n_rec = 0;
  drop_graph(&A);
  return HYP_OK;
}

hyp_status hyp_adapt_eval(hyp_adapt h, const double* theta, double* e, double* grad) {
  if (!h || !e || (!h->a.ops.empty() && (!theta || !grad)))
    return fail(HYP_ERR_ARG, "hyp_adapt_eval: NULL argument");
  std::vector<double> g(h->a.ops.size());
  hyp_status r = evaluate(&h->a, theta, e, g.data());
  if (r == HYP_OK && grad) std::memcpy(grad, g.data(), sizeof(double) * g.size());
  return r;
}

// Current state U(theta)|HF> (the adapt dtype) into psi_dev; waits for completion.
hyp_status hyp_adapt_state(hyp_adapt h, void* psi_dev) {
  if (!h || !psi_dev) return fail(HYP_ERR_ARG, "hyp_adapt_state: NULL argument");
  Adapt& A = h->a;
  hyp_status r = prepare_state(&A);
  if (r == HYP_OK) r = copy_vec(A.S, A.dt, A.psi, psi_dev, A.st);
  if (r == HYP_OK) HYP_HIP(hipStreamSynchronize(A.st));
  return r;
}

// Energy of the current ansatz replayed entirely in FP64 (state prep, H psi,
// <psi|H psi> / <psi|psi>), whatever the adapt's storage type.
hyp_status hyp_adapt_energy_fp64(hyp_adapt h, double* e) {
  if (!h || !e) return fail(HYP_ERR_ARG, "hyp_adapt_energy_fp64: NULL argument");
  Adapt& A = h->a;
  Sector* S = A.S;
  void *p = nullptr, *s = nullptr;
  double* d = nullptr;
  hipError_t he = hipMalloc(&p, S->dim * 8);
  if (he == hipSuccess) he = hipMalloc(&s, S->dim * 8);
  if (he == hipSuccess) he = hipMalloc(&d, 2 * sizeof(double));
  hyp_status r = HYP_OK;
  if (he != hipSuccess) r = hip_fail(he, "hyp_adapt_energy_fp64: allocation");
  const int j = (int)A.ops.size();
  if (r == HYP_OK && j) {
    std::memcpy(A.h_pin + 1, A.theta.data(), sizeof(double) * j);
    he = hipMemcpyAsync(A.d_theta, A.h_pin + 1, sizeof(double) * j, hipMemcpyHostToDevice, A.st);
    if (he != hipSuccess) r = hip_fail(he, "hyp_adapt_energy_fp64: theta upload");
  }
  if (r == HYP_OK) r = fill_hf(S, HYP_F64, p, A.st);
  for (int i = 0; i < j && r == HYP_OK; ++i)
    r = launch_rotate(S, HYP_F64, A.pool[A.ops[i]], 0.0, A.d_theta + i, p, A.st);
  if (r == HYP_OK) r = apply_h_internal(A.ham, HYP_F64, p, s, A.st);
  if (r == HYP_OK) r = launch_dot(S, HYP_F64, p, s, d, A.st);
  if (r == HYP_OK) r = launch_dot(S, HYP_F64, p, p, d + 1, A.st);
  double hv[2] = {0, 0};
  if (r == HYP_OK) {
    he = hipMemcpyAsync(hv, d, sizeof(hv), hipMemcpyDeviceToHost, A.st);
    if (he == hipSuccess) he = hipStreamSynchronize(A.st);
    if (he != hipSuccess) r = hip_fail(he, "hyp_adapt_energy_fp64: readback");
  }
  (void)hipFree(p);
  (void)hipFree(s);
  (void)hipFree(d);
  if (r == HYP_OK) *e = hv[0] / hv[1];
  return r;
}

}  // extern "C"
