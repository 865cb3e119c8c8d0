/*
 * FP64 CPU oracle for Fisher-vector encoding -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may call this
 * code.  The GPU library never links, loads or calls it, and this file shares no code,
 * headers, tables or constants with it.
 *
 * What it computes (Ma et al., GPU-FV, ICMR'16, Sec. 3.1 and Algorithm 1, and the improved
 * Fisher vector of Perronnin et al. that the paper cites for its encoding):
 *   1. s_kd = 1/sqrt(var_kd)                            (Alg. 1 precomputes the inverse std)
 *   2. per descriptor x_t and component k:
 *        delta_tk = sum_d ((x_td - mu_kd) * s_kd)^2     (squared diagonal Mahalanobis distance)
 *        l_tk     = ln w_k - 1/2 sum_d ln var_kd - 1/2 delta_tk   (Gaussian log-joint; the
 *                   -D/2 ln(2 pi) constant cancels in the posterior)
 *        m_t      = max_k l_tk
 *   3. e_tk = exp(l_tk - m_t),  Z_t = sum_k e_tk
 *   4. gamma_tk = e_tk / Z_t                             (soft assignment)
 *   5. U_kd = sum_t gamma_tk (x_td - mu_kd) s_kd
 *      V_kd = sum_t gamma_tk [((x_td - mu_kd) s_kd)^2 - 1]     (Alg. 1, second loop)
 *      optionally only terms with gamma_tk > tau (Alg. 1's threshold test; tau < 0 = off)
 *   6. u_kd = U_kd / (N sqrt(w_k)),  v_kd = V_kd / (N sqrt(2 w_k))   (Fisher-information
 *      normalisation of the improved FV; not printed in the paper)
 *   7. phi = [u (component-major) ; v (component-major)], length 2KD
 *   8. unless FVO_NO_POWER: phi_i <- sign(phi_i) sqrt(|phi_i|)
 *   9. unless FVO_NO_L2:    phi <- phi / ||phi||_2  (left as is when the norm is 0)
 * Everything is evaluated in IEEE double, sums run sequentially in index order.  Inputs are
 * the float32 arrays the GPU receives, promoted exactly to double, or (the _f64 entry points)
 * double descriptors, such as the exact output of a projection.  Weights are used as given.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FVO_NO_POWER 1u
#define FVO_NO_L2 2u

/* Exact promotion of float32 descriptors to double (NULL on OOM). */
static double* promote(int64_t N, int D, const float* X) {
  double* Xd = (double*)malloc(sizeof(double) * ((size_t)N * D + 1));
  if (!Xd) return NULL;
  for (size_t i = 0; i < (size_t)N * D; ++i) Xd[i] = (double)X[i];
  return Xd;
}

/* Steps 1-4 for one frame: gamma [N x K], row-major.  Returns 0, or -1 on bad sizes / OOM. */
int fvo_posteriors_f64(int64_t N, int K, int D, const double* X, const float* w, const float* mu,
                       const float* var, double* gamma) {
  if (N < 0 || K < 1 || D < 1) return -1;
  double* s = (double*)malloc(sizeof(double) * (size_t)K * D);
  double* logdet_half = (double*)malloc(sizeof(double) * K);
  if (!s || !logdet_half) { free(s); free(logdet_half); return -1; }
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int d = 0; d < D; ++d) {
      double v = (double)var[(size_t)k * D + d];
      s[(size_t)k * D + d] = 1.0 / sqrt(v);
      acc += log(v);
    }
    logdet_half[k] = 0.5 * acc;
  }
  for (int64_t t = 0; t < N; ++t) {
    const double* x = X + (size_t)t * D;
    double* g = gamma + (size_t)t * K;
    double m = -INFINITY;
    for (int k = 0; k < K; ++k) {
      double delta = 0.0;
      for (int d = 0; d < D; ++d) {
        double z = ((double)x[d] - (double)mu[(size_t)k * D + d]) * s[(size_t)k * D + d];
        delta += z * z;
      }
      double l = log((double)w[k]) - logdet_half[k] - 0.5 * delta;
      g[k] = l;
      if (l > m) m = l;
    }
    double Z = 0.0;
    for (int k = 0; k < K; ++k) {
      g[k] = exp(g[k] - m);
      Z += g[k];
    }
    for (int k = 0; k < K; ++k) g[k] = g[k] / Z;
  }
  free(s);
  free(logdet_half);
  return 0;
}

int fvo_posteriors(int64_t N, int K, int D, const float* X, const float* w, const float* mu,
                   const float* var, double* gamma) {
  if (N < 0 || K < 1 || D < 1) return -1;
  double* Xd = promote(N, D, X);
  if (!Xd) return -1;
  int rc = fvo_posteriors_f64(N, K, D, Xd, w, mu, var, gamma);
  free(Xd);
  return rc;
}

/* Steps 1-9 for one frame.  out has 2KD doubles.  tau < 0 disables the threshold. */
int fvo_encode_tau_f64(int64_t N, int K, int D, const double* X, const float* w, const float* mu,
                       const float* var, unsigned flags, double tau, double* out) {
  if (N < 0 || K < 1 || D < 1) return -1;
  const size_t KD = (size_t)K * D;
  memset(out, 0, sizeof(double) * 2 * KD);
  if (N == 0) return 0;
  double* gamma = (double*)malloc(sizeof(double) * (size_t)N * K);
  double* s = (double*)malloc(sizeof(double) * KD);
  if (!gamma || !s) { free(gamma); free(s); return -1; }
  if (fvo_posteriors_f64(N, K, D, X, w, mu, var, gamma) != 0) { free(gamma); free(s); return -1; }
  for (size_t i = 0; i < KD; ++i) s[i] = 1.0 / sqrt((double)var[i]);
  double* U = out;
  double* V = out + KD;
  for (int64_t t = 0; t < N; ++t) {
    const double* x = X + (size_t)t * D;
    for (int k = 0; k < K; ++k) {
      double g = gamma[(size_t)t * K + k];
      if (tau >= 0.0 && !(g > tau)) continue;
      for (int d = 0; d < D; ++d) {
        double z = ((double)x[d] - (double)mu[(size_t)k * D + d]) * s[(size_t)k * D + d];
        U[(size_t)k * D + d] += z * g;
        V[(size_t)k * D + d] += (z * z - 1.0) * g;
      }
    }
  }
  for (int k = 0; k < K; ++k) {
    double cu = 1.0 / ((double)N * sqrt((double)w[k]));
    double cv = 1.0 / ((double)N * sqrt(2.0 * (double)w[k]));
    for (int d = 0; d < D; ++d) {
      U[(size_t)k * D + d] *= cu;
      V[(size_t)k * D + d] *= cv;
    }
  }
  if (!(flags & FVO_NO_POWER)) {
    for (size_t i = 0; i < 2 * KD; ++i) {
      double p = out[i];
      out[i] = (p > 0.0) ? sqrt(p) : ((p < 0.0) ? -sqrt(-p) : 0.0);
    }
  }
  if (!(flags & FVO_NO_L2)) {
    double ss = 0.0;
    for (size_t i = 0; i < 2 * KD; ++i) ss += out[i] * out[i];
    if (ss > 0.0) {
      double inv = 1.0 / sqrt(ss);
      for (size_t i = 0; i < 2 * KD; ++i) out[i] *= inv;
    }
  }
  free(gamma);
  free(s);
  return 0;
}

int fvo_encode_tau(int64_t N, int K, int D, const float* X, const float* w, const float* mu,
                   const float* var, unsigned flags, double tau, double* out) {
  if (N < 0 || K < 1 || D < 1) return -1;
  double* Xd = promote(N, D, X);
  if (!Xd) return -1;
  int rc = fvo_encode_tau_f64(N, K, D, Xd, w, mu, var, flags, tau, out);
  free(Xd);
  return rc;
}

int fvo_encode(int64_t N, int K, int D, const float* X, const float* w, const float* mu,
               const float* var, unsigned flags, double* out) {
  return fvo_encode_tau(N, K, D, X, w, mu, var, flags, -1.0, out);
}

/* Frames b = 0..B-1 are rows [offsets[b], offsets[b+1]) of X; out is [B x 2KD].  Frames are
 * independent, so nthreads > 1 only distributes whole frames over threads: each frame's
 * arithmetic is exactly the single-frame path above. */
int fvo_encode_batch(int B, const int64_t* offsets, int K, int D, const float* X, const float* w,
                     const float* mu, const float* var, unsigned flags, int nthreads, double* out) {
  if (B < 0 || K < 1 || D < 1) return -1;
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] < offsets[b]) return -1;
  int err = 0;
  const size_t L = 2 * (size_t)K * D;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
#endif
  for (int b = 0; b < B; ++b) {
    int64_t n = offsets[b + 1] - offsets[b];
    if (fvo_encode(n, K, D, X + (size_t)offsets[b] * D, w, mu, var, flags, out + (size_t)b * L))
      err |= 1;
  }
  return err ? -1 : 0;
}

int fvo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
