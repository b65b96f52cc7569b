/*
 * ft_oracle.c -- plain FP64 CPU reference of sparse FasterTucker
 * (Li, Duan, Yang, Li: "cuFasterTucker: A Stochastic Optimization Strategy
 * for Parallel Sparse FastTucker Decomposition on GPU Platform").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU baseline
 * of the benchmark do.  It shares no code with the GPU path.
 *
 * Model (Section 2.3, Eq. (1)): factor matrices A(n) (I_n x J_n) and core
 * matrices B(n) (J_n x R).  The Kruskal core sum_r b(1)_r o ... o b(N)_r is
 * multiplied by every A(n) in its mode.  With the cached intermediate
 * C(n) = A(n) B(n) (Section 3.1) the prediction of one element is
 *     xhat(i_1..i_N) = sum_r prod_n C(n)[i_n, r]                 (Eq. (12))
 * Every array is row-major FP64.  Coordinates are int32, structure of arrays:
 * the mode-n index of element x is coords[n * stride + x].
 *
 * Readings where the paper is silent or inconsistent:
 *  - update direction: the gradients of Eq. (10) and Eq. (11) are followed,
 *    a <- a - lr * (-(x - xhat) g + lam a); the pseudo-code of the GPU
 *    algorithms prints the opposite sign in places;
 *  - the weight decay lam * a is applied at every element visit (Eq. (7));
 *  - modes are updated in the order 0..N-1 (Algorithm 2);
 *  - the mode-m fibers are visited in lexicographic order of their fixed
 *    indices taken cyclically (i_{m+1}, ..., i_{N-1}, i_0, ..., i_{m-1}),
 *    the elements of a fiber by increasing i_m.  This is the preorder of the
 *    fiber tree whose leaves are the updated mode (Section 4.5);
 *  - the core module accumulates the gradient of every element and applies
 *    one step B <- B - lr (grad / |Omega| + lam B) per mode (Algorithm 5).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_NOMEM 2

/* C = A B : the reusable intermediate a(n)_{i_n} . b(n)_{:,r} for all rows
 * (Section 3.1; first step of Algorithm 2). */
void orc_refresh(int64_t I, int J, int R, const double* A, const double* B, double* C) {
  for (int64_t i = 0; i < I; ++i)
    for (int r = 0; r < R; ++r) {
      double s = 0.0;
      for (int j = 0; j < J; ++j) s += A[i * J + j] * B[(int64_t)j * R + r];
      C[i * R + r] = s;
    }
}

/* xhat = sum_r prod_n C(n)[i_n, r] (Eq. (1) evaluated through Eq. (12)). */
void orc_predict(int N, int R, const double* const* C, const int32_t* coords, int64_t q, int64_t stride,
                 double* out) {
  for (int64_t x = 0; x < q; ++x) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) {
      double p = 1.0;
      for (int n = 0; n < N; ++n) p *= C[n][(int64_t)coords[n * stride + x] * R + r];
      s += p;
    }
    out[x] = s;
  }
}

/* ---- fiber order of the mode-m passes ---- */
static int g_N, g_m;
static const int32_t* g_coords;
static int64_t g_stride;

static int cmp_fiber(const void* pa, const void* pb) {
  int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
  /* fixed indices, cyclically after m, then the free index i_m */
  for (int k = 1; k <= g_N; ++k) {
    int n = (g_m + k) % g_N;
    int32_t ia = g_coords[n * g_stride + a], ib = g_coords[n * g_stride + b];
    if (ia != ib) return ia < ib ? -1 : 1;
  }
  return (a > b) - (a < b);
}

/* Permutation of 0..nnz-1 that lists the mode-m fibers one after another. */
static int64_t* fiber_order(int N, int m, const int32_t* coords, int64_t nnz) {
  int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
  if (!ord) return NULL;
  for (int64_t x = 0; x < nnz; ++x) ord[x] = x;
  g_N = N;
  g_m = m;
  g_coords = coords;
  g_stride = nnz;
  qsort(ord, (size_t)nnz, sizeof(int64_t), cmp_fiber);
  return ord;
}

static int same_fiber(int N, int m, const int32_t* coords, int64_t nnz, int64_t a, int64_t b) {
  for (int n = 0; n < N; ++n)
    if (n != m && coords[n * nnz + a] != coords[n * nnz + b]) return 0;
  return 1;
}

/* w_r = s(m) q(m)_{:,r} = prod_{n != m} C(n)[i_n, r]           (Eq. (12))
 * g_j = (B(m) Q(m)^T s(m)^T)_j = sum_r B(m)[j, r] w_r           (Section 3.2) */
static void fiber_w_g(int N, int m, int J, int R, const double* Bm, const double* const* C, const int32_t* coords,
                      int64_t nnz, int64_t x, double* w, double* g) {
  for (int r = 0; r < R; ++r) {
    double p = 1.0;
    for (int n = 0; n < N; ++n)
      if (n != m) p *= C[n][(int64_t)coords[n * nnz + x] * R + r];
    w[r] = p;
  }
  for (int j = 0; j < J; ++j) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += Bm[(int64_t)j * R + r] * w[r];
    g[j] = s;
  }
}

/*
 * Factor module of Algorithm 2 for mode m: for every mode-m fiber compute w
 * and the shared g once, then for every element of the fiber take one SGD
 * step (Eq. (9) with a one-element sample) on a(m)_{i_m} with the gradient
 * of Eq. (10):  e = x - a.g ;  a <- a + lr (e g - lam a).
 * C(m) is not refreshed here (the caller does it, as Algorithm 2 does after
 * the module).
 */
int orc_factor_pass(int N, const int64_t* dims, const int* Jv, int R, double* const* A, const double* const* B,
                    const double* const* C, const int32_t* coords, const double* vals, int64_t nnz, int m, double lr,
                    double lam) {
  (void)dims;
  if (N < 2 || m < 0 || m >= N) return ORC_ERR_ARG;
  int J = Jv[m];
  double* Am = A[m];
  const double* Bm = B[m];
  int64_t* ord = fiber_order(N, m, coords, nnz);
  double* w = (double*)malloc(sizeof(double) * R);
  double* g = (double*)malloc(sizeof(double) * J);
  if (!ord || !w || !g) { free(ord); free(w); free(g); return ORC_ERR_NOMEM; }
  int64_t p = 0;
  while (p < nnz) {
    int64_t first = ord[p];
    fiber_w_g(N, m, J, R, Bm, C, coords, nnz, first, w, g);
    int64_t q = p;
    while (q < nnz && same_fiber(N, m, coords, nnz, first, ord[q])) {
      int64_t x = ord[q];
      double* a = Am + (int64_t)coords[m * nnz + x] * J;
      double xhat = 0.0;
      for (int j = 0; j < J; ++j) xhat += a[j] * g[j];
      double e = vals[x] - xhat;
      for (int j = 0; j < J; ++j) a[j] = a[j] + lr * (e * g[j] - lam * a[j]);
      ++q;
    }
    p = q;
  }
  free(ord); free(w); free(g);
  return ORC_OK;
}

/* ---- row order of the relaxed pass: i_m first, then the fiber order ---- */
static int cmp_row(const void* pa, const void* pb) {
  int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
  for (int k = 0; k < g_N; ++k) {
    int n = (g_m + k) % g_N;
    int32_t ia = g_coords[n * g_stride + a], ib = g_coords[n * g_stride + b];
    if (ia != ib) return ia < ib ? -1 : 1;
  }
  return (a > b) - (a < b);
}

/* one SGD step of Eq. (9)/(10) on a, returns ||g||^2 */
static double sgd_step(int N, int m, int J, int R, const double* Bm, const double* const* C, const int32_t* coords,
                       const double* vals, int64_t nnz, int64_t x, double lr, double lam, double* a, double* w,
                       double* g) {
  fiber_w_g(N, m, J, R, Bm, C, coords, nnz, x, w, g);
  double xhat = 0.0, gg = 0.0;
  for (int j = 0; j < J; ++j) {
    xhat += a[j] * g[j];
    gg += g[j] * g[j];
  }
  double e = vals[x] - xhat;
  for (int j = 0; j < J; ++j) a[j] = a[j] + lr * (e * g[j] - lam * a[j]);
  return gg;
}

/*
 * Relaxed factor module for mode m: a deterministic model of the concurrent
 * row updates of the GPU factor algorithm (Algorithm 4 lets many workers read
 * and write one row without ordering).  This is a reading of that algorithm,
 * not the serial result of Algorithm 2.
 *
 * A row's elements are taken in the order i_m, i_{m+1}, ..., i_{m-1} (the
 * per-row order of the fiber traversal).  A row of at most `head` elements is
 * updated serially, exactly as in orc_factor_pass.  A longer row of L
 * elements is first dealt in stride order: with Q = ceil(L / head), its
 * positions 0, Q, 2Q, ..., then 1, 1 + Q, ..., then 2, ... (a worker that
 * takes a piece of a long row sees a sample of the whole row, not a narrow
 * slice of the sorted order; with contiguous pieces the pass diverged on a
 * learning workload once the head reached 4096 elements).  Then, in that order:
 *   - its first `head` elements update the row serially, from a0 to a_H;
 *   - the rest is cut into chunks of `chunk` elements; every chunk k runs its
 *     steps serially from a_H (all chunks read the row as the head left it),
 *     reaching b_k after L_k steps.  Its increment beyond the decay of a_H is
 *     d_k = b_k - rho^{L_k} a_H, with rho = 1 - lr lam;
 *   - the increments are merged in the order of the chunks, each decayed by
 *     the steps that follow it: S = sum_k rho^{T_k} d_k, where T_k counts the
 *     row's elements after chunk k.  Without a guard the row would become
 *     rho^{L - head} a_H + S;
 *   - guard: with G = sum of ||g||^2 over the chunked elements,
 *     omega = min(1, 1 / (lr G)) scales that whole step:
 *         a = a_H + omega ((rho^{L - head} - 1) a_H + S).
 * If the chunk steps did not depend on the row (g g^T a dropped from the
 * step), the unguarded row would be the serial result exactly; as it is, it
 * differs from the serial result by O(lr^2) while omega = 1.  To first order
 * the merged step is lr times the row's full-batch gradient over the chunked
 * elements; omega keeps lr omega sum g g^T below I, so the summed increments
 * cannot overshoot when many chunks fit the same row, and since it scales
 * the decay too, the rows it damps are not pulled towards zero.
 */
int orc_factor_pass_relaxed(int N, const int64_t* dims, const int* Jv, int R, double* const* A,
                            const double* const* B, const double* const* C, const int32_t* coords, const double* vals,
                            int64_t nnz, int m, double lr, double lam, int64_t head, int64_t chunk) {
  (void)dims;
  if (N < 2 || m < 0 || m >= N || head < 0 || chunk < 1) return ORC_ERR_ARG;
  int J = Jv[m];
  double* Am = A[m];
  const double* Bm = B[m];
  const double rho = 1.0 - lr * lam;
  int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
  double* w = (double*)malloc(sizeof(double) * R);
  double* g = (double*)malloc(sizeof(double) * J);
  double* b = (double*)malloc(sizeof(double) * J);
  double* S = (double*)malloc(sizeof(double) * J);
  int64_t* dealt = (int64_t*)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
  if (!ord || !w || !g || !b || !S || !dealt) {
    free(ord); free(w); free(g); free(b); free(S); free(dealt);
    return ORC_ERR_NOMEM;
  }
  for (int64_t x = 0; x < nnz; ++x) ord[x] = x;
  g_N = N;
  g_m = m;
  g_coords = coords;
  g_stride = nnz;
  qsort(ord, (size_t)nnz, sizeof(int64_t), cmp_row);
  int64_t p = 0;
  while (p < nnz) {
    int32_t row = coords[m * nnz + ord[p]];
    int64_t q = p;
    while (q < nnz && coords[m * nnz + ord[q]] == row) ++q;
    int64_t L = q - p;
    double* a = Am + (int64_t)row * J;
    int64_t hl = L <= head ? L : head;
    if (L > head && head > 0) {
      int64_t Q = (L + head - 1) / head, o = 0;
      for (int64_t r = 0; r < Q; ++r)
        for (int64_t t = r; t < L; t += Q) dealt[o++] = ord[p + t];
      for (int64_t t = 0; t < L; ++t) ord[p + t] = dealt[t];
    }
    for (int64_t t = 0; t < hl; ++t) sgd_step(N, m, J, R, Bm, C, coords, vals, nnz, ord[p + t], lr, lam, a, w, g);
    if (L > head) {
      /* a holds a_H from here on */
      double G = 0.0;
      for (int j = 0; j < J; ++j) S[j] = 0.0;
      for (int64_t c0 = head; c0 < L; c0 += chunk) {
        int64_t c1 = c0 + chunk < L ? c0 + chunk : L;
        for (int j = 0; j < J; ++j) b[j] = a[j];
        for (int64_t t = c0; t < c1; ++t) G += sgd_step(N, m, J, R, Bm, C, coords, vals, nnz, ord[p + t], lr, lam, b, w, g);
        double decay_own = pow(rho, (double)(c1 - c0)), decay_after = pow(rho, (double)(L - c1));
        for (int j = 0; j < J; ++j) S[j] += decay_after * (b[j] - decay_own * a[j]);
      }
      double omega = lr * G > 1.0 ? 1.0 / (lr * G) : 1.0;
      double decay_rest = pow(rho, (double)(L - head));
      for (int j = 0; j < J; ++j) a[j] = a[j] + omega * ((decay_rest - 1.0) * a[j] + S[j]);
    }
    p = q;
  }
  free(ord); free(w); free(g); free(b); free(S); free(dealt);
  return ORC_OK;
}

/*
 * Core gradient of mode m over all elements at fixed parameters
 * (Eq. (11), summed over Omega as Algorithm 5 accumulates it):
 *     G[j, r] = sum_x e_x a(m)_{i_m}[j] w_x[r],  e_x = x - xhat_x.
 */
int orc_core_grad(int N, const int* Jv, int R, const double* const* A, const double* const* B, const double* const* C,
                  const int32_t* coords, const double* vals, int64_t nnz, int m, double* G) {
  if (N < 2 || m < 0 || m >= N) return ORC_ERR_ARG;
  int J = Jv[m];
  const double* Am = A[m];
  const double* Bm = B[m];
  int64_t* ord = fiber_order(N, m, coords, nnz);
  double* w = (double*)malloc(sizeof(double) * R);
  double* g = (double*)malloc(sizeof(double) * J);
  if (!ord || !w || !g) { free(ord); free(w); free(g); return ORC_ERR_NOMEM; }
  memset(G, 0, sizeof(double) * J * R);
  int64_t p = 0;
  while (p < nnz) {
    int64_t first = ord[p];
    fiber_w_g(N, m, J, R, Bm, C, coords, nnz, first, w, g);
    int64_t q = p;
    while (q < nnz && same_fiber(N, m, coords, nnz, first, ord[q])) {
      int64_t x = ord[q];
      const double* a = Am + (int64_t)coords[m * nnz + x] * J;
      double xhat = 0.0;
      for (int j = 0; j < J; ++j) xhat += a[j] * g[j];
      double e = vals[x] - xhat;
      for (int j = 0; j < J; ++j)
        for (int r = 0; r < R; ++r) G[j * R + r] += e * a[j] * w[r];
      ++q;
    }
    p = q;
  }
  free(ord); free(w); free(g);
  return ORC_OK;
}

/* Core module of Algorithm 2 for mode m: one step on B(m) with the gradient
 * accumulated over Omega, B <- B + lr (G / |Omega| - lam B) (Algorithm 5). */
int orc_core_pass(int N, const int* Jv, int R, const double* const* A, double* const* B, const double* const* C,
                  const int32_t* coords, const double* vals, int64_t nnz, int m, double lr, double lam) {
  int J = Jv[m];
  double* G = (double*)malloc(sizeof(double) * J * R);
  if (!G) return ORC_ERR_NOMEM;
  int rc = orc_core_grad(N, Jv, R, A, (const double* const*)B, C, coords, vals, nnz, m, G);
  if (rc == ORC_OK && nnz > 0) {
    double* Bm = B[m];
    for (int k = 0; k < J * R; ++k) Bm[k] = Bm[k] + lr * (G[k] / (double)nnz - lam * Bm[k]);
  }
  free(G);
  return rc;
}

/* One iteration of Algorithm 2: the factor module (modes 0..N-1, each
 * followed by a refresh of C(m)), then the core module (same order). */
int orc_epoch(int N, const int64_t* dims, const int* Jv, int R, double* const* A, double* const* B, double* const* C,
              const int32_t* coords, const double* vals, int64_t nnz, double lr_a, double lam_a, double lr_b,
              double lam_b) {
  for (int m = 0; m < N; ++m) {
    int rc = orc_factor_pass(N, dims, Jv, R, A, (const double* const*)B, (const double* const*)C, coords, vals, nnz,
                             m, lr_a, lam_a);
    if (rc) return rc;
    orc_refresh(dims[m], Jv[m], R, A[m], B[m], C[m]);
  }
  for (int m = 0; m < N; ++m) {
    int rc = orc_core_pass(N, Jv, R, (const double* const*)A, B, (const double* const*)C, coords, vals, nnz, m, lr_b,
                           lam_b);
    if (rc) return rc;
    orc_refresh(dims[m], Jv[m], R, A[m], B[m], C[m]);
  }
  return ORC_OK;
}

/* Objective of Eq. (6), split: out[0] = sum (x - xhat)^2, out[1] = RMSE
 * = sqrt(out[0] / |Omega|), out[2] = sum_n lam_a ||A(n)||^2,
 * out[3] = sum_n lam_b ||B(n)||^2. */
void orc_loss(int N, const int64_t* dims, const int* Jv, int R, const double* const* A, const double* const* B,
              const double* const* C, const int32_t* coords, const double* vals, int64_t nnz, double lam_a,
              double lam_b, double* out) {
  double sse = 0.0;
  for (int64_t x = 0; x < nnz; ++x) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) {
      double p = 1.0;
      for (int n = 0; n < N; ++n) p *= C[n][(int64_t)coords[n * nnz + x] * R + r];
      s += p;
    }
    double e = vals[x] - s;
    sse += e * e;
  }
  double ra = 0.0, rb = 0.0;
  for (int n = 0; n < N; ++n) {
    for (int64_t k = 0; k < dims[n] * Jv[n]; ++k) ra += A[n][k] * A[n][k];
    for (int64_t k = 0; k < (int64_t)Jv[n] * R; ++k) rb += B[n][k] * B[n][k];
  }
  out[0] = sse;
  out[1] = nnz > 0 ? sqrt(sse / (double)nnz) : 0.0;
  out[2] = lam_a * ra;
  out[3] = lam_b * rb;
}

/*
 * Gradient of a loss L(xhat) at fixed parameters, given dL/dxhat_x = delta_x
 * for every element (upstream == NULL means delta_x = -(x - xhat_x), the
 * gradient of 1/2 sum e^2).  For every mode n, by Eq. (10) and Eq. (11)
 * without the regularisers:
 *     dA(n)[i] = sum_{x: i_n = i} delta_x g(n)_x ,
 *     dB(n)    = sum_x delta_x a(n)_{i_n} w(n)_x^T .
 */
int orc_grad(int N, const int64_t* dims, const int* Jv, int R, const double* const* A, const double* const* B,
             const double* const* C, const int32_t* coords, const double* vals, int64_t nnz, const double* upstream,
             double* const* gA, double* const* gB) {
  int Jmax = 1;
  for (int n = 0; n < N; ++n) Jmax = Jv[n] > Jmax ? Jv[n] : Jmax;
  double* w = (double*)malloc(sizeof(double) * R);
  double* g = (double*)malloc(sizeof(double) * Jmax);
  if (!w || !g) { free(w); free(g); return ORC_ERR_NOMEM; }
  for (int n = 0; n < N; ++n) {
    memset(gA[n], 0, sizeof(double) * dims[n] * Jv[n]);
    memset(gB[n], 0, sizeof(double) * Jv[n] * R);
  }
  for (int64_t x = 0; x < nnz; ++x) {
    double delta;
    if (upstream) {
      delta = upstream[x];
    } else {
      double s = 0.0;
      for (int r = 0; r < R; ++r) {
        double p = 1.0;
        for (int n = 0; n < N; ++n) p *= C[n][(int64_t)coords[n * nnz + x] * R + r];
        s += p;
      }
      delta = -(vals[x] - s);
    }
    for (int n = 0; n < N; ++n) {
      int J = Jv[n];
      fiber_w_g(N, n, J, R, B[n], C, coords, nnz, x, w, g);
      int64_t i = coords[n * nnz + x];
      for (int j = 0; j < J; ++j) gA[n][i * J + j] += delta * g[j];
      const double* a = A[n] + i * J;
      for (int j = 0; j < J; ++j)
        for (int r = 0; r < R; ++r) gB[n][j * R + r] += delta * a[j] * w[r];
    }
  }
  free(w); free(g);
  return ORC_OK;
}
