/* Driver that runs every routine of the C oracle on small random inputs with
 * exactly sized heap buffers, for a build under the address and
 * undefined-behaviour sanitizers (tests/test_oracle_sanitize.py).  Every band
 * and vector is its own allocation of exactly the size the routine may touch,
 * so a read or write past a record array, a vector or a scratch buffer is
 * reported by the sanitizer.  The numbers are not checked here: the other
 * oracle tests pin them. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) {   /* xorshift64*, uniform in [0, 1) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}
static double nrand(void) { return urand() + urand() + urand() - 1.5; }

static double *alloc(int64_t count) {
  double *p = (double *)malloc((size_t)(count > 0 ? count : 1) * sizeof(double));
  for (int64_t i = 0; i < count; ++i) p[i] = nrand();
  return p;
}

/* Random lower factor (positive diagonal) and Q = band(L0 L0^T) by the
 * oracle's own product, pads zero. */
static void make_spd(int64_t n, int k, double **L0, double **Q) {
  const int64_t ld = k + 1;
  *L0 = alloc(n * ld);
  for (int64_t j = 0; j < n; ++j) {
    (*L0)[j * ld] = 1.0 + urand();
    for (int d = 1; d <= k; ++d)
      if (j + d >= n) (*L0)[j * ld + d] = 0.0;
  }
  *Q = alloc(n * ld);
  or_gbmm(n, k, 0, ld, *L0, 0, k, 0, ld, *L0, 1, k, 0, ld, *Q);
}

static void run_case(int64_t n, int k) {
  const int64_t ld = k + 1;
  double *L0, *Q;
  make_spd(n, k, &L0, &Q);
  double *L = alloc(n * ld), *S = alloc(n * ld), *Sw = alloc(n * (k + 3));
  double *y = alloc(n), *z = alloc(n), *x = alloc(n), *xb = alloc(n), *bb = alloc(n);
  double *Lb = alloc(n * ld), *Qb = alloc(n * ld), *Sb = alloc(n * ld), *Lb2 = alloc(n * ld);
  int info = or_chol(n, k, ld, Q, L);
  if (info != 0) {
    fprintf(stderr, "unexpected info %d at n=%lld k=%d\n", info, (long long)n, k);
    exit(2);
  }
  volatile double sink = or_logdet(n, k, ld, L);
  or_trsv(n, k, ld, L, 0, y, z);
  or_trsv(n, k, ld, L, 1, z, x);
  or_subset_inv(n, k, ld, L, k, ld, S);
  or_subset_inv(n, k, ld, L, k + 2, k + 3, Sw);
  or_chol_bwd(n, k, ld, L, Lb, Qb);
  or_subset_inv_bwd(n, k, ld, L, S, Sb, Lb2);
  for (int t = 0; t < 2; ++t) or_trsv_bwd(n, k, ld, L, t, x, xb, bb, Lb2);
  or_logdet_bwd(n, k, ld, L, 0.5, Lb2);
  or_gbmv(n, k, 0, ld, L, 0, y, z);
  or_gbmv(n, k, 0, ld, L, 1, y, z);
  double *O = alloc(n * (2 * k + 1));
  or_outer_band(n, k, k, 2 * k + 1, y, x, O);
  or_gbmm(n, k, 0, ld, L, 1, k, 0, ld, L, 0, k, k, 2 * k + 1, O);
  {
    const int lr = 2, ur = 3;
    double *R = alloc(n * (lr + ur + 1)), *Ob = alloc(n * (k + ur + 1));
    double *Om = alloc(n * (k + ur + 1)), *Rb = alloc(n * (lr + ur + 1)), *Lb3 = alloc(n * ld);
    or_solve_band_mat(n, k, ld, L, lr, ur, lr + ur + 1, R, k + ur + 1, Om);
    or_solve_band_mat_bwd(n, k, ld, L, lr, ur, k + ur + 1, Om, Ob, lr + ur + 1, Rb, Lb3);
    free(R); free(Ob); free(Om); free(Rb); free(Lb3);
  }
  {
    double parts[5], Ssym[1];
    (void)Ssym;
    double *Sq = alloc(n * ld);   /* symmetric band: diagonally dominant */
    for (int64_t j = 0; j < n; ++j) Sq[j * ld] = 4.0 + urand();
    double *Lo = alloc(n * ld), *zo = alloc(n), *So = alloc(n * ld), *Lbo = alloc(n * ld);
    or_gauss_loss(n, k, ld, Q, y, Sq, parts, Qb, bb, Lo, zo, So, Lbo);
    double *mask = alloc(n);
    for (int64_t j = 0; j < n; ++j) mask[j] = (urand() < 0.7) ? 1.0 : 0.0;
    double tau2b;
    or_marglik(n, k, ld, Q, mask, y, 0.1, parts, Qb, bb, &tau2b);
    double *Ll = alloc(n * ld);
    for (int64_t j = 0; j < n; ++j) {
      Ll[j * ld] = urand();
      for (int d = 1; d <= k; ++d) Ll[j * ld + d] = 0.0;
    }
    double *e1 = alloc(n), *e2 = alloc(n);
    or_natgp(n, k, ld, Q, y, Ll, x, parts, Qb, Lb, e1, e2);
    double *F = alloc(n), *Fb = alloc(n);
    or_whiten(n, k, ld, Q, y, Lo, F);
    or_whiten_bwd(n, k, ld, Lo, F, Fb, e1, Qb);
    or_vi_kl(n, k, ld, L, L0, y, x, parts, Lb, Lb2, e1, e2, So);
    free(Sq); free(Lo); free(zo); free(So); free(Lbo); free(mask); free(Ll);
    free(e1); free(e2); free(F); free(Fb);
  }
  (void)sink;
  free(L0); free(Q); free(L); free(S); free(Sw); free(y); free(z); free(x); free(xb);
  free(bb); free(Lb); free(Qb); free(Sb); free(Lb2); free(O);
}

static void run_batch(void) {
  const int nprob = 4;
  int64_t n[4] = {37, 1, 200, 9};
  int k[4] = {3, 0, 5, 11};
  int64_t boff[4], voff[4], nb = 0, nv = 0;
  for (int p = 0; p < nprob; ++p) {
    boff[p] = nb;
    voff[p] = nv;
    nb += n[p] * (k[p] + 1);
    nv += n[p];
  }
  double *Q = alloc(nb), *y = alloc(nv), *S = alloc(nb);
  for (int p = 0; p < nprob; ++p) {
    double *L0, *Qp;
    make_spd(n[p], k[p], &L0, &Qp);
    memcpy(Q + boff[p], Qp, (size_t)(n[p] * (k[p] + 1)) * sizeof(double));
    memcpy(S + boff[p], Qp, (size_t)(n[p] * (k[p] + 1)) * sizeof(double));
    free(L0);
    free(Qp);
  }
  double *L = alloc(nb), *Sig = alloc(nb), *z = alloc(nv), *x = alloc(nv);
  double *Qb = alloc(nb), *yb = alloc(nv), *Lq = alloc(nb), *Lp = alloc(nb), *mb = alloc(nv);
  double logdet[4], parts[16];
  int info[4];
  or_forward_batch(nprob, n, k, boff, voff, Q, y, L, z, x, Sig, logdet, info);
  or_forward_batch(nprob, n, k, boff, voff, Q, y, NULL, NULL, NULL, NULL, logdet, info);
  or_gauss_loss_batch(nprob, n, k, boff, voff, Q, y, S, parts, Qb, yb, info);
  or_vi_kl_batch(nprob, n, k, boff, voff, L, L, y, x, parts, Lq, Lp, mb, yb);
  free(Q); free(y); free(S); free(L); free(Sig); free(z); free(x); free(Qb); free(yb);
  free(Lq); free(Lp); free(mb);
}

int main(void) {
  const int64_t ns[] = {1, 2, 3, 7, 40};
  const int ks[] = {0, 1, 3, 5, 11, 12};
  for (size_t a = 0; a < sizeof(ns) / sizeof(ns[0]); ++a)
    for (size_t b = 0; b < sizeof(ks) / sizeof(ks[0]); ++b) run_case(ns[a], ks[b]);
  run_batch();
  printf("oracle sanitizer run ok\n");
  return 0;
}
