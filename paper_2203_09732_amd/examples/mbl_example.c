/* A plain C99 caller of the library's C ABI (include/mbl.h): no Python, no
 * torch. It builds the S^z = 0 basis of Eq. (1) for a chain of length L
 * (first argument) with the L fields read from stdin, then
 *   1. y = (H - sigma) x for x_i = sin(i + 1), sigma = 0.25;
 *   2. sigma_mid = (E_min + E_max) / 2 (Sec. IV A);
 *   3. preconditioned MINRES (Alg. 2) for (H - sigma_mid) v = x, tol 1e-12;
 *   4. the four eigenpairs nearest sigma_mid by shift-invert Lanczos (Alg. 1)
 *      and their twist overlaps z (Sec. III).
 * It prints "key value ..." lines on stdout; every library error ends the
 * program with the status and mbl_last_error(). Device memory comes from
 * the HIP runtime API. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "mbl.h"

static void check(mbl_status st, const char* what) {
  if (st < 0) {
    fprintf(stderr, "%s failed: status %d: %s\n", what, (int)st, mbl_last_error());
    exit(2);
  }
}

static void hcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s failed: %s\n", what, hipGetErrorString(e));
    exit(3);
  }
}

static void print_vec(const char* key, const double* v, int64_t n) {
  printf("%s", key);
  for (int64_t i = 0; i < n; ++i) printf(" %.17g", v[i]);
  printf("\n");
}

int main(int argc, char** argv) {
  const int L = argc > 1 ? atoi(argv[1]) : 12;
  double h[32];
  if (L < 4 || L > 32) return 1;
  for (int j = 0; j < L; ++j)
    if (scanf("%lf", &h[j]) != 1) return 1;

  mbl_basis b = NULL;
  check(mbl_build_basis(L, 0, NULL, &b), "mbl_build_basis");
  int64_t n = 0;
  check(mbl_basis_dim(b, &n), "mbl_basis_dim");
  printf("version %s\nn %lld\n", mbl_version(), (long long)n);

  double* xh = (double*)malloc(sizeof(double) * (size_t)n);
  double* yh = (double*)malloc(sizeof(double) * (size_t)n);
  if (!xh || !yh) return 4;
  for (int64_t i = 0; i < n; ++i) xh[i] = sin((double)(i + 1));
  double *xd = NULL, *yd = NULL, *vd = NULL;
  hcheck(hipMalloc((void**)&xd, sizeof(double) * (size_t)n), "hipMalloc");
  hcheck(hipMalloc((void**)&yd, sizeof(double) * (size_t)n), "hipMalloc");
  hcheck(hipMalloc((void**)&vd, sizeof(double) * (size_t)n), "hipMalloc");
  hcheck(hipMemcpy(xd, xh, sizeof(double) * (size_t)n, hipMemcpyHostToDevice), "hipMemcpy");

  /* 1. the matrix-free product */
  check(mbl_apply_H(b, h, 0.25, xd, yd, NULL), "mbl_apply_H");
  hcheck(hipMemcpy(yh, yd, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy");
  print_vec("apply", yh, n);

  /* 2. the spectral midpoint */
  double emin = 0, emax = 0, sigma = 0;
  check(mbl_sigma_midpoint(b, h, 1e-12, 0, &emin, &emax, &sigma, NULL), "mbl_sigma_midpoint");
  printf("sigma %.17g %.17g %.17g\n", emin, emax, sigma);

  /* 3. MINRES at the midpoint */
  mbl_workspace ws = NULL;
  check(mbl_workspace_create(b, 0, MBL_FP64, &ws), "mbl_workspace_create");
  hcheck(hipMemset(vd, 0, sizeof(double) * (size_t)n), "hipMemset");
  mbl_minres_info info;
  const mbl_status st = mbl_minres_solve(b, h, sigma, xd, vd, 1e-12, 10000000, MBL_FP64,
                                         MBL_PRECOND_ROW, ws, &info, NULL);
  check(st, "mbl_minres_solve");
  printf("minres %d %lld %.3e %.3e\n", (int)st, (long long)info.iters, info.phi, info.true_res);
  hcheck(hipMemcpy(yh, vd, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy");
  print_vec("solution", yh, n);
  mbl_workspace_free(ws);

  /* 4. eigenpairs nearest the midpoint and their twist overlaps */
  const int nev = 4, mmax = 80;
  mbl_workspace wl = NULL;
  check(mbl_workspace_create(b, mmax, MBL_FP64, &wl), "mbl_workspace_create");
  double* U = NULL;
  hcheck(hipMalloc((void**)&U, sizeof(double) * (size_t)n * nev), "hipMalloc");
  double evals[4], resid[4], z[8];
  mbl_si_info si;
  const double escale = fabs(emin) > fabs(emax) ? fabs(emin) : fabs(emax);
  const mbl_status sl = mbl_si_lanczos(b, h, sigma, nev, mmax, 1e-12, 10000000, 1e-10, 1e-5,
                                       escale, NULL, 7, MBL_FP64, MBL_PRECOND_ROW, wl, evals, U,
                                       n, resid, &si, NULL);
  check(sl, "mbl_si_lanczos");
  check(mbl_twist_expect(b, U, n, nev, z, NULL), "mbl_twist_expect");
  printf("lanczos %d %d %d\n", (int)sl, (int)si.steps, (int)si.nconv);
  print_vec("evals", evals, nev);
  print_vec("resid", resid, nev);
  print_vec("z", z, 2 * nev);

  hcheck(hipFree(U), "hipFree");
  mbl_workspace_free(wl);
  hcheck(hipFree(xd), "hipFree");
  hcheck(hipFree(yd), "hipFree");
  hcheck(hipFree(vd), "hipFree");
  free(xh);
  free(yh);
  mbl_basis_free(b);
  return 0;
}
