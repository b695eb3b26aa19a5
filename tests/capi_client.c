/*
 * A plain C99 client of libifnso: only include/ifnso.h, the HIP runtime API and the library,
 * no Python and no torch. Used by the test suite to show that the C ABI stands on its own.
 *
 * 1. float32 plan, Gram basis, no normalisation, coefficients summing to one: a matrix with
 *    orthonormal rows, Q = [I | 0], is a fixed point of the polynomial (Y = Q).
 * 2. bfloat16 batched plan over a wide and a tall problem, Frobenius normalisation: for
 *    M = [diag(sigma) | 0] (or its transpose) the method acts on singular values only, so
 *    Y = [diag(f(sigma / ||sigma||)) | 0] with f(x) = x p(x^2), p(g) = sum_k c_k g^(e_k);
 *    the client computes f in double precision and compares every entry.
 *
 * Prints one line per check and returns 0 when all pass.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ifnso.h"

#define HIPCK(x)                                                             \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                              \
    }                                                                        \
  } while (0)
#define IFCK(x)                                                                            \
  do {                                                                                     \
    ifnso_status s_ = (x);                                                                 \
    if (s_ != IFNSO_OK) {                                                                  \
      printf("ifnso status %d at line %d: %s\n", (int)s_, __LINE__, ifnso_last_error()); \
      return 1;                                                                            \
    }                                                                                      \
  } while (0)

static uint16_t to_bf16(float f) {  /* round to nearest even */
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static float from_bf16(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

static const int32_t kExps[3] = {0, 1, 2};
static const double kCoeffs[3] = {1.875, -1.25, 0.375};

static double poly(double g) { return kCoeffs[0] + kCoeffs[1] * g + kCoeffs[2] * g * g; }

static int check_fixed_point(void) {
  const int64_t h = 96, w = 200;
  ifnso_poly_desc d = {3, kExps, kCoeffs, IFNSO_BASIS_GRAM, IFNSO_NORM_NONE, IFNSO_COMPUTE_F32,
                       IFNSO_COEFF_FIXED, NULL, 0, IFNSO_FLAG_ENFORCE_SUM_ONE};
  ifnso_plan_t plan = NULL;
  IFCK(ifnso_plan(&d, 1, &h, &w, IFNSO_F32, IFNSO_F32, 0, &plan));
  size_t wsb = 0;
  IFCK(ifnso_plan_workspace_bytes(plan, &wsb));
  float *hq = (float *)calloc((size_t)(h * w), sizeof(float));
  float *hy = (float *)calloc((size_t)(h * w), sizeof(float));
  for (int64_t i = 0; i < h; i++) hq[i * w + i] = 1.f;
  void *dm = NULL, *dy = NULL, *ws = NULL;
  HIPCK(hipMalloc(&dm, (size_t)(h * w) * 4));
  HIPCK(hipMalloc(&dy, (size_t)(h * w) * 4));
  HIPCK(hipMalloc(&ws, wsb));
  HIPCK(hipMemcpy(dm, hq, (size_t)(h * w) * 4, hipMemcpyHostToDevice));
  IFCK(ifnso_orthogonalize(plan, dm, w, dy, w, ws, wsb, NULL));
  HIPCK(hipDeviceSynchronize());
  HIPCK(hipMemcpy(hy, dy, (size_t)(h * w) * 4, hipMemcpyDeviceToHost));
  double err = 0.0;
  for (int64_t k = 0; k < h * w; k++) err = fmax(err, fabs((double)hy[k] - (double)hq[k]));
  printf("fixed point [I | 0], %lldx%lld float32: max |Y - Q| = %.3e\n", (long long)h, (long long)w, err);
  IFCK(ifnso_plan_destroy(plan));
  HIPCK(hipFree(dm));
  HIPCK(hipFree(dy));
  HIPCK(hipFree(ws));
  free(hq);
  free(hy);
  return err <= 1e-5 ? 0 : 1;
}

static int check_batched_closed_form(void) {
  /* problem 0: wide 128 x 384; problem 1: tall 512 x 160 */
  const int64_t rows[2] = {128, 512}, cols[2] = {384, 160};
  ifnso_poly_desc d = {3, kExps, kCoeffs, IFNSO_BASIS_GRAM, IFNSO_NORM_FROBENIUS, IFNSO_COMPUTE_BF16,
                       IFNSO_COEFF_FIXED, NULL, 0, 0};
  ifnso_plan_t plan = NULL;
  IFCK(ifnso_plan(&d, 2, rows, cols, IFNSO_BF16, IFNSO_BF16, 0, &plan));
  size_t wsb = 0;
  IFCK(ifnso_plan_workspace_bytes(plan, &wsb));
  void *ws = NULL;
  HIPCK(hipMalloc(&ws, wsb));
  void *dm[2], *dy[2];
  uint16_t *hm[2], *hy[2];
  double *sig[2];
  int64_t hh[2];
  for (int p = 0; p < 2; p++) {
    const int64_t r = rows[p], c = cols[p], n = r * c, h = r < c ? r : c;
    hh[p] = h;
    hm[p] = (uint16_t *)calloc((size_t)n, 2);
    hy[p] = (uint16_t *)calloc((size_t)n, 2);
    sig[p] = (double *)calloc((size_t)h, sizeof(double));
    for (int64_t i = 0; i < h; i++) {
      sig[p][i] = 0.5 + (double)(i % 8) / 16.0; /* exact in bfloat16 */
      hm[p][i * c + i] = to_bf16((float)sig[p][i]);
    }
    HIPCK(hipMalloc(&dm[p], (size_t)n * 2));
    HIPCK(hipMalloc(&dy[p], (size_t)n * 2));
    HIPCK(hipMemcpy(dm[p], hm[p], (size_t)n * 2, hipMemcpyHostToDevice));
  }
  const void *mp[2] = {dm[0], dm[1]};
  void *yp[2] = {dy[0], dy[1]};
  IFCK(ifnso_orthogonalize_batched(plan, mp, cols, yp, cols, ws, wsb, NULL));
  HIPCK(hipDeviceSynchronize());
  int bad = 0;
  for (int p = 0; p < 2; p++) {
    const int64_t r = rows[p], c = cols[p], h = hh[p];
    HIPCK(hipMemcpy(hy[p], dy[p], (size_t)(r * c) * 2, hipMemcpyDeviceToHost));
    double nrm = 0.0;
    for (int64_t i = 0; i < h; i++) nrm += sig[p][i] * sig[p][i];
    nrm = sqrt(nrm);
    double err = 0.0, ref = 0.0;
    for (int64_t i = 0; i < r; i++)
      for (int64_t j = 0; j < c; j++) {
        double want = 0.0;
        if (i == j) {
          const double x = sig[p][i] / nrm;
          want = x * poly(x * x);
        }
        const double got = (double)from_bf16(hy[p][i * c + j]);
        err = fmax(err, fabs(got - want));
        ref = fmax(ref, fabs(want));
      }
    printf("closed form, %lldx%lld bf16 (batched): max |Y - Y*| / max |Y*| = %.3e\n", (long long)r, (long long)c,
           err / ref);
    if (!(err <= 2e-2 * ref)) bad = 1;
    HIPCK(hipFree(dm[p]));
    HIPCK(hipFree(dy[p]));
    free(hm[p]);
    free(hy[p]);
    free(sig[p]);
  }
  IFCK(ifnso_plan_destroy(plan));
  HIPCK(hipFree(ws));
  return bad;
}

int main(void) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    printf("no GPU\n");
    return 2;
  }
  int rc = check_fixed_point();
  rc |= check_batched_closed_form();
  printf(rc ? "FAILED\n" : "OK\n");
  return rc;
}
