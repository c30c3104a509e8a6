/*
 * A plain C client of the library: reads a molecule from a binary file,
 * evaluates its profile on HIP device 0 through the C ABI alone, and writes
 * I(q) (FP64) to a second file.  Also exercises the status/error reporting.
 *
 * Input file: int64 n, int32 t, int32 nq, float coords[n][3], int32 types[n],
 * float table[t][nq], double q[nq].  Output file: double I[nq].
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sas_debye.h"

#define HIPCHECK(x)                                                         \
  do {                                                                      \
    hipError_t e_ = (x);                                                    \
    if (e_ != hipSuccess) {                                                 \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
      return 2;                                                             \
    }                                                                       \
  } while (0)

static int read_all(FILE* f, void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes ? 0 : -1; }

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input.bin output.bin\n", argv[0]);
    return 1;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int64_t n = 0;
  int32_t t = 0, nq = 0;
  if (read_all(f, &n, 8) || read_all(f, &t, 4) || read_all(f, &nq, 4)) return 1;
  if (n < 0 || t < 1 || nq < 1) return 1;
  float* coords = malloc(sizeof(float) * 3 * (n > 0 ? n : 1));
  int32_t* types = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  float* table = malloc(sizeof(float) * (size_t)t * nq);
  double* q = malloc(sizeof(double) * nq);
  double* I = malloc(sizeof(double) * nq);
  if (read_all(f, coords, sizeof(float) * 3 * n) || read_all(f, types, sizeof(int32_t) * n) ||
      read_all(f, table, sizeof(float) * (size_t)t * nq) || read_all(f, q, sizeof(double) * nq))
    return 1;
  fclose(f);

  /* error reporting without a context */
  sas_status st = sas_debye_profile(NULL, NULL, NULL, n, table, t, q, nq, NULL, NULL, 0, NULL);
  if (st != SAS_ERR_INVALID_ARG || strlen(sas_last_error()) == 0) {
    fprintf(stderr, "expected SAS_ERR_INVALID_ARG, got %d (%s)\n", (int)st, sas_status_string(st));
    return 3;
  }

  sas_ctx* ctx = NULL;
  st = sas_create(0, &ctx);
  if (st != SAS_OK) {
    fprintf(stderr, "sas_create: %s: %s\n", sas_status_string(st), sas_last_error());
    return 4;
  }
  void *dc = NULL, *dt = NULL, *dtab = NULL, *dI = NULL, *ws = NULL;
  HIPCHECK(hipMalloc(&dc, sizeof(float) * 3 * (n > 0 ? n : 1)));
  HIPCHECK(hipMalloc(&dt, sizeof(int32_t) * (n > 0 ? n : 1)));
  HIPCHECK(hipMalloc(&dtab, sizeof(float) * (size_t)t * nq));
  HIPCHECK(hipMalloc(&dI, sizeof(double) * nq));
  HIPCHECK(hipMemcpy(dc, coords, sizeof(float) * 3 * n, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dt, types, sizeof(int32_t) * n, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dtab, table, sizeof(float) * (size_t)t * nq, hipMemcpyHostToDevice));
  const size_t wsb = sas_debye_workspace_size(ctx, n, t, nq, 0);
  if (wsb == 0) return 5;
  HIPCHECK(hipMalloc(&ws, wsb));
  /* a 256-byte workspace is refused before any device work */
  st = sas_debye_profile(ctx, dc, dt, n, dtab, t, q, nq, dI, ws, 256, NULL);
  if (st != SAS_ERR_WORKSPACE_TOO_SMALL) return 6;
  st = sas_debye_profile(ctx, dc, dt, n, dtab, t, q, nq, dI, ws, wsb, NULL);
  if (st != SAS_OK) {
    fprintf(stderr, "sas_debye_profile: %s: %s\n", sas_status_string(st), sas_last_error());
    return 7;
  }
  HIPCHECK(hipDeviceSynchronize());
  HIPCHECK(hipMemcpy(I, dI, sizeof(double) * nq, hipMemcpyDeviceToHost));
  f = fopen(argv[2], "wb");
  if (!f || fwrite(I, sizeof(double), nq, f) != (size_t)nq) return 8;
  fclose(f);
  HIPCHECK(hipFree(ws));
  HIPCHECK(hipFree(dI));
  HIPCHECK(hipFree(dtab));
  HIPCHECK(hipFree(dt));
  HIPCHECK(hipFree(dc));
  sas_destroy(ctx);
  free(coords);
  free(types);
  free(table);
  free(q);
  free(I);
  printf("sas_client: %lld atoms, %d types, %d q: ok (library version %d)\n", (long long)n, t, nq, sas_version());
  return 0;
}
