/* One QP solved through the C ABI of librelu_qp alone (C99, no Python): reads n, m and
 * P, q, A, l, u (FP64, row-major, raw little-endian files) from a directory, runs the offline
 * stage and one solve on the GPU, and writes x, z, y, the iteration count, the status and the
 * per-check penalty indices back to the same directory.
 *
 * Usage: relu_qp_example DIR MAX_ITER PRECISION   (PRECISION: 0 = FP64, 1 = FP32)
 * Inputs:  DIR/dims.txt ("n m"), DIR/P.bin (n*n), q.bin (n), A.bin (m*n), l.bin, u.bin (m)
 * Outputs: DIR/x.bin (n), z.bin, y.bin (m) as FP64; DIR/info.txt ("iterations status" and the
 *          penalty index after each check). Exit status 0 on success. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "relu_qp.h"

static double* read_f64(const char* dir, const char* name, size_t count) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  double* v = (double*)malloc(count * sizeof(double));
  if (v && fread(v, sizeof(double), count, f) != count) {
    free(v);
    v = NULL;
  }
  fclose(f);
  return v;
}

static int write_f64(const char* dir, const char* name, const double* v, size_t count) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "wb");
  if (!f) return 1;
  const int bad = fwrite(v, sizeof(double), count, f) != count;
  fclose(f);
  return bad;
}

/* device buffer of `count` elements of `size` bytes, copied back as FP64 */
static int to_host_f64(const void* dev, size_t count, int fp64, double* out) {
  if (fp64) return hipMemcpy(out, dev, count * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
  float* tmp = (float*)malloc(count * sizeof(float));
  if (!tmp) return 1;
  int bad = hipMemcpy(tmp, dev, count * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess;
  for (size_t i = 0; i < count && !bad; ++i) out[i] = tmp[i];
  free(tmp);
  return bad;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s DIR MAX_ITER PRECISION\n", argv[0]);
    return 2;
  }
  const char* dir = argv[1];
  const int max_iter = atoi(argv[2]), fp64 = atoi(argv[3]) == 0;
  char path[4096];
  snprintf(path, sizeof path, "%s/dims.txt", dir);
  FILE* fd = fopen(path, "r");
  int n = 0, m = 0;
  if (!fd || fscanf(fd, "%d %d", &n, &m) != 2 || n < 1 || m < 1) {
    fprintf(stderr, "bad %s\n", path);
    return 2;
  }
  fclose(fd);
  double *P = read_f64(dir, "P.bin", (size_t)n * n), *q = read_f64(dir, "q.bin", n);
  double *A = read_f64(dir, "A.bin", (size_t)m * n), *l = read_f64(dir, "l.bin", m), *u = read_f64(dir, "u.bin", m);
  if (!P || !q || !A || !l || !u) {
    fprintf(stderr, "missing input files in %s\n", dir);
    return 2;
  }

  relu_qp_settings s;
  relu_qp_default_settings(&s);
  s.precision = fp64 ? RQP_FP64 : RQP_FP32;
  s.engine = RQP_ENGINE_SINGLE;
  s.n_rho = 8;
  s.eps_abs = 0.0;
  s.eps_rel = 0.0;
  s.max_iter = max_iter;
  relu_qp_handle* h = NULL;
  if (relu_qp_setup(&h, n, m, P, q, A, l, u, &s, NULL) != RQP_OK) {
    fprintf(stderr, "relu_qp_setup: %s\n", relu_qp_last_error());
    return 1;
  }
  const int checks = relu_qp_max_checks(h);
  const size_t es = fp64 ? sizeof(double) : sizeof(float);
  relu_qp_result out;
  memset(&out, 0, sizeof out);
  if (hipMalloc(&out.x, n * es) != hipSuccess || hipMalloc(&out.y, m * es) != hipSuccess ||
      hipMalloc(&out.z, m * es) != hipSuccess || hipMalloc((void**)&out.iterations, sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&out.status, sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&out.rho_index, sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&out.rho_hist, checks * sizeof(int)) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  if (relu_qp_solve(h, NULL, &out) != RQP_OK || hipDeviceSynchronize() != hipSuccess) {
    fprintf(stderr, "relu_qp_solve: %s\n", relu_qp_last_error());
    return 1;
  }
  double *x = (double*)malloc(n * sizeof(double)), *y = (double*)malloc(m * sizeof(double));
  double* z = (double*)malloc(m * sizeof(double));
  int it = 0, st = 0;
  int* hist = (int*)malloc(checks * sizeof(int));
  if (!x || !y || !z || !hist || to_host_f64(out.x, n, fp64, x) || to_host_f64(out.y, m, fp64, y) ||
      to_host_f64(out.z, m, fp64, z) ||
      hipMemcpy(&it, out.iterations, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&st, out.status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hist, out.rho_hist, checks * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "copies back failed\n");
    return 1;
  }
  if (write_f64(dir, "x.bin", x, n) || write_f64(dir, "z.bin", z, m) || write_f64(dir, "y.bin", y, m)) return 1;
  snprintf(path, sizeof path, "%s/info.txt", dir);
  FILE* fi = fopen(path, "w");
  if (!fi) return 1;
  fprintf(fi, "%d %d\n", it, st);
  const int done = (it + s.check_interval - 1) / s.check_interval;
  for (int c = 0; c < done && c < checks; ++c) fprintf(fi, "%d ", hist[c]);
  fprintf(fi, "\n");
  fclose(fi);
  relu_qp_cleanup(h);
  hipFree(out.x);
  hipFree(out.y);
  hipFree(out.z);
  hipFree(out.iterations);
  hipFree(out.status);
  hipFree(out.rho_index);
  hipFree(out.rho_hist);
  free(P), free(q), free(A), free(l), free(u), free(x), free(y), free(z), free(hist);
  printf("relu_qp_example: n=%d m=%d iterations=%d status=%d\n", n, m, it, st);
  return 0;
}
