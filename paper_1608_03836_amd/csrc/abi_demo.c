/* A plain C consumer of libwadg.so: the sweep through the C ABI alone, with
 * no Python and no torch (the GPU tests run it and compare its output with
 * the Python binding's).
 *
 * usage: abi_demo IN OUT
 *   IN  (little-endian, packed): int32 N, nq1, K, S, nsteps, kernel;
 *       double dt, tau_p, tau_u; double x[K][(N+1)^2], y[K][(N+1)^2];
 *       int32 etoe[K][4], etof[K][4]; double Q0[S * slice] (tiled layout,
 *       slice = wadg_state_doubles).
 *   OUT double Q[S * slice] after nsteps LSRK steps of every slice, then
 *       double norms[S][4] (wadg_norms of Q against nothing).
 * Exit status 0 on success; otherwise the library's status text and detail
 * on stderr. */

#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "wadg.h"

static int check(int st, const char* what) {
  if (st != WADG_OK && st != WADG_E_NONFINITE) {
    fprintf(stderr, "%s: %s (%s)\n", what, wadg_status_string(st), wadg_last_error());
    exit(1);
  }
  return st;
}

static void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    exit(1);
  }
}

static void* read_n(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(1);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) {
    perror(argv[1]);
    return 1;
  }
  int32_t* hdr = (int32_t*)read_n(f, 6 * sizeof(int32_t));
  const int32_t N = hdr[0], nq1 = hdr[1], K = hdr[2], S = hdr[3], nsteps = hdr[4],
                kernel = hdr[5];
  double* sc = (double*)read_n(f, 3 * sizeof(double));
  const size_t np = (size_t)(N + 1) * (N + 1);
  double* x = (double*)read_n(f, (size_t)K * np * sizeof(double));
  double* y = (double*)read_n(f, (size_t)K * np * sizeof(double));
  int32_t* etoe = (int32_t*)read_n(f, (size_t)K * 4 * sizeof(int32_t));
  int32_t* etof = (int32_t*)read_n(f, (size_t)K * 4 * sizeof(int32_t));

  wadg_mesh m;
  m.N = N;
  m.nq1 = nq1;
  m.K = K;
  m.x = x;
  m.y = y;
  m.etoe = etoe;
  m.etof = etof;
  m.c2q = NULL;
  m.tau_p = sc[1];
  m.tau_u = sc[2];
  wadg_ctx ctx = NULL;
  check(wadg_create(&m, 0, &ctx), "wadg_create");
  check(wadg_set_kernel(ctx, kernel), "wadg_set_kernel");

  size_t slice = 0, wbytes = 0;
  check(wadg_state_doubles(ctx, &slice), "wadg_state_doubles");
  check(wadg_workspace_bytes(ctx, S, &wbytes), "wadg_workspace_bytes");
  const size_t qbytes = (size_t)S * slice * sizeof(double);
  double* q = (double*)read_n(f, qbytes);
  fclose(f);

  double *dq = NULL, *dw = NULL;
  hip_check(hipMalloc((void**)&dq, qbytes), "hipMalloc");
  hip_check(hipMalloc((void**)&dw, wbytes), "hipMalloc");
  hip_check(hipMemcpy(dq, q, qbytes, hipMemcpyHostToDevice), "hipMemcpy");
  check(wadg_integrate(ctx, dq, dw, S, sc[0], nsteps, NULL), "wadg_integrate");
  double* norms = (double*)malloc((size_t)S * 4 * sizeof(double));
  size_t nbytes = 0;
  void* dn = NULL;
  check(wadg_norms_workspace_bytes(ctx, S, &nbytes), "wadg_norms_workspace_bytes");
  hip_check(hipMalloc(&dn, nbytes), "hipMalloc");
  check(wadg_norms(ctx, dq, NULL, S, dn, nbytes, norms, NULL), "wadg_norms");
  hip_check(hipMemcpy(q, dq, qbytes, hipMemcpyDeviceToHost), "hipMemcpy");

  FILE* g = fopen(argv[2], "wb");
  if (!g || fwrite(q, 1, qbytes, g) != qbytes ||
      fwrite(norms, sizeof(double), (size_t)S * 4, g) != (size_t)S * 4) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    return 1;
  }
  fclose(g);
  hip_check(hipFree(dq), "hipFree");
  hip_check(hipFree(dw), "hipFree");
  hip_check(hipFree(dn), "hipFree");
  wadg_destroy(ctx);
  free(hdr);
  free(sc);
  free(x);
  free(y);
  free(etoe);
  free(etof);
  free(q);
  free(norms);
  return 0;
}
