/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE: runs the oracle's setup, V-cycle
 * and PCG on inputs read from one binary file, so that the oracle can be built
 * and run under AddressSanitizer / UndefinedBehaviorSanitizer in a plain C
 * process (tests/test_oracle_sanitized.py writes the file and checks the run).
 *
 * File layout (native endianness): int32 n, int64 nnzb, int32 ntv,
 * int64 rp[n+1], int32 ci[nnzb], double v[nnzb*9], double V0[n*3*ntv],
 * double f[n*3].  Argument 2: SRQCG iterations per level (n_rq).
 * Prints "iterations <k> status <s> relres <r>".  The oracle's source is
 * included so that its parameter block is known here.
 */
#include "aspamg_oracle.c"

static void *read_n(FILE *fp, size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, fp) != bytes) {
    fprintf(stderr, "short read\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *fp = fopen(argv[1], "rb");
  if (!fp) return 2;
  int32_t n, ntv;
  int64_t nnzb;
  if (fread(&n, 4, 1, fp) != 1 || fread(&nnzb, 8, 1, fp) != 1 || fread(&ntv, 4, 1, fp) != 1) return 2;
  int64_t *rp = read_n(fp, (size_t)(n + 1) * 8);
  int32_t *ci = read_n(fp, (size_t)nnzb * 4);
  double *v = read_n(fp, (size_t)nnzb * 9 * 8);
  double *V0 = read_n(fp, (size_t)n * 3 * ntv * 8);
  double *f = read_n(fp, (size_t)n * 3 * 8);
  fclose(fp);
  oparams params;
  oracle_default_params(&params);
  params.n_rq = atoi(argv[2]);
  ohier *h = NULL;
  int rc = oracle_setup(&params, n, rp, ci, v, ntv, V0, &h);
  if (rc < 0) {
    printf("setup failed %d\n", rc);
    return 3;
  }
  double *z = calloc((size_t)n * 3, 8), *u = calloc((size_t)n * 3, 8);
  oracle_vcycle(h, f, z);
  int32_t it = 0;
  double rr = 0.0;
  rc = oracle_pcg(h, f, u, 1e-10, 500, &it, &rr);
  printf("iterations %d status %d relres %.3e\n", it, rc, rr);
  oracle_free(h);
  free(rp); free(ci); free(v); free(V0); free(f); free(z); free(u);
  return rc == 0 ? 0 : 4;
}
