/* A C client of the serving API (include/tabnet.h), built and run by tests/test_gpu_c_serve.py.
 *
 * T threads submit N requests each, of 1..MAXR rows taken from the start of one shared
 * input matrix, back to back, and wait for them.  Rows are independent, so row i of every
 * request must carry exactly (bit for bit) the outputs of row i of every other request:
 * the first completed request that covers row i is the reference.  Every mask row must be
 * finite, non-negative and sum to 1.  Exit status 0 when all checks pass.
 *
 * usage: serve_load <model.tnw> <threads> <requests per thread> <max rows> */
#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "tabnet.h"

static tabnet_server* srv;
static int N, MAXR, D, NOUT;
static float* X;
static float *ref_lo, *ref_ag;     /* reference outputs per row, filled under ref_lock */
static int* ref_set;
static pthread_mutex_t ref_lock = PTHREAD_MUTEX_INITIALIZER;
static int failures;

static int check_rows(const float* lo, const float* ag, int rows) {
  int bad = 0;
  for (int r = 0; r < rows; ++r) {
    double sum = 0;
    for (int j = 0; j < D; ++j) {
      const float v = ag[(size_t)r * D + j];
      if (!isfinite(v) || v < 0.f) ++bad;
      sum += v;
    }
    if (fabs(sum - 1.0) > 2e-5) ++bad;
    for (int o = 0; o < NOUT; ++o)
      if (!isfinite(lo[(size_t)r * NOUT + o])) ++bad;
    pthread_mutex_lock(&ref_lock);
    if (!ref_set[r]) {
      memcpy(ref_lo + (size_t)r * NOUT, lo + (size_t)r * NOUT, sizeof(float) * NOUT);
      memcpy(ref_ag + (size_t)r * D, ag + (size_t)r * D, sizeof(float) * D);
      ref_set[r] = 1;
    } else if (memcmp(ref_lo + (size_t)r * NOUT, lo + (size_t)r * NOUT, sizeof(float) * NOUT) != 0 ||
               memcmp(ref_ag + (size_t)r * D, ag + (size_t)r * D, sizeof(float) * D) != 0) {
      ++bad;
    }
    pthread_mutex_unlock(&ref_lock);
  }
  return bad;
}

static void* worker(void* arg) {
  unsigned seed = (unsigned)(size_t)arg * 7919u + 1u;
  int* rows = malloc(sizeof(int) * (size_t)N);
  size_t* offs = malloc(sizeof(size_t) * (size_t)N);
  uint64_t* ids = malloc(sizeof(uint64_t) * (size_t)N);
  size_t total = 0;
  for (int k = 0; k < N; ++k) {
    seed = seed * 1103515245u + 12345u;
    rows[k] = 1 + (int)((seed >> 8) % (unsigned)MAXR);
    offs[k] = total;
    total += (size_t)rows[k];
  }
  float* lo = malloc(total * (size_t)NOUT * sizeof(float));
  float* ag = malloc(total * (size_t)D * sizeof(float));
  int bad = 0;
  for (int k = 0; k < N; ++k)
    if (tabnet_serve_submit(srv, 0, X, rows[k], lo + offs[k] * NOUT, ag + offs[k] * D, NULL, 0, &ids[k]) != TABNET_OK) {
      fprintf(stderr, "submit failed: %s\n", tabnet_last_error());
      ++bad;
      ids[k] = 0;
    }
  for (int k = 0; k < N; ++k) {
    if (ids[k] == 0) continue;
    if (tabnet_serve_wait(srv, ids[k], -1) != TABNET_OK) {
      ++bad;
      continue;
    }
    bad += check_rows(lo + offs[k] * NOUT, ag + offs[k] * D, rows[k]);
  }
  pthread_mutex_lock(&ref_lock);
  failures += bad;
  pthread_mutex_unlock(&ref_lock);
  free(rows); free(offs); free(ids); free(lo); free(ag);
  return NULL;
}

int main(int argc, char** argv) {
  if (argc < 5) return 2;
  const int T = atoi(argv[2]);
  N = atoi(argv[3]);
  MAXR = atoi(argv[4]);
  if (T < 1 || T > 16 || N < 1 || MAXR < 1) return 2;
  tabnet_handle* h = NULL;
  if (tabnet_load(argv[1], TABNET_BF16, 0, &h) != TABNET_OK) {
    fprintf(stderr, "load: %s\n", tabnet_last_error());
    return 3;
  }
  tabnet_config cfg;
  tabnet_get_config(h, &cfg);
  D = cfg.D;
  NOUT = cfg.n_out;
  X = malloc((size_t)MAXR * D * sizeof(float));
  for (size_t i = 0; i < (size_t)MAXR * D; ++i) X[i] = (float)((i * 37) % 101) / 50.0f - 1.0f;
  ref_lo = calloc((size_t)MAXR * NOUT, sizeof(float));
  ref_ag = calloc((size_t)MAXR * D, sizeof(float));
  ref_set = calloc((size_t)MAXR, sizeof(int));
  if (tabnet_serve_start(&h, 1, NULL, &srv) != TABNET_OK) {
    fprintf(stderr, "start: %s\n", tabnet_last_error());
    return 4;
  }
  pthread_t th[16];
  for (int t = 0; t < T; ++t) pthread_create(&th[t], NULL, worker, (void*)(size_t)t);
  for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
  tabnet_serve_stats st;
  tabnet_serve_get_stats(srv, &st);
  printf("completed %llu requests, %llu rows, %llu launches, failures %d\n", (unsigned long long)st.completed,
         (unsigned long long)st.rows_completed, (unsigned long long)st.launches, failures);
  tabnet_serve_stop(srv);
  tabnet_free(h);
  free(X); free(ref_lo); free(ref_ag); free(ref_set);
  return failures == 0 && st.completed == (unsigned long long)T * (unsigned long long)N ? 0 : 1;
}
