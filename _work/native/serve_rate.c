/* Native closed-loop load against the GPU server through the public C API (include/tabnet.h):
 * T threads each submit N requests of 1..MAXR rows back to back (outputs into a per-thread
 * ring, drained when full), then wait; prints requests/s and the server's statistics.  It
 * measures the server's capacity, not latency (requests queue into large launches).
 *
 * build: gcc -std=c99 -O2 -D_POSIX_C_SOURCE=199309L -I include tests/native/serve_rate.c \
 *            -o serve_rate -L paper_2510_19689_amd -ltabnet -Wl,-rpath,<repo>/paper_2510_19689_amd -pthread
 * usage: serve_rate <model.tnw (BF16 is loaded)> <threads> <requests per thread> <max rows> */
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include "tabnet.h"

static tabnet_server* srv;
static int N, MAXR, D = 108, NOUT = 2;
static float* X;

static double now_s(void) { struct timespec t; clock_gettime(CLOCK_MONOTONIC, &t); return t.tv_sec + 1e-9 * t.tv_nsec; }

static void* worker(void* arg) {
  unsigned seed = (unsigned)(size_t)arg * 7919u + 1u;
  const size_t ring_rows = 1u << 20;
  float* lo = malloc(ring_rows * NOUT * sizeof(float));
  float* ag = malloc(ring_rows * D * sizeof(float));
  uint64_t* ids = malloc(sizeof(uint64_t) * (size_t)N);
  size_t off = 0, nid = 0;
  for (int k = 0; k < N; ++k) {
    seed = seed * 1103515245u + 12345u;
    int rows = 1 + (int)((seed >> 8) % (unsigned)MAXR);
    if (off + (size_t)rows > ring_rows) {
      for (size_t i = 0; i < nid; ++i) tabnet_serve_wait(srv, ids[i], -1);
      nid = 0; off = 0;
    }
    uint64_t id;
    if (tabnet_serve_submit(srv, 0, X, rows, lo + off * NOUT, ag + off * D, NULL, 0, &id) == TABNET_OK) ids[nid++] = id;
    off += (size_t)rows;
  }
  for (size_t i = 0; i < nid; ++i) tabnet_serve_wait(srv, ids[i], -1);
  free(lo); free(ag); free(ids);
  return NULL;
}

int main(int argc, char** argv) {
  if (argc < 5) return 2;
  int T = atoi(argv[2]); N = atoi(argv[3]); MAXR = atoi(argv[4]);
  tabnet_handle* h = NULL;
  if (tabnet_load(argv[1], TABNET_BF16, 0, &h) != TABNET_OK) { printf("load: %s\n", tabnet_last_error()); return 3; }
  X = malloc((size_t)MAXR * D * sizeof(float));
  for (int i = 0; i < MAXR * D; ++i) X[i] = (float)((i * 37) % 101) / 50.0f - 1.0f;
  if (tabnet_serve_start(&h, 1, NULL, &srv) != TABNET_OK) { printf("start: %s\n", tabnet_last_error()); return 4; }
  pthread_t th[64];
  double t0 = now_s();
  for (int t = 0; t < T; ++t) pthread_create(&th[t], NULL, worker, (void*)(size_t)t);
  for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
  double sec = now_s() - t0;
  tabnet_serve_stats st;
  tabnet_serve_get_stats(srv, &st);
  printf("[native] threads %d maxrows %d: %.0f req/s, %.2f M rows/s, launches %llu, rows/launch %.0f, p50 %.3f ms, p99 %.3f ms\n",
         T, MAXR, (double)st.completed / sec, (double)st.rows_completed / sec / 1e6, (unsigned long long)st.launches,
         (double)st.rows_completed / (double)st.launches, st.p50_us / 1e3, st.p99_us / 1e3);
  tabnet_serve_stop(srv);
  tabnet_free(h);
  return 0;
}
