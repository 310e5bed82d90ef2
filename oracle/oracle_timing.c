/*
 * oracle_timing.c -- timing harness for the CPU baseline (TEST INFRASTRUCTURE ONLY).
 *
 * Runs the scalar oracle over one buffer or one batch and reports the fastest of
 * several repetitions, measured with CLOCK_MONOTONIC (a steady clock, as the paper's
 * own measurements use) around the work of every thread, each thread pinned to its
 * own CPU of the process affinity mask.  A warm-up repetition comes first, so every
 * timed repetition writes into output pages that are already mapped.
 *
 * With T > 1 threads a buffer is cut into T pieces at character boundaries: a UTF-8
 * cut backs up at most 3 bytes to a byte that is not a continuation byte, a UTF-16
 * cut never falls between a high surrogate and the word after it.  Every validation
 * rule is local to a character, so each piece's first error, taken at the smallest
 * offset, is the whole buffer's first error.  Piece k writes its output at the
 * output position of its first input unit times the worst-case expansion (1 word
 * per byte, 3 bytes per word), and the combined result is built from the pieces'
 * results: the first piece with an encoding error gives status and offset, written
 * = the pieces before it plus its own written.  A batch is cut into T runs of
 * consecutive items with about equal input bytes.
 *
 * This file calls only the oracle's public functions (utf_oracle.h).
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "utf_oracle.h"

enum { OP_U8_TO_U16 = 0, OP_U16_TO_U8 = 1, OP_VALIDATE_U8 = 2, OP_VALIDATE_U16 = 3, OP_BATCH = 4 };

#define MAX_THREADS 256

typedef struct {
  int op;
  const uint8_t *in;      /* buffer ops: the input; OP_BATCH: the input arena */
  uint8_t *out;           /* buffer ops: the output; OP_BATCH: the output arena */
  size_t in_bytes, out_bytes;
  const utfx_ref_item *items;
  utfx_ref_result *results;
  size_t lo, hi;          /* input units (buffer ops) or items (batch) of this thread */
  size_t out_cap;         /* output units of this thread's piece */
  utfx_ref_result r;      /* this thread's result (buffer ops) */
  int cpu;
  int reps;
  pthread_barrier_t *bar;
  uint64_t *ns;           /* per repetition, written by thread 0 */
  struct timespec *t0;
} job_t;

static uint64_t elapsed_ns(const struct timespec *a, const struct timespec *b) {
  return (uint64_t)(b->tv_sec - a->tv_sec) * 1000000000ull + (uint64_t)b->tv_nsec - (uint64_t)a->tv_nsec;
}

static void run_piece(job_t *j) {
  switch (j->op) {
    case OP_U8_TO_U16:
      j->r = utfx_ref_utf8_to_utf16le(j->in + j->lo, j->hi - j->lo, (uint16_t *)(void *)j->out + j->lo, j->out_cap);
      break;
    case OP_U16_TO_U8:
      j->r = utfx_ref_utf16le_to_utf8((const uint16_t *)(const void *)j->in + j->lo, j->hi - j->lo,
                                      j->out + 3 * j->lo, j->out_cap);
      break;
    case OP_VALIDATE_U8:
      j->r = utfx_ref_validate_utf8(j->in + j->lo, j->hi - j->lo);
      break;
    case OP_VALIDATE_U16:
      j->r = utfx_ref_validate_utf16le((const uint16_t *)(const void *)j->in + j->lo, j->hi - j->lo);
      break;
    default:
      utfx_ref_batch(j->in, j->in_bytes, j->out, j->out_bytes, j->items + j->lo, j->hi - j->lo, j->results + j->lo);
      break;
  }
}

static void *worker(void *arg) {
  job_t *j = (job_t *)arg;
  if (j->cpu >= 0) {
    cpu_set_t set;
    CPU_ZERO(&set);
    CPU_SET(j->cpu, &set);
    pthread_setaffinity_np(pthread_self(), sizeof(set), &set);
  }
  for (int r = 0; r <= j->reps; r++) {  /* repetition 0 is the warm-up */
    pthread_barrier_wait(j->bar);
    if (j->ns) clock_gettime(CLOCK_MONOTONIC, j->t0);
    run_piece(j);
    pthread_barrier_wait(j->bar);
    if (j->ns) {
      struct timespec t1;
      clock_gettime(CLOCK_MONOTONIC, &t1);
      j->ns[r] = elapsed_ns(j->t0, &t1);
    }
  }
  return 0;
}

/* CPUs of the process affinity mask, in order; returns how many (at most max). */
static int allowed_cpus(int *cpus, int max) {
  cpu_set_t set;
  int k = 0;
  if (sched_getaffinity(0, sizeof(set), &set) != 0) return 0;
  for (int c = 0; c < CPU_SETSIZE && k < max; c++)
    if (CPU_ISSET(c, &set)) cpus[k++] = c;
  return k;
}

static int is_cont(uint8_t b) { return b >= 0x80 && b <= 0xBF; }

/* Piece boundaries of a buffer op: cuts[0] = 0, cuts[t] = n. */
static void cut_buffer(int op, const uint8_t *in, size_t n, int t, size_t *cuts) {
  const int in16 = (op == OP_U16_TO_U8 || op == OP_VALIDATE_U16);
  const uint16_t *w = (const uint16_t *)(const void *)in;
  cuts[0] = 0;
  for (int k = 1; k < t; k++) {
    size_t b = (size_t)((unsigned __int128)n * (unsigned)k / (unsigned)t);
    if (in16) {
      if (b > 0 && b < n && w[b - 1] >= 0xD800 && w[b - 1] <= 0xDBFF) b--;
    } else {
      for (int back = 0; back < 3 && b > 0 && b < n && is_cont(in[b]); back++) b--;
    }
    if (b < cuts[k - 1]) b = cuts[k - 1];
    cuts[k] = b;
  }
  cuts[t] = n;
}

static int encoding_error(int32_t st) { return st >= UTFX_REF_E_STRAY_CONT && st <= UTFX_REF_E_BAD_BYTE; }

/* Times one op.  op 0..3: buffer ops over in[0:n] (units), with out of room
 * out_cap units (transcodes; must hold n words or 3n bytes when threads > 1).
 * threads: 0 = every CPU of the affinity mask.  Writes the fastest repetition (ns)
 * to *ns_min, the combined result to *result, the threads used to *threads_used and,
 * if piece_lo / piece_written are not NULL, each piece's first unit and output units
 * written (at most MAX_THREADS entries).  Returns 0, or -1 on a bad argument. */
int utfx_ref_time_buffer(int op, const void *in, size_t n, void *out, size_t out_cap, int threads, int reps,
                         uint64_t *ns_min, utfx_ref_result *result, int *threads_used, uint64_t *piece_lo,
                         uint64_t *piece_written) {
  int cpus[MAX_THREADS];
  int nc = allowed_cpus(cpus, MAX_THREADS);
  if (op < OP_U8_TO_U16 || op > OP_VALIDATE_U16 || reps < 1 || (n > 0 && !in)) return -1;
  int t = threads > 0 ? threads : (nc > 0 ? nc : 1);
  if (t > MAX_THREADS) t = MAX_THREADS;
  if ((size_t)t > n && n > 0) t = (int)n;
  if (t < 1) t = 1;
  const int transcode = (op == OP_U8_TO_U16 || op == OP_U16_TO_U8);
  const size_t expand = op == OP_U16_TO_U8 ? 3 : 1;
  if (transcode && t > 1 && out_cap < expand * n) return -1;
  size_t cuts[MAX_THREADS + 1];
  cut_buffer(op, (const uint8_t *)in, n, t, cuts);
  job_t jobs[MAX_THREADS];
  pthread_t tid[MAX_THREADS];
  pthread_barrier_t bar;
  struct timespec t0;
  uint64_t *ns = (uint64_t *)calloc((size_t)reps + 1, sizeof(uint64_t));
  if (!ns) return -1;
  pthread_barrier_init(&bar, 0, (unsigned)t);
  for (int k = 0; k < t; k++) {
    job_t *j = &jobs[k];
    memset(j, 0, sizeof(*j));
    j->op = op;
    j->in = (const uint8_t *)in;
    j->out = (uint8_t *)out;
    j->lo = cuts[k];
    j->hi = cuts[k + 1];
    j->out_cap = t == 1 ? out_cap : expand * (j->hi - j->lo);
    j->cpu = nc > 0 ? cpus[k % nc] : -1;
    j->reps = reps;
    j->bar = &bar;
    j->ns = k == 0 ? ns : 0;
    j->t0 = &t0;
  }
  cpu_set_t caller;
  const int have_caller = pthread_getaffinity_np(pthread_self(), sizeof(caller), &caller) == 0;
  for (int k = 1; k < t; k++) pthread_create(&tid[k], 0, worker, &jobs[k]);
  worker(&jobs[0]);  /* the calling thread runs piece 0, pinned like the others */
  for (int k = 1; k < t; k++) pthread_join(tid[k], 0);
  if (have_caller) pthread_setaffinity_np(pthread_self(), sizeof(caller), &caller);
  pthread_barrier_destroy(&bar);
  uint64_t best = ns[1];
  for (int r = 2; r <= reps; r++)
    if (ns[r] < best) best = ns[r];
  free(ns);
  /* combine the pieces */
  utfx_ref_result c = {UTFX_REF_OK, 0, 0, 0};
  uint64_t total = 0;
  int err_piece = -1;
  for (int k = 0; k < t; k++) {
    if (encoding_error(jobs[k].r.status)) {
      err_piece = k;
      break;
    }
    total += jobs[k].r.count;
  }
  if (err_piece >= 0) {
    const utfx_ref_result r = jobs[err_piece].r;
    c.status = r.status;
    c.count = cuts[err_piece] + r.count;
    c.written = transcode ? total + r.written : c.count;
  } else if (transcode) {
    c.status = total > out_cap ? UTFX_REF_E_OUTPUT_TOO_SMALL : UTFX_REF_OK;
    c.count = total;
    c.written = c.status == UTFX_REF_OK ? total : 0;
  } else {
    c.count = c.written = n;
  }
  *ns_min = best;
  *result = c;
  *threads_used = t;
  for (int k = 0; k < t; k++) {
    if (piece_lo) piece_lo[k] = cuts[k];
    if (piece_written) piece_written[k] = encoding_error(jobs[k].r.status) ? jobs[k].r.written : jobs[k].r.count;
  }
  return 0;
}

/* Times utfx_ref_batch over n_items items (threads as above; runs of consecutive
 * items with about equal input bytes).  Results go to results[]; returns the number
 * of OK items through *n_ok. */
int utfx_ref_time_batch(const uint8_t *in_arena, size_t in_bytes, uint8_t *out_arena, size_t out_bytes,
                        const utfx_ref_item *items, size_t n_items, utfx_ref_result *results, int threads, int reps,
                        uint64_t *ns_min, int *threads_used, uint64_t *n_ok) {
  int cpus[MAX_THREADS];
  int nc = allowed_cpus(cpus, MAX_THREADS);
  if (reps < 1 || (n_items > 0 && (!items || !results))) return -1;
  int t = threads > 0 ? threads : (nc > 0 ? nc : 1);
  if (t > MAX_THREADS) t = MAX_THREADS;
  if ((size_t)t > n_items && n_items > 0) t = (int)n_items;
  if (t < 1) t = 1;
  uint64_t bytes = 0;
  for (size_t i = 0; i < n_items; i++) bytes += items[i].in_len * (items[i].dir == 1 ? 2 : 1);
  size_t cuts[MAX_THREADS + 1];
  cuts[0] = 0;
  {
    uint64_t acc = 0;
    size_t i = 0;
    for (int k = 1; k < t; k++) {
      const uint64_t want = (uint64_t)((unsigned __int128)bytes * (unsigned)k / (unsigned)t);
      while (i < n_items && acc < want) {
        acc += items[i].in_len * (items[i].dir == 1 ? 2 : 1);
        i++;
      }
      cuts[k] = i;
    }
    cuts[t] = n_items;
  }
  job_t jobs[MAX_THREADS];
  pthread_t tid[MAX_THREADS];
  pthread_barrier_t bar;
  struct timespec t0;
  uint64_t *ns = (uint64_t *)calloc((size_t)reps + 1, sizeof(uint64_t));
  if (!ns) return -1;
  pthread_barrier_init(&bar, 0, (unsigned)t);
  for (int k = 0; k < t; k++) {
    job_t *j = &jobs[k];
    memset(j, 0, sizeof(*j));
    j->op = OP_BATCH;
    j->in = in_arena;
    j->out = out_arena;
    j->in_bytes = in_bytes;
    j->out_bytes = out_bytes;
    j->items = items;
    j->results = results;
    j->lo = cuts[k];
    j->hi = cuts[k + 1];
    j->cpu = nc > 0 ? cpus[k % nc] : -1;
    j->reps = reps;
    j->bar = &bar;
    j->ns = k == 0 ? ns : 0;
    j->t0 = &t0;
  }
  cpu_set_t caller;
  const int have_caller = pthread_getaffinity_np(pthread_self(), sizeof(caller), &caller) == 0;
  for (int k = 1; k < t; k++) pthread_create(&tid[k], 0, worker, &jobs[k]);
  worker(&jobs[0]);  /* the calling thread runs piece 0, pinned like the others */
  for (int k = 1; k < t; k++) pthread_join(tid[k], 0);
  if (have_caller) pthread_setaffinity_np(pthread_self(), sizeof(caller), &caller);
  pthread_barrier_destroy(&bar);
  uint64_t best = ns[1];
  for (int r = 2; r <= reps; r++)
    if (ns[r] < best) best = ns[r];
  free(ns);
  uint64_t ok = 0;
  for (size_t i = 0; i < n_items; i++) ok += results[i].status == UTFX_REF_OK;
  *ns_min = best;
  *threads_used = t;
  *n_ok = ok;
  return 0;
}
