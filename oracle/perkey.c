/*
 * Per-key parallel checker -- TEST INFRASTRUCTURE ONLY (part of the oracle).
 *
 * Same question as the serial replay in oracle.c: do the committed
 * transactions, executed one at a time in their reported serial order from
 * the initial tables, reproduce every reported read value and the final
 * tables?  (Serializable isolation, Section 3 "CC Schemes Migration and
 * Implementation" and Section 4.1 "CC Scheme Selection".)
 *
 * Every operation touches one cell (table, row, field), and a cell appears at
 * most once per transaction.  The value a READ, ADD or COND_ADD leaves in its
 * cell depends only on that cell's previous value and the operation's own
 * argument, so the history of each cell can be replayed on its own: the
 * operations on the cell, in serial order, starting from its initial value.
 * A WRITE_SLOT's new value also needs the value its source operation read;
 * the checker takes the value the run reported for the source, which is
 * itself checked on the source's own cell.  By induction over the serial
 * order, every reported read and every final cell agrees with the per-cell
 * replays exactly when it agrees with the serial replay, so this check and
 * the serial one accept and reject the same runs.
 *
 * Cells are independent, so the work is split over host threads (OpenMP):
 * the committed transactions' operations are scattered into buckets by a
 * hash of their cell, each bucket is sorted by (cell, serial rank) and its
 * cells replayed; cells no committed operation touches must keep their
 * initial values.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PK_OK 0
#define PK_E_RANGE (-2)
#define PK_E_KIND (-3)
#define PK_E_SRC (-4)
#define PK_E_NOMEM (-5)
#define PK_E_ARG (-6)
#define PK_E_DUPKEY (-7)

enum { PK_READ = 0, PK_ADD = 1, PK_COND_ADD = 2, PK_WRITE_SLOT = 3 };

typedef struct {
  uint64_t hi, lo;
  uint32_t txn;
} keyed_txn;

typedef struct {
  uint64_t cell;  /* global cell index: the table's first cell + row * fields + field */
  int64_t src;    /* WRITE_SLOT: the value its source operation reported as read */
  uint32_t rank;  /* position of the transaction in the serial order */
  uint32_t op;    /* operation index in the batch */
} entry;

static int cmp_key(const void *a, const void *b) {
  const keyed_txn *x = (const keyed_txn *)a, *y = (const keyed_txn *)b;
  if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
  if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
  return 0;
}

static int cmp_entry(const void *a, const void *b) {
  const entry *x = (const entry *)a, *y = (const entry *)b;
  if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
  return x->rank < y->rank ? -1 : (x->rank > y->rank);
}

static uint64_t hash_cell(uint64_t c) {
  c ^= c >> 33;
  c *= 0xff51afd7ed558ccdull;
  c ^= c >> 33;
  return c;
}

/* New value of a cell from its previous value (the pre-image). */
static int64_t apply(uint8_t kind, int64_t pre, int64_t arg, int64_t src) {
  switch (kind) {
    case PK_ADD:
      return (int64_t)((uint64_t)pre + (uint64_t)arg);
    case PK_COND_ADD: {
      int64_t v = (int64_t)((uint64_t)pre + (uint64_t)arg);
      return v < 10 ? (int64_t)((uint64_t)v + 91u) : v;
    }
    case PK_WRITE_SLOT: {
      uint64_t a = (uint64_t)arg;
      int64_t mul = (int64_t)((a >> 8) & 0xFFFFFFu);
      if (mul & 0x800000) mul -= 0x1000000;
      int64_t add = (int64_t)(int32_t)(uint32_t)(a >> 32);
      return (int64_t)((uint64_t)src * (uint64_t)mul + (uint64_t)add);
    }
    default:
      return pre;
  }
}

/*
 * Check a run.  status / serial_hi / serial_lo: per transaction (status 1 =
 * committed); got_reads: per op; init / final: per table, row-major.
 * n_threads <= 0 uses OpenMP's default.  out[0] = read mismatches, out[1] =
 * cell mismatches, out[2] = lowest mismatching op (or -1), out[3] = lowest
 * mismatching global cell (or -1), out[4] = committed transactions, out[5] =
 * threads used.  Returns 0, PK_E_DUPKEY if two committed transactions share a
 * serial key, or another negative code on malformed input.
 */
int oracle_perkey_check(uint32_t n_tables, const uint64_t *n_rows, const uint32_t *n_fields,
                        int64_t *const *init, int64_t *const *final_, const uint64_t *first_op,
                        const uint32_t *n_ops, const uint32_t *row, const uint16_t *table, const uint8_t *field,
                        const uint8_t *kind, const int64_t *arg, uint64_t n_txns, uint64_t total_ops,
                        const uint32_t *status, const uint64_t *serial_hi, const uint64_t *serial_lo,
                        const int64_t *got_reads, int n_threads, int64_t *out) {
  if (n_tables == 0 || n_tables > 64 || n_txns > 0xFFFFFFFFull || total_ops > 0xFFFFFFFFull) return PK_E_ARG;
  if (n_threads <= 0) n_threads = omp_get_max_threads();
  uint64_t base[65];
  base[0] = 0;
  for (uint32_t t = 0; t < n_tables; ++t) base[t + 1] = base[t] + n_rows[t] * n_fields[t];
  const uint64_t n_cells = base[n_tables];

  /* 1. serial rank of every committed transaction */
  uint64_t n_comm = 0;
  for (uint64_t t = 0; t < n_txns; ++t) n_comm += status[t] == 1;
  keyed_txn *kt = (keyed_txn *)malloc((n_comm ? n_comm : 1) * sizeof(keyed_txn));
  uint32_t *rank = (uint32_t *)malloc((n_txns ? n_txns : 1) * sizeof(uint32_t));
  if (!kt || !rank) { free(kt); free(rank); return PK_E_NOMEM; }
  uint64_t k = 0;
  for (uint64_t t = 0; t < n_txns; ++t)
    if (status[t] == 1) { kt[k].hi = serial_hi[t]; kt[k].lo = serial_lo[t]; kt[k].txn = (uint32_t)t; ++k; }
  qsort(kt, n_comm, sizeof(keyed_txn), cmp_key);
  for (uint64_t i = 0; i < n_txns; ++i) rank[i] = 0xFFFFFFFFu;
  for (uint64_t i = 0; i < n_comm; ++i) {
    if (i && kt[i].hi == kt[i - 1].hi && kt[i].lo == kt[i - 1].lo) { free(kt); free(rank); return PK_E_DUPKEY; }
    rank[kt[i].txn] = (uint32_t)i;
  }
  free(kt);

  /* 2. scatter the committed operations into buckets by cell (two passes,
        the same static split of transactions over threads in both) */
  const int nb_log = 14;
  const uint64_t NB = 1ull << nb_log;
  uint64_t *cnt = (uint64_t *)calloc((size_t)n_threads * NB, sizeof(uint64_t));
  uint64_t *start = (uint64_t *)malloc((NB + 1) * sizeof(uint64_t));
  if (!cnt || !start) { free(cnt); free(start); free(rank); return PK_E_NOMEM; }
  int bad_input = 0;
#pragma omp parallel num_threads(n_threads) reduction(| : bad_input)
  {
    const int me = omp_get_thread_num(), nt = omp_get_num_threads();
    const uint64_t lo = n_txns * (uint64_t)me / (uint64_t)nt, hi = n_txns * (uint64_t)(me + 1) / (uint64_t)nt;
    uint64_t *c = cnt + (size_t)me * NB;
    for (uint64_t t = lo; t < hi; ++t) {
      if (rank[t] == 0xFFFFFFFFu) continue;
      for (uint32_t i = 0; i < n_ops[t]; ++i) {
        const uint64_t op = first_op[t] + i;
        if (op >= total_ops || table[op] >= n_tables || row[op] >= n_rows[table[op]] ||
            field[op] >= n_fields[table[op]] || kind[op] > PK_WRITE_SLOT) {
          bad_input = 1;
          continue;
        }
        const uint64_t cell = base[table[op]] + (uint64_t)row[op] * n_fields[table[op]] + field[op];
        ++c[hash_cell(cell) & (NB - 1)];
      }
    }
  }
  if (bad_input) { free(cnt); free(start); free(rank); return PK_E_RANGE; }
  /* bucket starts, and each thread's offset inside each bucket */
  uint64_t total = 0;
  for (uint64_t b = 0; b < NB; ++b) {
    start[b] = total;
    for (int th = 0; th < n_threads; ++th) {
      const uint64_t v = cnt[(size_t)th * NB + b];
      cnt[(size_t)th * NB + b] = total;
      total += v;
    }
  }
  start[NB] = total;
  entry *e = (entry *)malloc((total ? total : 1) * sizeof(entry));
  if (!e) { free(cnt); free(start); free(rank); return PK_E_NOMEM; }
  int bad_src = 0;
#pragma omp parallel num_threads(n_threads) reduction(| : bad_src)
  {
    const int me = omp_get_thread_num(), nt = omp_get_num_threads();
    const uint64_t lo = n_txns * (uint64_t)me / (uint64_t)nt, hi = n_txns * (uint64_t)(me + 1) / (uint64_t)nt;
    uint64_t *c = cnt + (size_t)me * NB;
    for (uint64_t t = lo; t < hi; ++t) {
      if (rank[t] == 0xFFFFFFFFu) continue;
      for (uint32_t i = 0; i < n_ops[t]; ++i) {
        const uint64_t op = first_op[t] + i;
        const uint64_t cell = base[table[op]] + (uint64_t)row[op] * n_fields[table[op]] + field[op];
        entry x;
        x.cell = cell;
        x.rank = rank[t];
        x.op = (uint32_t)op;
        x.src = 0;
        if (kind[op] == PK_WRITE_SLOT) {
          const uint32_t s = (uint32_t)((uint64_t)arg[op] & 0xFFu);
          if (s >= i) bad_src = 1;
          else x.src = got_reads[first_op[t] + s];
        }
        e[c[hash_cell(cell) & (NB - 1)]++] = x;
      }
    }
  }
  free(cnt);
  free(rank);
  if (bad_src) { free(e); free(start); return PK_E_SRC; }

  /* 3. replay every touched cell on its own */
  int64_t read_bad = 0, cell_bad = 0, touched_changed = 0;
  int64_t first_bad_op = INT64_MAX, first_bad_cell = INT64_MAX;
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 16) \
    reduction(+ : read_bad, cell_bad, touched_changed) reduction(min : first_bad_op, first_bad_cell)
  for (uint64_t b = 0; b < NB; ++b) {
    entry *x = e + start[b];
    const uint64_t n = start[b + 1] - start[b];
    qsort(x, n, sizeof(entry), cmp_entry);
    uint64_t i = 0;
    while (i < n) {
      const uint64_t cell = x[i].cell;
      uint32_t t = 0;
      while (base[t + 1] <= cell) ++t;
      const uint64_t local = cell - base[t];
      int64_t cur = init[t][local];
      for (; i < n && x[i].cell == cell; ++i) {
        const uint32_t op = x[i].op;
        if (got_reads[op] != cur) {
          ++read_bad;
          if ((int64_t)op < first_bad_op) first_bad_op = op;
        }
        cur = apply(kind[op], cur, arg[op], x[i].src);
      }
      if (final_[t][local] != cur) {
        ++cell_bad;
        if ((int64_t)cell < first_bad_cell) first_bad_cell = (int64_t)cell;
      }
      touched_changed += final_[t][local] != init[t][local];
    }
  }
  free(e);
  free(start);

  /* 4. cells nothing committed touched keep their initial values:
        (all changed cells) - (changed touched cells) must be 0 */
  int64_t changed = 0;
  for (uint32_t t = 0; t < n_tables; ++t) {
    const uint64_t m = n_rows[t] * n_fields[t];
    const int64_t *a = init[t], *f = final_[t];
#pragma omp parallel for num_threads(n_threads) schedule(static) reduction(+ : changed)
    for (uint64_t j = 0; j < m; ++j) changed += a[j] != f[j];
  }
  cell_bad += changed - touched_changed;
  (void)n_cells;
  out[0] = read_bad;
  out[1] = cell_bad;
  out[2] = first_bad_op == INT64_MAX ? -1 : first_bad_op;
  out[3] = first_bad_cell == INT64_MAX ? -1 : first_bad_cell;
  out[4] = (int64_t)n_comm;
  out[5] = n_threads;
  return PK_OK;
}
