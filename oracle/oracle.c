/*
 * CPU oracle for the batch transaction engine -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no code, header or constant table with
 * the HIP engine; it restates from the paper what a correct run must produce.
 *
 * What is checked.  Every concurrency-control scheme in the paper guarantees
 * serializable isolation (Section 3, opening of "CC Schemes Migration and
 * Implementation"; Section 4.1, "CC Scheme Selection").  A batch therefore has
 * a correct outcome exactly when some serial order of its committed
 * transactions, executed one at a time from the initial tables, reproduces
 * every value the run reported as read and the final tables.  Serial
 * execution is the textbook definition the paper relies on (Section 2,
 * "Concurrency control schemes ensure the isolation property ...").  The
 * batch model, its constraints (reads and writes only, no inserts or
 * deletes, read/write sets fixed in advance) and its retry-until-commit rule
 * are in Section 4.1, "Constraints" and "Experimental Procedure".
 *
 * The functions here:
 *   oracle_replay      executes a list of transactions serially, in the
 *                      given order, and records each operation's read value;
 *   oracle_bruteforce  tries every order of k <= 8 transactions and counts the
 *                      orders that reproduce given read values and tables.
 *
 * Operation semantics (one field of one row per operation; the pre-image is
 * the value reported as read for every kind):
 *   READ       value unchanged;
 *   ADD        value + arg (two's-complement wrap);
 *   COND_ADD   v = value + arg; if v < 10 then v = v + 91 -- the order-entry
 *              stock replenishing rule of TPC-C NewOrder, which the paper
 *              evaluates (Section 4.1, "Benchmark Selection");
 *   WRITE_SLOT value := read[src] * mul + add, where read[src] is what an
 *              earlier operation src of the same transaction read; arg packs
 *              src in bits 0-7, mul as a signed 24-bit number in bits 8-31
 *              and add as a signed 32-bit number in bits 32-63.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define E_RANGE (-2)
#define E_KIND (-3)
#define E_SRC (-4)
#define E_NOMEM (-5)
#define E_ARG (-6)

enum { K_READ = 0, K_ADD = 1, K_COND_ADD = 2, K_WRITE_SLOT = 3 };

typedef struct {
  uint32_t n_tables;
  const uint64_t *n_rows;
  const uint32_t *n_fields;
  int64_t **data; /* data[t][r * n_fields[t] + f] */
} tables_t;

typedef struct {
  const uint64_t *first_op;
  const uint32_t *n_ops;
  const uint32_t *row;
  const uint16_t *table;
  const uint8_t *field;
  const uint8_t *kind;
  const int64_t *arg;
} batch_t;

static int64_t add_wrap(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
static int64_t mul_wrap(int64_t a, int64_t b) { return (int64_t)((uint64_t)a * (uint64_t)b); }

/* Execute transaction t alone against the tables; record read values. */
static int run_one(const tables_t *db, const batch_t *b, uint64_t t, int64_t *reads) {
  uint64_t first = b->first_op[t];
  uint32_t n = b->n_ops[t];
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t op = first + i;
    uint32_t tab = b->table[op];
    if (tab >= db->n_tables) return E_RANGE;
    if (b->row[op] >= db->n_rows[tab] || b->field[op] >= db->n_fields[tab]) return E_RANGE;
    int64_t *cell = &db->data[tab][(uint64_t)b->row[op] * db->n_fields[tab] + b->field[op]];
    int64_t old = *cell;
    reads[op] = old;
    switch (b->kind[op]) {
      case K_READ:
        break;
      case K_ADD:
        *cell = add_wrap(old, b->arg[op]);
        break;
      case K_COND_ADD: {
        int64_t v = add_wrap(old, b->arg[op]);
        if (v < 10) v = add_wrap(v, 91);
        *cell = v;
        break;
      }
      case K_WRITE_SLOT: {
        uint64_t a = (uint64_t)b->arg[op];
        uint32_t src = (uint32_t)(a & 0xFFu);
        int64_t mul = (int64_t)((a >> 8) & 0xFFFFFFu);
        if (mul & 0x800000) mul -= 0x1000000;
        int64_t addend = (int64_t)(int32_t)(uint32_t)(a >> 32);
        if (src >= i) return E_SRC;
        *cell = add_wrap(mul_wrap(reads[first + src], mul), addend);
        break;
      }
      default:
        return E_KIND;
    }
  }
  return OK;
}

/*
 * Serially execute transactions order[0], order[1], ..., order[n_order-1]
 * (indices into the batch) against `data`, which is updated in place from the
 * initial tables to the final tables.  reads[op] receives the value each
 * operation of those transactions read; other entries are left untouched.
 * Returns 0, or a negative code on a malformed operation.
 */
int oracle_replay(uint32_t n_tables, const uint64_t *n_rows, const uint32_t *n_fields, int64_t **data,
                  const uint64_t *first_op, const uint32_t *n_ops, const uint32_t *row,
                  const uint16_t *table, const uint8_t *field, const uint8_t *kind, const int64_t *arg,
                  uint64_t n_txns, const int64_t *order, uint64_t n_order, int64_t *reads) {
  tables_t db = {n_tables, n_rows, n_fields, data};
  batch_t b = {first_op, n_ops, row, table, field, kind, arg};
  for (uint64_t k = 0; k < n_order; ++k) {
    if (order[k] < 0 || (uint64_t)order[k] >= n_txns) return E_ARG;
    int rc = run_one(&db, &b, (uint64_t)order[k], reads);
    if (rc) return rc;
  }
  return OK;
}

static int next_permutation(int64_t *p, int n) {
  int i = n - 2;
  while (i >= 0 && p[i] >= p[i + 1]) --i;
  if (i < 0) return 0;
  int j = n - 1;
  while (p[j] <= p[i]) --j;
  int64_t tmp = p[i]; p[i] = p[j]; p[j] = tmp;
  for (int a = i + 1, c = n - 1; a < c; ++a, --c) { tmp = p[a]; p[a] = p[c]; p[c] = tmp; }
  return 1;
}

/*
 * Count the serial orders of the k transactions in `txns` (k <= 8) that,
 * executed from the initial tables `init`, reproduce `got_reads` on every
 * operation of those transactions and end in exactly the tables `got_final`.
 * A correct (serializable) outcome has a count of at least one.  Returns the
 * count, or a negative code.
 */
int64_t oracle_bruteforce(uint32_t n_tables, const uint64_t *n_rows, const uint32_t *n_fields,
                          int64_t *const *init, int64_t *const *got_final,
                          const uint64_t *first_op, const uint32_t *n_ops, const uint32_t *row,
                          const uint16_t *table, const uint8_t *field, const uint8_t *kind,
                          const int64_t *arg, uint64_t n_txns, const int64_t *txns, int k,
                          const int64_t *got_reads, uint64_t total_ops) {
  if (k < 0 || k > 8) return E_ARG;
  for (int i = 0; i < k; ++i)
    if (txns[i] < 0 || (uint64_t)txns[i] >= n_txns) return E_ARG;
  int64_t **work = (int64_t **)calloc(n_tables ? n_tables : 1, sizeof(int64_t *));
  int64_t *reads = (int64_t *)malloc((total_ops ? total_ops : 1) * sizeof(int64_t));
  if (!work || !reads) { free(work); free(reads); return E_NOMEM; }
  for (uint32_t t = 0; t < n_tables; ++t) {
    work[t] = (int64_t *)malloc((n_rows[t] * n_fields[t] > 0 ? n_rows[t] * n_fields[t] : 1) * sizeof(int64_t));
    if (!work[t]) { for (uint32_t u = 0; u < t; ++u) free(work[u]); free(work); free(reads); return E_NOMEM; }
  }
  int64_t perm[8];
  for (int i = 0; i < k; ++i) perm[i] = i;
  int64_t order[8];
  int64_t matches = 0;
  do {
    for (uint32_t t = 0; t < n_tables; ++t)
      memcpy(work[t], init[t], n_rows[t] * n_fields[t] * sizeof(int64_t));
    for (int i = 0; i < k; ++i) order[i] = txns[perm[i]];
    tables_t db = {n_tables, n_rows, n_fields, work};
    batch_t b = {first_op, n_ops, row, table, field, kind, arg};
    int bad = 0;
    for (int i = 0; i < k && !bad; ++i)
      if (run_one(&db, &b, (uint64_t)order[i], reads)) bad = 1;
    for (int i = 0; i < k && !bad; ++i) {
      uint64_t f = first_op[order[i]];
      for (uint32_t j = 0; j < n_ops[order[i]]; ++j)
        if (reads[f + j] != got_reads[f + j]) { bad = 1; break; }
    }
    for (uint32_t t = 0; t < n_tables && !bad; ++t)
      if (memcmp(work[t], got_final[t], n_rows[t] * n_fields[t] * sizeof(int64_t))) bad = 1;
    if (!bad) ++matches;
  } while (next_permutation(perm, k));
  for (uint32_t t = 0; t < n_tables; ++t) free(work[t]);
  free(work);
  free(reads);
  return matches;
}
