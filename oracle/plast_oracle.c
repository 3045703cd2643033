/*
 * Plain C oracle for the PLAST-P bank-versus-bank hot path -- TEST INFRASTRUCTURE.
 *
 * Scalar, unblocked loops that state what the GPU library computes; used by the
 * tests on inputs too large for the numpy oracle and timed as the CPU baseline.
 * It shares no code, header, table or constant with the GPU library.  The
 * substitution matrix is passed in by the caller (the Python oracle's
 * transcription); the subset-seed classes are defined here.
 *
 * Paper: Nguyen & Lavenier, INRIA RR-6513 (2008).
 *   - seed key and index: Sec. 3.3.1 (subset-seed table, look-up table plus
 *     occurrence lists);
 *   - one-hit ungapped extension of every same-key pair: Sec. 3.2 generic
 *     algorithm and Sec. 3.3.3, score composition from the GPU kernel of
 *     Annex 4 (best rightward prefix, then best leftward prefix added to it);
 *   - work distribution: Sec. 5.1, threads take seeds one at a time from a
 *     shared counter;
 *   - small gapped filter: Sec. 3.3.4 (stage 3.1) and Sec. 5.2.2 (one
 *     extension on each side of the seed), banded affine-gap DP.
 *
 * Bank storage: codes[] holds, for sequence i, residues 0..19 at
 * [seq_start[i], seq_start[i+1] - pad); everything else is padding and is never
 * read here (scans are clipped at sequence ends).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NKEYS 8800
#define ORC_W 4

static const char ORC_ALPHA[] = "ACDEFGHIKLMNPQRSTVWY";
/* position-2 classes (2) and position-3 classes (11) of the subset seed */
static const char* ORC_POS2[2] = {"CFYWMLIV", "GPATSNHQEDRK"};
static const char* ORC_POS3[11] = {"A", "C", "FYW", "G", "IV", "ML", "NH", "P", "QED", "RK", "TS"};

static int orc_letter(char c) {
  for (int i = 0; i < 20; ++i)
    if (ORC_ALPHA[i] == c) return i;
  return -1;
}

static void orc_classes(int c2[20], int c3[20]) {
  for (int k = 0; k < 2; ++k)
    for (const char* p = ORC_POS2[k]; *p; ++p) c2[orc_letter(*p)] = k;
  for (int k = 0; k < 11; ++k)
    for (const char* p = ORC_POS3[k]; *p; ++p) c3[orc_letter(*p)] = k;
}

static int64_t orc_len(const int64_t* seq_start, int32_t pad, int32_t i) {
  return seq_start[i + 1] - seq_start[i] - pad;
}

/* Stage 0: key_off[8801], occ_seq/occ_pos ascending (seq, pos) within a key.
 * Returns the number of words. */
int64_t orc_build_index(const uint8_t* codes, const int64_t* seq_start, int32_t n_seqs, int32_t pad,
                        int64_t* key_off, int32_t* occ_seq, int32_t* occ_pos) {
  int c2[20], c3[20];
  orc_classes(c2, c3);
  int64_t* count = (int64_t*)calloc(ORC_NKEYS, sizeof(int64_t));
  for (int32_t s = 0; s < n_seqs; ++s) {
    const uint8_t* a = codes + seq_start[s];
    int64_t len = orc_len(seq_start, pad, s);
    for (int64_t p = 0; p + ORC_W <= len; ++p) {
      int key = ((a[p] * 2 + c2[a[p + 1]]) * 11 + c3[a[p + 2]]) * 20 + a[p + 3];
      count[key]++;
    }
  }
  key_off[0] = 0;
  for (int k = 0; k < ORC_NKEYS; ++k) key_off[k + 1] = key_off[k] + count[k];
  memset(count, 0, ORC_NKEYS * sizeof(int64_t));
  for (int32_t s = 0; s < n_seqs; ++s) {
    const uint8_t* a = codes + seq_start[s];
    int64_t len = orc_len(seq_start, pad, s);
    for (int64_t p = 0; p + ORC_W <= len; ++p) {
      int key = ((a[p] * 2 + c2[a[p + 1]]) * 11 + c3[a[p + 2]]) * 20 + a[p + 3];
      int64_t slot = key_off[key] + count[key]++;
      occ_seq[slot] = s;
      occ_pos[slot] = (int32_t)p;
    }
  }
  int64_t total = key_off[ORC_NKEYS];
  free(count);
  return total;
}

typedef struct {
  const uint8_t* codes;
  const int64_t* seq_start;
  int32_t n_seqs, pad;
  const int64_t* key_off;
  const int32_t* occ_seq;
  const int32_t* occ_pos;
} orc_bank_t;

/* Score of one pair: best rightward prefix over min(right, remaining) letters
 * plus best leftward prefix over min(nbr, available) letters. */
static int orc_pair_score(const orc_bank_t* A, int32_t s1, int32_t p1, const orc_bank_t* B, int32_t s2,
                          int32_t p2, const int8_t* mat, int nbr, int right) {
  const uint8_t* a = A->codes + A->seq_start[s1];
  const uint8_t* b = B->codes + B->seq_start[s2];
  int64_t la = orc_len(A->seq_start, A->pad, s1), lb = orc_len(B->seq_start, B->pad, s2);
  int64_t rmax = right;
  if (la - p1 < rmax) rmax = la - p1;
  if (lb - p2 < rmax) rmax = lb - p2;
  int s = 0, best_r = 0;
  for (int64_t t = 0; t < rmax; ++t) {
    s += mat[a[p1 + t] * 20 + b[p2 + t]];
    if (s > best_r) best_r = s;
  }
  int64_t lmax = nbr;
  if (p1 < lmax) lmax = p1;
  if (p2 < lmax) lmax = p2;
  s = 0;
  int best_l = 0;
  for (int64_t t = 1; t <= lmax; ++t) {
    s += mat[a[p1 - t] * 20 + b[p2 - t]];
    if (s > best_l) best_l = s;
  }
  return best_r + best_l;
}

typedef struct {
  const orc_bank_t *A, *B;
  const int8_t* mat;
  int32_t s1, nbr, right;
  const int32_t* keys;
  int32_t n_keys;
  int64_t next;          /* shared key counter */
  int64_t n_hits;        /* shared output cursor */
  int64_t n_ext;
  int32_t* out;
  int64_t cap;
  pthread_mutex_t lock;
} orc_job_t;

static void orc_flush(orc_job_t* J, const int32_t* buf, int64_t n) {
  pthread_mutex_lock(&J->lock);
  int64_t at = J->n_hits;
  J->n_hits += n;
  pthread_mutex_unlock(&J->lock);
  for (int64_t h = 0; h < n; ++h)
    if (at + h < J->cap) memcpy(J->out + 5 * (at + h), buf + 5 * h, 5 * sizeof(int32_t));
}

static void* orc_worker(void* arg) {
  orc_job_t* J = (orc_job_t*)arg;
  int64_t bufcap = 4096, nbuf = 0, ext = 0;
  int32_t* buf = (int32_t*)malloc(bufcap * 5 * sizeof(int32_t));
  for (;;) {
    int64_t q = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (q >= J->n_keys) break;
    int32_t k = J->keys ? J->keys[q] : (int32_t)q;
    for (int64_t i = J->A->key_off[k]; i < J->A->key_off[k + 1]; ++i) {
      for (int64_t j = J->B->key_off[k]; j < J->B->key_off[k + 1]; ++j) {
        int sc = orc_pair_score(J->A, J->A->occ_seq[i], J->A->occ_pos[i], J->B, J->B->occ_seq[j],
                                J->B->occ_pos[j], J->mat, J->nbr, J->right);
        ++ext;
        if (sc >= J->s1) {
          if (nbuf == bufcap) {
            orc_flush(J, buf, nbuf);
            nbuf = 0;
          }
          int32_t* r = buf + 5 * nbuf++;
          r[0] = J->A->occ_seq[i];
          r[1] = J->A->occ_pos[i];
          r[2] = J->B->occ_seq[j];
          r[3] = J->B->occ_pos[j];
          r[4] = sc;
        }
      }
    }
  }
  orc_flush(J, buf, nbuf);
  free(buf);
  __atomic_fetch_add(&J->n_ext, ext, __ATOMIC_RELAXED);
  return NULL;
}

/* Stage 2 over the listed keys (all keys when keys == NULL).  Writes at most
 * cap hit rows (seq1, pos1, seq2, pos2, score) in unspecified order and returns
 * the total number of hits; *n_ext receives the number of pairs scored. */
int64_t orc_ungapped(const uint8_t* codes1, const int64_t* start1, int32_t n1, const int64_t* key_off1,
                     const int32_t* occ_seq1, const int32_t* occ_pos1, const uint8_t* codes2,
                     const int64_t* start2, int32_t n2, const int64_t* key_off2, const int32_t* occ_seq2,
                     const int32_t* occ_pos2, int32_t pad, const int8_t* mat, int32_t s1, int32_t nbr,
                     int32_t right, const int32_t* keys, int32_t n_keys, int32_t nthreads, int32_t* out,
                     int64_t cap, int64_t* n_ext) {
  orc_bank_t A = {codes1, start1, n1, pad, key_off1, occ_seq1, occ_pos1};
  orc_bank_t B = {codes2, start2, n2, pad, key_off2, occ_seq2, occ_pos2};
  orc_job_t J;
  memset(&J, 0, sizeof(J));
  J.A = &A;
  J.B = &B;
  J.mat = mat;
  J.s1 = s1;
  J.nbr = nbr;
  J.right = right;
  J.keys = keys;
  J.n_keys = keys ? n_keys : ORC_NKEYS;
  J.out = out;
  J.cap = cap;
  pthread_mutex_init(&J.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_worker, &J);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&J.lock);
  if (n_ext) *n_ext = J.n_ext;
  return J.n_hits;
}

/* ------------------------------------------------------------------ gapped */

#define ORC_NEG (-(1 << 28))

/* Anchored banded affine-gap DP over x[0..lx) and y[0..ly) read with strides
 * dx, dy (+1 rightward, -1 leftward).  Cell (i, j) exists iff i <= lx, j <= ly
 * and |i - j| <= band.  Gap of length k costs open + k*ext.
 * Returns max(0, best H over existing cells). */
static int orc_gapped_side(const uint8_t* x, int lx, int dx, const uint8_t* y, int ly, int dy,
                           const int8_t* mat, int band, int open, int ext) {
  int W1 = ly + 1;
  int* H = (int*)malloc(sizeof(int) * (lx + 1) * W1);
  int* E = (int*)malloc(sizeof(int) * (lx + 1) * W1);
  int* F = (int*)malloc(sizeof(int) * (lx + 1) * W1);
  int best = 0;
  for (int i = 0; i <= lx; ++i) {
    for (int j = 0; j <= ly; ++j) {
      int c = i * W1 + j;
      H[c] = E[c] = F[c] = ORC_NEG;
      if ((i > j ? i - j : j - i) > band) continue;
      if (i == 0 && j == 0) {
        H[c] = 0;
        continue;
      }
      if (j >= 1 && (i > j - 1 ? i - (j - 1) : (j - 1) - i) <= band) {
        int e1 = E[c - 1] - ext, e2 = H[c - 1] - open - ext;
        E[c] = e1 > e2 ? e1 : e2;
      }
      if (i >= 1 && ((i - 1) > j ? (i - 1) - j : j - (i - 1)) <= band) {
        int f1 = F[c - W1] - ext, f2 = H[c - W1] - open - ext;
        F[c] = f1 > f2 ? f1 : f2;
      }
      int h = ORC_NEG;
      if (i >= 1 && j >= 1) h = H[c - W1 - 1] + mat[x[(i - 1) * dx] * 20 + y[(j - 1) * dy]];
      if (E[c] > h) h = E[c];
      if (F[c] > h) h = F[c];
      if (h < ORC_NEG) h = ORC_NEG;
      H[c] = h;
      if (h > best) best = h;
    }
  }
  free(H);
  free(E);
  free(F);
  return best;
}

typedef struct {
  const orc_bank_t *A, *B;
  const int32_t* hits;
  int64_t n;
  const int8_t* mat;
  int32_t window, band, open, ext;
  int32_t* gscore;
  int64_t next;
} orc_gjob_t;

static void* orc_gworker(void* arg) {
  orc_gjob_t* J = (orc_gjob_t*)arg;
  for (;;) {
    int64_t h = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (h >= J->n) break;
    const int32_t* r = J->hits + 5 * h;
    int32_t s1 = r[0], p1 = r[1], s2 = r[2], p2 = r[3];
    const uint8_t* a = J->A->codes + J->A->seq_start[s1];
    const uint8_t* b = J->B->codes + J->B->seq_start[s2];
    int64_t la = orc_len(J->A->seq_start, J->A->pad, s1), lb = orc_len(J->B->seq_start, J->B->pad, s2);
    int rx = (int)(la - p1 < J->window ? la - p1 : J->window);
    int ry = (int)(lb - p2 < J->window ? lb - p2 : J->window);
    int lx = p1 < J->window ? p1 : J->window;
    int ly = p2 < J->window ? p2 : J->window;
    int right = orc_gapped_side(a + p1, rx, 1, b + p2, ry, 1, J->mat, J->band, J->open, J->ext);
    int left = orc_gapped_side(a + p1 - 1, lx, -1, b + p2 - 1, ly, -1, J->mat, J->band, J->open, J->ext);
    J->gscore[h] = right + left;
  }
  return NULL;
}

void orc_gapped(const uint8_t* codes1, const int64_t* start1, const uint8_t* codes2, const int64_t* start2,
                int32_t pad, const int32_t* hits, int64_t n, const int8_t* mat, int32_t window, int32_t band,
                int32_t open, int32_t ext, int32_t nthreads, int32_t* gscore) {
  orc_bank_t A = {codes1, start1, 0, pad, 0, 0, 0};
  orc_bank_t B = {codes2, start2, 0, pad, 0, 0, 0};
  orc_gjob_t J = {&A, &B, hits, n, mat, window, band, open, ext, gscore, 0};
  if (nthreads < 1) nthreads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_gworker, &J);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
}

/* ------------------------------------------------------ full gapped alignment */

/* Stage 3.2 (Sec. 3.3.4): the hits that pass S2 get a full gapped alignment;
 * a list of the ungapped pieces (diagonal, first and one-past-last position in
 * sequence 1) of the alignments already computed for a sequence pair lets a
 * hit lying on one of them skip its own.
 *
 * One side: the anchored affine-gap recurrences of orc_gapped_side with no band
 * and no window.  best = max over cells of H (H(0,0) = 0); the end cell is the
 * first cell in row-major order with H == best.  Trace-back preferences: state
 * H came from the diagonal if that gives H, else from E, else from F; state E
 * (F) came from a gap opening if that gives its value, else from an extension. */

typedef struct {
  int* H;
  int* E;
  int* F;
  size_t cap;
  char* moves; /* from the end cell back to the anchor */
  size_t mcap;
} orc_dp_t;

static void orc_dp_reserve(orc_dp_t* D, int lx, int ly) {
  size_t need = (size_t)(lx + 1) * (size_t)(ly + 1);
  if (need > D->cap) {
    free(D->H);
    free(D->E);
    free(D->F);
    D->H = (int*)malloc(sizeof(int) * need);
    D->E = (int*)malloc(sizeof(int) * need);
    D->F = (int*)malloc(sizeof(int) * need);
    D->cap = need;
  }
  if ((size_t)(lx + ly + 1) > D->mcap) {
    free(D->moves);
    D->mcap = (size_t)(lx + ly + 1);
    D->moves = (char*)malloc(D->mcap);
  }
}

/* Returns best; *n_moves moves in D->moves, in order from the end cell back to
 * the anchor ('D' pair, 'E' letter of y against a gap, 'F' letter of x). */
static int orc_full_side(orc_dp_t* D, const uint8_t* x, int lx, int dx, const uint8_t* y, int ly, int dy,
                         const int8_t* mat, int open, int ext, int* n_moves) {
  orc_dp_reserve(D, lx, ly);
  int W1 = ly + 1;
  int *H = D->H, *E = D->E, *F = D->F;
  int best = 0, bi = 0, bj = 0;
  for (int i = 0; i <= lx; ++i) {
    for (int j = 0; j <= ly; ++j) {
      int c = i * W1 + j;
      H[c] = E[c] = F[c] = ORC_NEG;
      if (i == 0 && j == 0) {
        H[c] = 0;
        continue;
      }
      if (j >= 1) {
        int e1 = E[c - 1] - ext, e2 = H[c - 1] - open - ext;
        E[c] = e1 > e2 ? e1 : e2;
      }
      if (i >= 1) {
        int f1 = F[c - W1] - ext, f2 = H[c - W1] - open - ext;
        F[c] = f1 > f2 ? f1 : f2;
      }
      int h = ORC_NEG;
      if (i >= 1 && j >= 1) h = H[c - W1 - 1] + mat[x[(i - 1) * dx] * 20 + y[(j - 1) * dy]];
      if (E[c] > h) h = E[c];
      if (F[c] > h) h = F[c];
      if (h < ORC_NEG) h = ORC_NEG;
      H[c] = h;
      if (h > best) {
        best = h;
        bi = i;
        bj = j;
      }
    }
  }
  int i = bi, j = bj, n = 0;
  char state = 'H';
  while (i > 0 || j > 0) {
    int c = i * W1 + j;
    if (state == 'H') {
      if (i >= 1 && j >= 1 && H[c] == H[c - W1 - 1] + mat[x[(i - 1) * dx] * 20 + y[(j - 1) * dy]]) {
        D->moves[n++] = 'D';
        --i;
        --j;
        continue;
      }
      state = H[c] == E[c] ? 'E' : 'F';
    } else if (state == 'E') {
      D->moves[n++] = 'E';
      state = E[c] == H[c - 1] - open - ext ? 'H' : 'E';
      --j;
    } else {
      D->moves[n++] = 'F';
      state = F[c] == H[c - W1] - open - ext ? 'H' : 'F';
      --i;
    }
  }
  *n_moves = n;
  return best;
}

typedef struct {
  int32_t diag, first, last, owner; /* pairs on diagonal diag at positions [first, last) of sequence 1 */
} orc_piece_t;

typedef struct {
  const orc_bank_t *A, *B;
  const int32_t* hits;
  const int32_t* gscore;
  const int64_t* order; /* passing hits sorted by (seq1, seq2, -gscore, pos1, pos2) */
  const int64_t* group; /* group g = order[group[g] .. group[g + 1]) */
  int64_t n_groups;
  const int8_t* mat;
  int32_t open, ext;
  int32_t* out; /* 14 int32 per alignment */
  int32_t* cover;
  int64_t next, n_out;
} orc_ajob_t;

/* Walks one side's moves from the anchor outward (moves[] is stored end-first),
 * appending pieces; step +1 pairs a[p1 + i] with b[p2 + j], step -1 pairs
 * a[p1 - 1 - i] with b[p2 - 1 - j].  Adds identities, mismatches and gap
 * openings to st[0..2]; returns the letters consumed in st[3] (x) and st[4] (y). */
static void orc_side_walk(const uint8_t* a, int p1, const uint8_t* b, int p2, const char* moves, int n, int step,
                          int32_t owner, orc_piece_t** pieces, int64_t* np, int64_t* pcap, int st[5]) {
  int i = 0, j = 0, open_run = 0;
  char prev = 0;
  for (int k = n - 1; k >= 0; --k) {
    char m = moves[k];
    if (m == 'D') {
      int pa = step > 0 ? p1 + i : p1 - 1 - i;
      int pb = step > 0 ? p2 + j : p2 - 1 - j;
      if (a[pa] == b[pb]) st[0]++;
      else st[1]++;
      if (!open_run) {
        if (*np == *pcap) {
          *pcap = *pcap ? 2 * *pcap : 64;
          *pieces = (orc_piece_t*)realloc(*pieces, sizeof(orc_piece_t) * (size_t)*pcap);
        }
        orc_piece_t* q = &(*pieces)[(*np)++];
        q->diag = pa - pb;
        q->first = pa;
        q->last = pa + 1;
        q->owner = owner;
        open_run = 1;
      } else {
        orc_piece_t* q = &(*pieces)[*np - 1];
        if (step > 0) q->last = pa + 1;
        else q->first = pa;
      }
      ++i;
      ++j;
    } else {
      open_run = 0;
      if (m != prev) st[2]++;
      if (m == 'E') ++j;
      else ++i;
    }
    prev = m;
  }
  st[3] = i;
  st[4] = j;
}

static void* orc_aworker(void* arg) {
  orc_ajob_t* J = (orc_ajob_t*)arg;
  orc_dp_t D = {0};
  orc_piece_t* pieces = NULL;
  int64_t pcap = 0;
  for (;;) {
    int64_t g = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (g >= J->n_groups) break;
    int64_t np = 0;
    for (int64_t k = J->group[g]; k < J->group[g + 1]; ++k) {
      int64_t h = J->order[k];
      const int32_t* r = J->hits + 5 * h;
      int32_t s1 = r[0], p1 = r[1], s2 = r[2], p2 = r[3];
      int32_t owner = -1;
      for (int64_t q = 0; q < np && owner < 0; ++q)
        if (pieces[q].diag == p1 - p2 && pieces[q].first <= p1 && p1 < pieces[q].last) owner = pieces[q].owner;
      if (owner >= 0) {
        J->cover[h] = owner;
        continue;
      }
      J->cover[h] = (int32_t)h;
      const uint8_t* a = J->A->codes + J->A->seq_start[s1];
      const uint8_t* b = J->B->codes + J->B->seq_start[s2];
      int la = (int)orc_len(J->A->seq_start, J->A->pad, s1), lb = (int)orc_len(J->B->seq_start, J->B->pad, s2);
      int nmR, nmL, stR[5] = {0}, stL[5] = {0};
      int bR = orc_full_side(&D, a + p1, la - p1, 1, b + p2, lb - p2, 1, J->mat, J->open, J->ext, &nmR);
      orc_side_walk(a, p1, b, p2, D.moves, nmR, +1, (int32_t)h, &pieces, &np, &pcap, stR);
      int bL = orc_full_side(&D, a + p1 - 1, p1, -1, b + p2 - 1, p2, -1, J->mat, J->open, J->ext, &nmL);
      orc_side_walk(a, p1, b, p2, D.moves, nmL, -1, (int32_t)h, &pieces, &np, &pcap, stL);
      int64_t o = __atomic_fetch_add(&J->n_out, 1, __ATOMIC_RELAXED);
      int32_t* w = J->out + 14 * o;
      w[0] = s1;
      w[1] = s2;
      w[2] = p1;
      w[3] = p2;
      w[4] = p1 - stL[3];
      w[5] = p1 + stR[3];
      w[6] = p2 - stL[4];
      w[7] = p2 + stR[4];
      w[8] = bR + bL;
      w[9] = nmR + nmL;
      w[10] = stR[0] + stL[0];
      w[11] = stR[1] + stL[1];
      w[12] = stR[2] + stL[2];
      w[13] = (int32_t)h;
    }
  }
  free(D.H);
  free(D.E);
  free(D.F);
  free(D.moves);
  free(pieces);
  return NULL;
}

static const int32_t* orc_sort_hits;
static const int32_t* orc_sort_gscore;

static int orc_cmp_hit(const void* pa, const void* pb) {
  int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
  const int32_t *x = orc_sort_hits + 5 * a, *y = orc_sort_hits + 5 * b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[2] != y[2]) return x[2] < y[2] ? -1 : 1;
  if (orc_sort_gscore[a] != orc_sort_gscore[b]) return orc_sort_gscore[a] > orc_sort_gscore[b] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  if (x[3] != y[3]) return x[3] < y[3] ? -1 : 1;
  return 0;
}

/* Full gapped alignments of the hits with pass[h] != 0.  out holds up to n
 * records of 14 int32 (seq1, seq2, seed1, seed2, start1, end1, start2, end2,
 * score, length, identities, mismatches, gap openings, hit), in no particular
 * order; cover[h] = the hit whose alignment covers h (h itself when it computed
 * one), -1 when h did not pass.  Returns the number of records. */
int64_t orc_full_align(const uint8_t* codes1, const int64_t* start1, const uint8_t* codes2, const int64_t* start2,
                       int32_t pad, const int32_t* hits, const int32_t* gscore, const uint8_t* pass, int64_t n,
                       const int8_t* mat, int32_t open, int32_t ext, int32_t nthreads, int32_t* out,
                       int32_t* cover) {
  orc_bank_t A = {codes1, start1, 0, pad, 0, 0, 0};
  orc_bank_t B = {codes2, start2, 0, pad, 0, 0, 0};
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t h = 0; h < n; ++h) {
    cover[h] = -1;
    if (pass[h]) order[m++] = h;
  }
  orc_sort_hits = hits;
  orc_sort_gscore = gscore;
  qsort(order, (size_t)m, sizeof(int64_t), orc_cmp_hit);
  int64_t* group = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
  int64_t ng = 0;
  for (int64_t k = 0; k < m; ++k) {
    const int32_t *x = hits + 5 * order[k], *y = k ? hits + 5 * order[k - 1] : NULL;
    if (!y || x[0] != y[0] || x[2] != y[2]) group[ng++] = k;
  }
  group[ng] = m;
  orc_ajob_t J = {&A, &B, hits, gscore, order, group, ng, mat, open, ext, out, cover, 0, 0};
  if (nthreads < 1) nthreads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_aworker, &J);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  free(order);
  free(group);
  return J.n_out;
}
