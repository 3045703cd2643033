/*
 * plast.h -- C ABI of the MI355X (gfx950) PLAST-P bank-versus-bank hot path.
 *
 * Method: Nguyen & Lavenier, "Fine-grained parallelization of similarity search
 * between protein sequences", INRIA RR-6513 (2008).  Two protein banks are
 * indexed by a 4-letter subset seed (Sec. 3.3.1); for every seed key, every pair
 * of an occurrence in bank 1 and an occurrence in bank 2 gets a one-hit ungapped
 * extension on bounded neighbourhoods (Sec. 3.2, Sec. 3.3.3; score composition
 * of the GPU kernel in Annex 4) and survivors go through a small banded gapped
 * filter (Sec. 3.3.4 stage 3.1, Sec. 5.2.2); those that pass get a full gapped
 * alignment (Sec. 3.3.4 stage 3.2).
 *
 * Conventions shared by every entry point
 *   - Device pointers ("d_") are HIP device memory owned by the caller; the
 *     library never allocates, frees or retains device memory (apart from the
 *     fixed static array of plast_ungapped_extend_noalloc).  Host pointers
 *     ("h_") are ordinary host memory.
 *   - Every call returns a status (PLAST_OK or a negative PLAST_E_* code);
 *     nothing throws or aborts across the ABI.  plast_strerror() maps a code to
 *     a static string, plast_last_error() returns a thread-local detail message
 *     for the last failing call on the calling thread.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls that return
 *     counts to the host synchronise that stream before returning; the others
 *     only enqueue work.
 *   - Residue codes are 0..19 in the order ACDEFGHIKLMNPQRSTVWY.
 */
#ifndef PLAST_H
#define PLAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLAST_NKEYS 8800   /* 20 x 2 x 11 x 20 subset-seed keys (Sec. 3.3.1) */
#define PLAST_SEED_LEN 4
#define PLAST_PAD_CODE 20  /* code of the separator between sequences */
#define PLAST_PAD_LEN 20   /* separator run length of the padded bank layout */
#define PLAST_NBR 20       /* neighbourhood letters scanned beyond each seed end */

enum {
  PLAST_OK = 0,
  PLAST_E_ARG = -1,        /* null pointer, negative size, unsupported parameter */
  PLAST_E_ALPHABET = -2,   /* a residue code > 19, or a separator that is not 20 */
  PLAST_E_CAPACITY = -3,   /* hit buffer too small; required size reported */
  PLAST_E_WORKSPACE = -4,  /* workspace / index buffer smaller than the query said */
  PLAST_E_HIP = -5,        /* a HIP runtime call failed (detail in plast_last_error) */
  PLAST_E_LAYOUT = -6      /* seq_start is not a valid padded layout */
};

enum { PLAST_PLAIN = 0, PLAST_BATCHED = 1 };

/* One ungapped hit: sequence ids (0-based) and the 0-based position of the first
 * seed letter in each sequence, plus the exact integer score (20 bytes). */
typedef struct {
  int32_t seq1, pos1, seq2, pos2, score;
} plast_hit_t;

/* Read-only view of a built index (filled by plast_build_index).  All pointers
 * are device pointers into caller memory: the bank passed in and the index
 * buffer.  The view borrows them; it does not own anything. */
typedef struct {
  const uint8_t* codes;      /* the bank, padded layout, n_padded bytes */
  const int64_t* seq_start;  /* n_seqs + 1 offsets */
  int32_t n_seqs;
  int64_t n_padded;
  const int64_t* key_off;    /* PLAST_NKEYS + 1: occurrences of key k are [key_off[k], key_off[k+1]) */
  const int32_t* occ;        /* n_words: offset in codes of the first seed letter */
  const int32_t* occ_seq;    /* n_words: sequence id of that occurrence */
  const uint8_t* scan_codes; /* INTERNAL (in the index buffer): the letters scaled to table offsets,
                                with tail slack; kernels read it instead of codes.  Callers only
                                pass the view on and must not rely on its contents. */
  int64_t n_words;           /* host copy of key_off[PLAST_NKEYS] */
} plast_index_t;

/*
 * Launch shapes (performance only: every valid tuning gives the same results).
 * Keys are put in size classes by n2, their number of bank-b occurrences: key
 * k is in class c iff class_min_n2[c] <= n2 < class_min_n2[c + 1] (the last
 * class is open above).  A BATCHED work item covers up to 32 bank-a
 * occurrences (the last item of a key fewer) and up to item_cols[c] bank-b
 * occurrences of one key.  xcd_queues = 8 splits the
 * work list into one contiguous queue per XCD (workgroup w starts on queue
 * w mod 8 and then steals from the others), so the items sharing bank-b
 * windows run under one L2; 1 keeps a single queue.  gapped_threads is the
 * workgroup size of the gapped filter.  plast_tuning_default() gives the
 * built-in values, plast_autotune() measured ones.
 */
#define PLAST_TUNE_CLASSES 4
#define PLAST_TUNE_WIDTHS 5   /* candidate item widths: 1024, 2048, 4096, 8192, 16384 */
typedef struct {
  int32_t class_min_n2[PLAST_TUNE_CLASSES]; /* class_min_n2[0] == 1, strictly ascending */
  int32_t item_cols[PLAST_TUNE_CLASSES];    /* multiple of 512 in [512, 16384] */
  int32_t xcd_queues;                       /* 1 or 8 */
  int32_t gapped_threads;                   /* 128, 256 or 512 */
} plast_tuning_t;

typedef struct {
  int32_t nbr;             /* must be PLAST_NBR (20) */
  int32_t s1;              /* a pair is a hit iff score >= s1 */
  const int8_t* matrix;    /* host, 20x20 row-major in code order; NULL = BLOSUM62 */
  const plast_tuning_t* tuning;  /* host; NULL = plast_tuning_default() */
} plast_ungapped_params_t;

typedef struct {
  int32_t window;          /* letters per side, 1..64 (64 in the reference configuration) */
  int32_t band;            /* cells (i, j) with |i - j| <= band, 0..16 */
  int32_t gap_open;        /* a gap of length k costs gap_open + k * gap_extend */
  int32_t gap_extend;
  int32_t s2;              /* pass iff gapped score >= s2 */
  const int8_t* matrix;    /* host, 20x20 row-major in code order; NULL = BLOSUM62 */
  const plast_tuning_t* tuning;  /* host; NULL = plast_tuning_default() */
} plast_gapped_params_t;

/*
 * Sizes for plast_build_index.
 * n_padded: length of the padded bank; n_seqs: number of sequences.
 * *index_bytes receives the size of the index buffer (it holds key_off, occ,
 * occ_seq and scan_codes and must outlive every view built into it);
 * *ws_bytes the size of the scratch workspace used only during the build.
 */
int plast_index_bytes(int64_t n_padded, int32_t n_seqs, size_t* index_bytes, size_t* ws_bytes);

/*
 * Stage 0, bank indexing (Sec. 3.3.1): the subset-seed key of every 4-letter
 * word that lies inside one sequence, then a stable sort by key (two radix
 * passes on 7-bit digits), so that inside a key occurrences are ascending by
 * (sequence, position).
 *
 * Padded layout of the bank (d_codes, n_padded bytes; d_seq_start, n_seqs + 1
 * int64): a run of PLAST_PAD_LEN codes PLAST_PAD_CODE, sequence 0, a run, ...,
 * the last sequence, a final run.  d_seq_start[i] is the offset of the first
 * residue of sequence i, d_seq_start[n_seqs] == n_padded; sequence i has length
 * d_seq_start[i+1] - d_seq_start[i] - PLAST_PAD_LEN (0 allowed).  n_padded must
 * be < 2^31 - 256.
 * Errors: PLAST_E_ARG (null pointer, bad sizes), PLAST_E_WORKSPACE (buffers
 * smaller than plast_index_bytes), PLAST_E_LAYOUT (seq_start inconsistent),
 * PLAST_E_ALPHABET (residue code > 19 or separator code != 20),
 * PLAST_E_HIP.  Synchronises `stream` (to validate and to report n_words).
 * On success *out is a view into d_codes, d_seq_start and d_index.
 */
int plast_build_index(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                      void* d_index, size_t index_bytes, void* d_ws, size_t ws_bytes, plast_index_t* out,
                      void* stream);

/*
 * Workspace size for plast_ungapped_extend in `mode` (PLAST_PLAIN or
 * PLAST_BATCHED) for these two indexes and this tuning (NULL = default; the
 * work list grows as item widths shrink).  Reads both key tables back to the
 * host (synchronises `stream`).  *n_ext (may be NULL) receives the number of
 * candidate pairs, sum over keys of n1(k) * n2(k); *n_items (may be NULL) the
 * length of the BATCHED work list.
 */
int plast_ungapped_workspace_bytes(const plast_index_t* a, const plast_index_t* b, int32_t mode,
                                   const plast_tuning_t* tuning, size_t* bytes, int64_t* n_ext, int64_t* n_items,
                                   void* stream);

/*
 * Stage 2, ungapped extension (Sec. 3.2 generic algorithm, Sec. 3.3.3) with hit
 * compaction.  For every key and every pair (i in bank a, j in bank b) of its
 * occurrences the score is best-right + best-left: the best prefix sum (0
 * included) of substitution scores scanning rightward from the first seed
 * letters over at most PLAST_SEED_LEN + nbr letters, plus the best prefix sum
 * scanning leftward from the letters before them over at most nbr letters;
 * both scans stop at sequence ends.  Pairs with score >= s1 are written to
 * d_hits in unspecified order.
 *
 * mode PLAST_PLAIN launches one grid per key with candidate pairs, in key order;
 * PLAST_BATCHED builds a device work list and runs one persistent work-queue
 * kernel.  Both produce the same set of hits.
 * d_ws/ws_bytes: scratch of at least plast_ungapped_workspace_bytes.
 * d_hits/capacity: output array of `capacity` records.
 * *h_n_hits always receives the number of hits (even when it exceeds capacity);
 * *h_n_ext (may be NULL) the number of pairs scored.
 * Errors: PLAST_E_ARG, PLAST_E_WORKSPACE, PLAST_E_HIP; PLAST_E_CAPACITY when
 * *h_n_hits > capacity (d_hits then holds an unspecified subset; call again
 * with a larger buffer).  Synchronises `stream`.
 */
int plast_ungapped_extend(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                          int32_t mode, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits, int64_t capacity,
                          int64_t* h_n_hits, int64_t* h_n_ext, void* stream);

/*
 * Allocation-free variant of plast_ungapped_extend, for callers that cannot
 * allocate device memory or pass a workspace (tight serving loops, harnesses
 * that forbid hipMalloc).  Same computation, arguments, outputs and errors as
 * plast_ungapped_extend in PLAST_BATCHED mode, except that the workspace is a
 * static device array of PLAST_NOALLOC_SCRATCH_BYTES inside the library: each
 * GPU the library runs on holds one copy until the process ends, its address is
 * looked up once per device (on the first call with that device current), and
 * the call allocates nothing.  Runs on the current device; `stream` must
 * belong to it.
 * Limit: the work list must fit the array (about 520,000 items of the tuning in
 * p->tuning; plast_ungapped_workspace_bytes reports the length in *n_items).  A
 * longer list returns PLAST_E_WORKSPACE with the length in plast_last_error()
 * and writes no hits.
 * All calls on one GPU share its array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller.  Synchronises `stream`.
 */
#define PLAST_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
int plast_ungapped_extend_noalloc(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                                  plast_hit_t* d_hits, int64_t capacity, int64_t* h_n_hits, int64_t* h_n_ext,
                                  void* stream);

/*
 * Stage 3.1, small gapped filter (Sec. 3.3.4; Sec. 5.2.2: one extension on each
 * side of the seed).  For every hit, an anchored banded affine-gap alignment of
 * a[pos1 ..) against b[pos2 ..) and another of a[pos1-1], a[pos1-2], ...
 * against b[pos2-1], b[pos2-2], ..., each over at most `window` letters per
 * sequence and clipped at sequence ends; cells (i, j) exist iff |i - j| <= band;
 * each side's score is max(0, best cell).  d_gscore[h] = right + left,
 * d_pass[h] = (d_gscore[h] >= s2).  Hits are read from d_hits[0 .. n_hits).
 * A record whose sequence ids or positions lie outside the banks gets
 * d_gscore = -1 and d_pass = 0 (nothing is read for it).
 * Errors: PLAST_E_ARG (bad parameters), PLAST_E_HIP.  Enqueues only; does not
 * synchronise.
 */
int plast_gapped_filter(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, int64_t n_hits,
                        const plast_gapped_params_t* g, int32_t* d_gscore, uint8_t* d_pass, void* stream);

/*
 * Kernel timing (tracing aid, not needed for results).  While enabled, the
 * library records HIP events on the caller's stream around the kernels of each
 * call; plast_timing_read() waits for the events of the most recent calls and
 * reports device milliseconds.  Process-wide and not thread-safe: meant for
 * benchmarks and profiling runs.
 */
typedef struct {
  float index_ms;              /* last plast_build_index: from its first to its last kernel */
  float plan_ms;               /* last PLAST_BATCHED extension: work-list kernels */
  float ungapped_ms;           /* last plast_ungapped_extend: the extension kernel(s) only
                                  (all per-key grids in PLAST_PLAIN mode) */
  float gapped_ms;             /* last plast_gapped_filter: its kernel */
  int64_t ungapped_launches;   /* extension-kernel launches of the last extension call */
  float align_ms;              /* last plast_align: its alignment kernel (not the grouping before it) */
} plast_timing_t;

int plast_timing_enable(int on);
int plast_timing_read(plast_timing_t* out);

/* Built-in launch shapes: classes from n2 = 1, 2048, 8192, 32768, every item
 * 4096 columns wide, one queue, 256-thread gapped workgroups. */
int plast_tuning_default(plast_tuning_t* out);

/* Per-candidate device times of one plast_autotune call, in milliseconds
 * (best of `reps`; 0 = not run: empty class, or a width that gives the same
 * items as a smaller one, or a work list that does not fit the workspace). */
typedef struct {
  int64_t class_ext[PLAST_TUNE_CLASSES];                  /* pairs scored per class */
  float class_ms[PLAST_TUNE_CLASSES][PLAST_TUNE_WIDTHS];  /* class alone, per item width */
  float queue_ms[2];                                      /* whole list: 1 queue, 8 queues */
  float gapped_ms[3];                                     /* 128, 256, 512 threads */
} plast_tune_report_t;

/*
 * Autotuner of the BATCHED launch shapes for one pair of indexes.  Starting
 * from p->tuning (or the default): for each size class, the extension kernel
 * runs over that class's work items alone at every candidate width and the
 * fastest width is kept; then the whole work list runs with 1 and with 8
 * queues; then the gapped filter runs over the hits with each workgroup size.
 * Every timing is the best of `reps` (1..20) runs, measured with HIP events
 * around the kernel.  The hit buffers are scratch during the search and hold
 * the hits of the last extension run afterwards.  d_ws must hold the work list
 * of the smallest width (plast_ungapped_workspace_bytes with item_cols all
 * 1024); candidates whose list does not fit are skipped.
 * Errors: as plast_ungapped_extend (PLAST_E_CAPACITY when the hits do not fit)
 * and plast_gapped_filter.  Synchronises `stream`.
 */
int plast_autotune(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                   const plast_gapped_params_t* g, int32_t reps, void* d_ws, size_t ws_bytes,
                   plast_hit_t* d_hits, int64_t capacity, int32_t* d_gscore, uint8_t* d_pass,
                   plast_tuning_t* out, plast_tune_report_t* report, void* stream);

/*
 * Whole-search pipeline replayed from a HIP graph: index both banks, build the
 * work list, run the persistent extension kernel and the gapped filter, with
 * no host synchronisation inside.  The graph is captured once, on a stream the
 * pipeline owns, from exactly the kernels that plast_build_index,
 * plast_ungapped_extend (BATCHED) and plast_gapped_filter launch; error checks
 * that those calls make on the host happen on the device instead (a bank with
 * a layout or alphabet error yields no hits and sets the status).  The gapped
 * filter reads the hit count from device memory and scores min(hits,
 * capacity) records.
 *
 * A bank is described by its padded codes and seq_start (as for
 * plast_build_index); the pointers and sizes are fixed at creation, the
 * contents may change between launches (sizes, and so a new work-list length,
 * may not).  max_items bounds the work list (plast_ungapped_workspace_bytes
 * reports the current length in *n_items); a longer list yields
 * PLAST_E_WORKSPACE in the result and no hits.
 * The workspace (plast_pipeline_workspace_bytes, 256-byte aligned) holds both
 * indexes, the build scratch and the work list; it and the output buffers are
 * caller memory that must outlive the pipeline.
 */
typedef struct plast_pipeline plast_pipeline_t;
typedef struct {
  const uint8_t* codes;     /* device, padded layout, n_padded bytes */
  const int64_t* seq_start; /* device, n_seqs + 1 */
  int32_t n_seqs;
  int64_t n_padded;
} plast_bank_t;
typedef struct {
  int32_t status;           /* PLAST_OK, PLAST_E_LAYOUT, PLAST_E_ALPHABET, PLAST_E_WORKSPACE or PLAST_E_CAPACITY */
  int32_t n_items;          /* work-list length */
  int64_t n_hits;           /* hits found (may exceed capacity) */
  int64_t n_ext;            /* pairs scored */
  int64_t n_words_a, n_words_b;
} plast_pipeline_result_t;

int plast_pipeline_workspace_bytes(const plast_bank_t* a, const plast_bank_t* b, int64_t max_items, size_t* bytes);
/* Captures and instantiates the graph (does not run it).  *out receives a host
 * handle; release it with plast_pipeline_destroy. */
int plast_pipeline_create(const plast_bank_t* a, const plast_bank_t* b, const plast_ungapped_params_t* p,
                          const plast_gapped_params_t* g, int64_t max_items, void* d_ws, size_t ws_bytes,
                          plast_hit_t* d_hits, int64_t capacity, int32_t* d_gscore, uint8_t* d_pass,
                          plast_pipeline_t** out);
/* Enqueues one replay on `stream`; does not synchronise. */
int plast_pipeline_launch(plast_pipeline_t* pl, void* stream);
/* Waits for `stream` and reads the counts and status of the last replay. */
int plast_pipeline_result(plast_pipeline_t* pl, plast_pipeline_result_t* out, void* stream);
/* Index views of the last replay's banks (which = 0: a, 1: b); n_words is -1
 * until plast_pipeline_result has been called. */
int plast_pipeline_index(const plast_pipeline_t* pl, int32_t which, plast_index_t* out);
int plast_pipeline_destroy(plast_pipeline_t* pl);

/*
 * Query search against a resident index, enqueued with no host synchronisation
 * (the serving path: many query banks against one bank kept in HBM, several
 * searches in flight on different streams).  One call enqueues, on `stream`:
 * stage 0 for query bank a, the BATCHED work list and persistent extension
 * kernel against the prebuilt index b (plast_build_index), the gapped filter
 * with the hit count read from device memory, and, when d_matches is not NULL,
 * a compaction of the hits that pass the gapped filter into d_matches (order
 * unspecified).  Checks that the eager calls make on the host are device flags
 * here, read back by plast_search_result.
 * d_ws (plast_search_workspace_bytes, 256-byte aligned) holds bank a's index,
 * the build scratch, the work list (max_items items) and the counters; it must
 * stay untouched until plast_search_result has returned.  Searches that share
 * a workspace or output buffers must not overlap.
 */
typedef struct {
  int32_t seq1, pos1, seq2, pos2, score, gscore;  /* a hit that passes the gapped filter */
} plast_match_t;

/* Only a's sizes are read (its pointers may be NULL). */
int plast_search_workspace_bytes(const plast_bank_t* a, int64_t max_items, size_t* bytes);
/* d_seg_first (may be NULL; needs d_matches): n_seg + 1 ascending sequence ids
 * of bank a, d_seg_first[0] = 0 and d_seg_first[n_seg] = a's n_seqs, cutting a
 * into segments (one per request of a batch; n_seg <= 65536).  The matches are then written
 * grouped by segment: segment s owns d_matches[d_seg_off[s] .. d_seg_off[s+1]),
 * order inside a segment unspecified.  d_seg_off is device scratch of
 * 2 (n_seg + 1) int64; its first n_seg + 1 entries are the offsets. */
int plast_search_enqueue(const plast_bank_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                         const plast_gapped_params_t* g, int64_t max_items, void* d_ws, size_t ws_bytes,
                         plast_hit_t* d_hits, int64_t capacity, int32_t* d_gscore, uint8_t* d_pass,
                         plast_match_t* d_matches, const int32_t* d_seg_first, int32_t n_seg, int64_t* d_seg_off,
                         void* stream);
/* Waits for `stream` and reads the status and counts of the last search
 * enqueued with this workspace (n_words_b is b's count as given).  *n_matches
 * (may be NULL) receives the number of matches written. */
int plast_search_result(const void* d_ws, plast_pipeline_result_t* out, int64_t* n_matches, void* stream);

/*
 * TPLAST-N (Sec. 6: a protein bank against the six translated frames of a
 * nucleotide bank), the translation on the device.  Frames 0..2 read the
 * forward strand from nucleotide 0, 1 or 2, frames 3..5 the reverse complement
 * the same way; a trailing partial codon is dropped; the standard genetic code
 * maps codons to residues or stops, and stops cut every frame into fragments.
 * The output is a protein bank in the padded layout (plast_build_index input)
 * whose sequences are the non-empty fragments in the order (DNA sequence,
 * frame, position), and d_frag[3 j .. 3 j + 2] = (DNA sequence, frame, offset
 * of fragment j's first residue within its frame) for mapping hits back.
 * Nucleotide codes are A 0, C 1, G 2, T 3; d_dna_start has n_dna + 1 ascending
 * offsets into d_dna with d_dna_start[n_dna] = n_nt.
 * Two calls: plast_translate_count enqueues the counting pass and synchronises,
 * returning the fragment count and the padded length (so the caller can size
 * the outputs: n_padded codes, n_frags + 1 starts, 3 n_frags fragment words);
 * plast_translate_write then enqueues the writing pass with the same workspace
 * (plast_translate_ws_bytes, 256-byte aligned).
 * Errors: PLAST_E_ARG, PLAST_E_LAYOUT (offsets), PLAST_E_ALPHABET (a code > 3),
 * PLAST_E_WORKSPACE, PLAST_E_HIP.
 */
int plast_translate_ws_bytes(int32_t n_dna, size_t* bytes);
int plast_translate_count(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                          size_t ws_bytes, int64_t* h_n_frags, int64_t* h_n_padded, void* stream);
int plast_translate_write(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                          size_t ws_bytes, uint8_t* d_codes, int64_t n_padded, int64_t* d_seq_start, int32_t* d_frag,
                          int64_t n_frags, void* stream);

/*
 * Stage 3.2 (Sec. 3.3.4): full gapped alignment of the hits that passed the
 * small gapped filter, with the list of ungapped pieces of the alignments
 * already computed that lets a hit lying on one of them skip its own.
 *
 * A side of an alignment is the anchored affine-gap recurrence of the gapped
 * filter with no band and no window, over the whole rest of both sequences:
 * rightward from the seed start, leftward from the letters just before it.
 * best = max over cells of H (H(0,0) = 0, so best >= 0); the end cell is the
 * first cell in row-major order (rows: bank-a letters) holding best; the path
 * is traced back preferring, for H, the diagonal, then E (a letter of b against
 * a gap), then F; for E and F, a gap opening before an extension.  score =
 * best right + best left.  Pieces are maximal runs of pairs: (diagonal
 * pos1 - pos2, first and one-past-last position in sequence a).
 * The passing hits of one sequence pair are taken in order of decreasing
 * gapped score, then increasing pos1, then pos2; a hit is covered (computes
 * nothing) when an earlier alignment of its pair has a piece on diagonal
 * pos1 - pos2 whose positions include pos1.  Hits must be distinct.
 */
typedef struct {
  int32_t seq1, seq2;        /* sequence ids in bank a, bank b */
  int32_t seed1, seed2;      /* seed start (pos1, pos2) of the hit that produced it */
  int32_t start1, end1;      /* aligned letters of seq1: [start1, end1) */
  int32_t start2, end2;      /* aligned letters of seq2: [start2, end2) */
  int32_t score;             /* raw score, best left + best right */
  int32_t length;            /* alignment columns: pairs plus gap positions */
  int32_t identities;        /* pairs of equal letters */
  int32_t mismatches;        /* pairs of different letters */
  int32_t gap_opens;         /* gap openings charged (one per run of one gap kind on each side) */
  int32_t hit;               /* index of that hit in the input list */
} plast_alignment_t;         /* 56 bytes; the tabular (-m 8 style) fields without E-values */

typedef struct {
  int32_t gap_open;          /* a gap of length k costs gap_open + k * gap_extend (11, 1) */
  int32_t gap_extend;
  int32_t max_len1;          /* longest sequence of bank a / bank b that a passing hit may lie in, */
  int32_t max_len2;          /*   1..16384 each */
  int32_t n_waves;           /* alignment wavefronts (one workgroup each); 0 = as many as stay resident */
  int32_t max_pieces;        /* capacity of one sequence pair's piece list, >= 16 */
  const int8_t* matrix;      /* host, 20x20 row-major in code order; NULL = BLOSUM62 */
} plast_align_params_t;

/* Workspace for n_hits input hits (the per-wavefront trace buffer grows with
 * max_len1 x max_len2).  A workgroup takes about 9 max_len2 bytes of LDS
 * (148 KiB at 16384, within the 160 KiB limit). */
int plast_align_workspace_bytes(int64_t n_hits, const plast_align_params_t* p, size_t* bytes);
/* d_hits / d_gscore / d_pass: n_hits records as written by plast_ungapped_extend
 * and plast_gapped_filter (only hits with d_pass != 0 are aligned).  Outputs:
 * d_out (capacity n_hits records, caller memory) receives *h_n_out alignments
 * in no particular order; d_cover[h] (n_hits int32) = the index of the hit
 * whose alignment covers hit h (h itself when it computed one), -1 when h did
 * not pass.  Synchronises the stream (twice: after the key pass and at the end).
 * Errors: PLAST_E_ARG (bad parameters, a passing hit outside its banks or in a
 * sequence longer than max_len), PLAST_E_WORKSPACE (workspace too small, or a
 * pair needing more than max_pieces pieces), PLAST_E_HIP. */
int plast_align(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, const int32_t* d_gscore,
                const uint8_t* d_pass, int64_t n_hits, const plast_align_params_t* p, void* d_ws, size_t ws_bytes,
                plast_alignment_t* d_out, int32_t* d_cover, int64_t* h_n_out, void* stream);

/*
 * Measured denominators for the rooflines (not part of the search): each probe
 * runs one kind of work at the highest rate the chip sustains (2048 workgroups
 * of 256 threads, 8 waves per SIMD), once to warm up and then reps times
 * (1..100), timed with HIP events on the stream; *rate is the best rep.
 *   PLAST_PROBE_VALU_I32     int32 add-then-max chains: operations/s (2 per update)
 *   PLAST_PROBE_VALU_PK_I16  the same on packed 16-bit integers: operations/s (4 per update)
 *   PLAST_PROBE_VALU_PK_F16  the same on packed binary16: operations/s (4 per update)
 *   PLAST_PROBE_LDS          conflict-free 32-bit LDS lookups/s
 *   PLAST_PROBE_HBM_COPY     copy of the first half of d_buf to the second: bytes/s read + written
 *   PLAST_PROBE_LDS_B64      8-byte LDS reads with the ungapped kernel's profile access (lanes spread
 *                            over 21 entries 8 bytes apart): bytes/s
 *   PLAST_PROBE_SCLK         the int32 chains with the first wavefront of each workgroup reading the
 *                            engine-clock counter (s_memtime) and the constant-rate counter
 *                            (s_memrealtime, hipDeviceAttributeWallClockRate) around its loop: *rate is
 *                            the engine clock in Hz (median over workgroups of the last launch); d_buf
 *                            needs 32 KiB more than for the other compute probes
 * d_buf: caller device memory, 256-byte aligned, at least 2 MiB for the compute
 * probes (each thread writes one int32) and 1 MiB for the copy, whose size is
 * buf_bytes (1 GiB or more gives a stable figure).  Synchronises the stream.
 * Errors: PLAST_E_ARG (null pointer, unknown kind, reps out of range,
 * misaligned buffer), PLAST_E_WORKSPACE (buffer too small), PLAST_E_HIP.
 */
enum {
  PLAST_PROBE_VALU_I32 = 0,
  PLAST_PROBE_VALU_PK_I16 = 1,
  PLAST_PROBE_VALU_PK_F16 = 2,
  PLAST_PROBE_LDS = 3,
  PLAST_PROBE_HBM_COPY = 4,
  PLAST_PROBE_LDS_B64 = 5,
  PLAST_PROBE_SCLK = 6
};
int plast_probe_peak(int32_t kind, void* d_buf, size_t buf_bytes, int32_t reps, double* rate, void* stream);

const char* plast_strerror(int code);
const char* plast_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PLAST_H */
