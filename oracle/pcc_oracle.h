/*
 * pcc_oracle.h -- plain, slow, single-threaded CPU reference of the
 * cluster-preserving correction of lossy-compressed particle data
 * (Ren, Di, Heitmann, Cappello, Guo: "Preserving Clusters in Error-Bounded
 * Lossy Compression of Scientific Particle Data").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call it.  It shares no code with the GPU
 * library and the GPU library never calls it.
 *
 * Everything is computed in IEEE double precision from float32 inputs, with
 * floating-point contraction disabled, following the paper's definitions:
 *   Sec. 2.4    friends-of-friends links (d <= b) and their components;
 *   Sec. 3.1    the 2*sqrt(3)*xi distance perturbation bound, potentially-
 *               broken / potentially-created pairs, the vulnerable set V,
 *               active set A, editable set E, loss (Eq. 1), box (Eq. 2);
 *   Sec. 3.2    the vulnerable-pair, safe-component and halo-forest modes;
 *   Alg. 1      the correction loop, edits, flags and quantised edits;
 *   Sec. 3.3    the safety margins, tightened loss (Eq. 3), Huffman + ZSTD,
 *               reconstruction of the edited data;
 *   Sec. 4.2    Adam with alpha 1e-3, beta1 0.9, beta2 0.999, eps 1e-8.
 * Readings of points the paper leaves open are stated where they are used.
 *
 * Pins (tests/test_oracle_*.py): hand-derived dyadic fixtures for the pair
 * classes, labels and active sets; exhaustive O(N^2) search and breadth-first
 * components; a library minimum spanning tree for the halo forest; scalar
 * two-particle recurrences and the first-step closed form for the loop; a
 * hand-assembled stream for the decoder; the end-to-end theorems (zero
 * membership errors, |x' - x| <= xi, link preservation in VP mode).
 * Parity unpinned: the trajectory of many interacting particles beyond these
 * special cases (the paper prints none), and the stream bytes themselves.
 */
#ifndef PCC_ORACLE_H
#define PCC_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_VP = 0, ORC_SC = 1, ORC_HF = 2 };
enum { ORC_ADAM = 0, ORC_SGD = 1 };
enum { ORC_MARGIN_SAFE = 0, ORC_MARGIN_PAPER = 1 };
/* pair classes */
enum { ORC_NONE = 0, ORC_SAFE = 1, ORC_PB = 2, ORC_PC = 3 };
/* status */
enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_E_INVALID = -1, ORC_E_INPUT_BOUND = -5 };
/* linking lengths of one multi-threshold correction, at most */
#define ORC_MAX_THRESHOLDS 8

typedef struct {
  double b;            /* linking length */
  double xi;           /* absolute pointwise error bound */
  int32_t mode;        /* ORC_VP / ORC_SC / ORC_HF */
  int32_t m_bits;      /* edit bit depth: 8, 16 or 32 */
  int32_t optimizer;   /* ORC_ADAM or ORC_SGD */
  int32_t margin_policy;
  double lr, beta1, beta2, adam_eps;
  int64_t max_iters;   /* <= 0 selects the safety cap of 100000 */
  double loss_tol;     /* 0: stop when no active pair is violated */
  double box[3];       /* periodic side per axis, 0 = open axis */
} orc_params;

typedef struct {
  double rs, rv;           /* b -+ 2 sqrt(3) xi */
  double b2, rs2, rv2;     /* squared thresholds (rs2 < 0 when rs <= 0) */
  double eps_q;            /* maximum quantisation error of one edit */
  double qstep;            /* quantiser step */
  double delta_q;          /* per-coordinate decode error bound */
  double xi_p;             /* projection box half-width */
  double delta_t;          /* distance margin of the tightened loss */
  double bm, bp, bm2, bp2; /* b -+ delta_t and their squares */
} orc_consts;

typedef struct {
  uint32_t i, j;   /* i < j, particle indices */
  double d2;       /* squared (minimum-image) distance, float64 */
} orc_pair;

typedef struct {
  int32_t status;
  int64_t iters;                  /* gradient steps taken */
  int64_t n_pairs, n_safe, n_pb, n_pc;
  int64_t n_active, n_editable, n_flagged;
  double loss0, loss_final;
  int64_t viol0, viol_final;
  /* malloc'd arrays, released by orc_result_free */
  int32_t *labels;                /* [n] FoF labels (minimum member index) */
  int32_t *safe_labels;           /* [n] safe-component labels */
  int64_t n_a;
  uint32_t *a_i, *a_j;            /* active pairs, i < j, sorted by (i, j, threshold) */
  uint8_t *a_type;                /* ORC_PB or ORC_PC */
  uint8_t *a_thr;                 /* threshold index of each active pair */
  int64_t n_e;
  uint32_t *e_ids;                /* editable particles, ascending */
  double *p;                      /* [3*n] planar x|y|z, final float64 coords */
  double *loss_hist;              /* [iters+1] tightened loss at each check */
  int64_t *viol_hist;             /* [iters+1] violated active pairs */
  uint8_t *stream;                /* edit stream */
  int64_t stream_len;
} orc_result;

void orc_params_default(orc_params *p);
/* maxabs: largest |coordinate| over the original and reconstructed inputs */
void orc_constants(const orc_params *p, double maxabs, orc_consts *c);
double orc_max_abs(int64_t n, const float *const xyz[3], const float *const rec[3]);
int orc_classify(double d2, const orc_consts *c);
double orc_dist2(const float *const xyz[3], int64_t i, int64_t j, const double box[3]);

/* All unordered pairs with squared distance <= r2, sorted by (i, j).
 * *out is malloc'd; returns the count (or -1 on allocation failure). */
int64_t orc_pairs(int64_t n, const float *const xyz[3], const double box[3],
                  double r2, orc_pair **out);

/* Components of the graph whose edges are the pairs of the given classes.
 * which = 0: safe links; which = 1: all links (safe or potentially broken). */
void orc_components(int64_t n, const orc_pair *pairs, int64_t np,
                    const orc_consts *c, int which, int32_t *labels);

/* Active set of a mode; returns |A| and malloc'd arrays sorted by (i, j). */
int64_t orc_select(int mode, int64_t n, const orc_pair *pairs, int64_t np,
                   const orc_consts *c, const int32_t *safe_labels,
                   const int32_t *fof_labels, const float *const rec[3],
                   const double box[3], uint32_t **a_i, uint32_t **a_j,
                   uint8_t **a_type);

/* The whole correction (Alg. 1) with every intermediate result. */
int orc_correct(int64_t n, const float *const xyz[3], const float *const rec[3],
                const orc_params *p, orc_result *r);
void orc_result_free(orc_result *r);

/* The correction for several linking lengths at once (the extension the
   conclusion, Sec. 5 under Limitations, notes: the union of the selected
   pair sets of every threshold).
   b_list[0..nb) replaces p->b (nb <= ORC_MAX_THRESHOLDS); every threshold's
   constraints are selected as in orc_correct and each keeps its own
   b -+ delta_t in the loss; the active list is sorted by (i, j, threshold).
   labels_all, if not NULL, receives the FoF labels at every b ([nb][n]). */
int orc_correct_multi(int64_t n, const float *const xyz[3], const float *const rec[3],
                      const orc_params *p, const double *b_list, int32_t nb,
                      int32_t *labels_all, orc_result *r);

/* Decode an edit stream and apply it to the reconstruction (Sec. 3.3). */
int orc_decode(const uint8_t *stream, int64_t len, int64_t n,
               const float *const rec[3], float *const out[3]);

/* FoF labels (minimum member index) of a point set at linking length b. */
int orc_fof_labels(int64_t n, const float *const xyz[3], double b,
                   const double box[3], int32_t *labels);

void orc_free(void *ptr);

#ifdef __cplusplus
}
#endif
#endif
