/*
 * fpm_learn.h -- learned symbol-to-field grouping for occurrence
 * fingerprints (C ABI of libfpm, companion of fpm.h).
 *
 * The paper maps each fingerprint symbol c to one bit q by a fixed rule
 * (Section 3.2: the position of c in the chosen symbol set; Section 3: the
 * common / rare / mixed sets).  Any map that sends each byte to one field or
 * to none keeps Theorem 1 (one edit changes at most two fields by at most
 * one each) and hence Eq. 1, so a map may also send several symbols to one
 * bit; such a grouping can only change how many pairs the filter rejects,
 * never drop a true match.  These entry points learn a grouping that raises
 * the rejection rate:
 *
 *   per symbol c: features x_c -> h = relu(x_c W1 + b1) -> z = h W2 + b2 ->
 *   P_c = softmax(z) over B fields and "no field";
 *   if every symbol independently picks field j with probability P_cj, bit j
 *   of a string with symbol set S is clear with probability
 *   Z_S,j = prod_{c in S} (1 - P_cj), and for a pair of symbol sets (A, B)
 *   the expected F_D = sum_j Z_A,j + Z_B,j - 2 Z_{A u B},j (exact for
 *   one-hot P: then it is the popcount of the XOR of the two fingerprints);
 *   loss per non-matching pair (exact distance > k, labelled by the
 *   verifier) = softplus(beta (2k + 1 + margin - E[F_D])) / beta, plus
 *   entropy_weight * mean_c H(P_c) to harden the assignment;
 *   map[c] = argmax_j P_cj ("no field" -> 0xFF).
 *
 * Training runs on the GPU in FP32 with the library's own kernels (MLP
 * forward, pair loss and gradient, MLP backward, Adam).  Host buffers,
 * borrowed for the call.  Errors as in fpm.h.
 */
#ifndef FPM_LEARN_H
#define FPM_LEARN_H

#include "fpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t bits;        /* fingerprint bits B: 16 or 32 (occurrence variant) */
    uint32_t k;           /* distance bound the threshold 2k refers to: 1 or 2 */
    uint32_t hidden;      /* hidden width (default 64, at most 128) */
    uint32_t epochs;      /* passes over the pairs (default 40) */
    uint32_t batch;       /* pairs per Adam step (default 65536) */
    float lr;             /* Adam learning rate (default 0.01) */
    float margin;         /* target F_D above 2k + 1 (default 0.5) */
    float beta;           /* softplus sharpness (default 2) */
    float entropy_weight; /* final entropy weight, ramped up linearly over the epochs (default 0.05) */
    uint64_t seed;        /* weight initialisation */
} fpm_learn_config;

typedef struct {
    uint32_t sigma;        /* symbols in the model (bytes that occur in the dictionary, <= 128) */
    uint32_t d_in;         /* features per symbol (sigma one-hot + 4 statistics) */
    uint32_t n_params;     /* MLP parameters */
    uint32_t steps;        /* Adam steps taken */
    uint64_t train_pairs;  /* non-matching pairs the loss saw per epoch */
    float first_loss;      /* pair loss of the first step */
    float final_loss;      /* pair loss of the last epoch (mean) */
    float final_entropy;   /* mean symbol entropy at the end (nats) */
    float expected_fd;     /* mean expected F_D over training pairs at the end */
    float ms;              /* device time of the training loop */
} fpm_learn_report;

/* Learn a grouping for occurrence fingerprints of `cfg->bits` bits.
 * Symbols are the bytes that occur in the dictionary, ordered by frequency
 * (at most 128; rarer ones never get a field).  pairs holds 2 * n_pairs
 * uint32 (query index, word index); is_match[i] != 0 marks pairs within
 * distance k (they carry no loss: no grouping can reject them).  map_out
 * receives 256 entries (field or 0xFF) usable as a custom map of
 * fpm_build_fingerprints with FPM_OCC and the same bits. */
fpm_status fpm_learn_grouping(const uint8_t *dbytes, const uint64_t *doffsets, uint32_t n_words,
                              const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t n_queries,
                              const uint32_t *pairs, const uint8_t *is_match, uint64_t n_pairs,
                              const fpm_learn_config *cfg, uint8_t map_out[256], fpm_learn_report *report);

/* One forward and backward pass of the model on the GPU, without the
 * optimizer (for gradient checks).  Host buffers: X is sigma x d_in
 * (row-major), params packs W1 (d_in x hidden), b1 (hidden), W2
 * (hidden x (bits+1)), b2 (bits+1); masks_a / masks_b hold two uint64 per
 * pair (symbols 0..63, 64..127) and only non-matching pairs are passed.
 * Outputs: P_out sigma x (bits+1), loss_out[0] = mean pair loss,
 * loss_out[1] = mean symbol entropy, loss_out[2] = mean expected F_D,
 * grads_out packed like params (gradient of pair loss + entropy_weight *
 * mean entropy). */
fpm_status fpm_learn_step(uint32_t sigma, uint32_t d_in, uint32_t hidden, uint32_t bits, uint32_t k, const float *X,
                          const float *params, const uint64_t *masks_a, const uint64_t *masks_b, uint64_t n_pairs,
                          float margin, float beta, float entropy_weight, float *P_out, float *loss_out,
                          float *grads_out);

#ifdef __cplusplus
}
#endif

#endif /* FPM_LEARN_H */
