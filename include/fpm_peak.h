/*
 * fpm_peak.h -- peak-rate probes of the two units the match kernel runs on
 * (C ABI of libfpm, companion of fpm.h).
 *
 * The match kernel's roofline is priced against the GPU's published peaks
 * (32-bit integer vector ALUs: 256 compute units x 64 lanes x 2.4 GHz =
 * 3.93e13 lane-ops/s; dense int8 matrix cores: 5.0e15 ops/s).  This entry
 * point measures both on the device it runs on, with the instruction mixes
 * the kernel uses:
 *
 *   vector ALUs: per lane, 16 uniform 32-bit values (scalar registers)
 *     against 2 lane values, each pair costing one v_xor_b32, one
 *     v_bcnt_u32_b32 with accumulator and one v_alignbit_b32 -- the vector
 *     filter's three instructions per pair (Eq. 1 test, sign bit into a
 *     mask); 8 waves per SIMD, long unrolled loops;
 *   matrix cores: back-to-back v_mfma_i32_32x32x32_i8 (2 x 32 x 32 x 32
 *     ops each), two independent accumulator chains per wave, 8 waves per
 *     SIMD.
 *
 * Each probe runs once to warm up and once timed with HIP events on a
 * stream of its own; achieved rate = operations / duration.  Allocates a
 * small device buffer for the probes' results (freed before return).
 * Errors as in fpm.h (FPM_EINVAL for a null out, FPM_EDEVICE for HIP
 * failures).
 */
#ifndef FPM_PEAK_H
#define FPM_PEAK_H

#include "fpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double int_valu_ops_per_s;    /* measured 32-bit integer VALU lane-ops per second */
    double int8_matrix_ops_per_s; /* measured dense int8 matrix ops per second */
    uint64_t valu_ops;            /* lane-ops of the timed vector probe */
    uint64_t matrix_ops;          /* int8 ops of the timed matrix probe */
    float valu_ms;                /* duration of the timed vector probe */
    float matrix_ms;              /* duration of the timed matrix probe */
    uint32_t compute_units;       /* compute units the probes covered (8 blocks of 4 waves each) */
    uint32_t reserved;
} fpm_peaks;

/* Measure both peaks on the current HIP device. */
fpm_status fpm_measure_peaks(fpm_peaks *out);

#ifdef __cplusplus
}
#endif

#endif
