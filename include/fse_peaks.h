/*
 * fse_peaks.h -- measured device peaks, for the roofline fractions that the
 * benchmark reports beside the published ones.  Not part of the method: four
 * microbenchmarks timed with HIP events on the current device.
 */
#ifndef FSE_PEAKS_H
#define FSE_PEAKS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double fp32_fma_tflops;  /* vector FMA in float, no packed instructions */
  double fp64_fma_tflops;  /* vector FMA in double */
  double lds_read_tbps;    /* LDS reads (16 bytes per lane, no bank conflicts), all CUs */
  double hbm_copy_tbps;    /* device-to-device copy, bytes read + written */
  int32_t compute_units;
  int32_t reserved;
} fse_peaks;

/* Run the four microbenchmarks on the current device (a few hundred
 * milliseconds; allocates and frees 2 GiB of device memory) and fill `out`
 * with the best of several timed runs each.  Errors: FSE_ERR_INVALID (null
 * pointer), FSE_ERR_DEVICE (a HIP call failed), FSE_ERR_NOMEM (the copy
 * buffers could not be allocated). */
int32_t fse_measure_peaks(fse_peaks *out);

#ifdef __cplusplus
}
#endif
#endif
