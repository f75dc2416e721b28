/*
 * qsv_diag.h — diagnostics of libqsv.
 *
 * qsv_diag_copy copies `bytes` bytes (a multiple of 16) from device buffer src
 * to device buffer dst with a plain streaming kernel on the context stream and
 * waits for it. Its only use is to calibrate hardware byte counters: a copy of
 * B bytes reads B and writes B bytes of HBM, so the counters' readings for it
 * give the scale for the readings of the simulation kernels. Ownership: the
 * caller owns both buffers. Errors: QSV_ERR_ARG (null pointer or size not a
 * multiple of 16), QSV_ERR_DEVICE.
 */
#ifndef QSV_DIAG_H
#define QSV_DIAG_H

#include "qsv.h"

#ifdef __cplusplus
extern "C" {
#endif

qsv_status qsv_diag_copy(qsv_context* ctx, void* dst, const void* src, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* QSV_DIAG_H */
