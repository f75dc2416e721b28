/*
 * qsv_plan.h — host-only inspection of the planner of libqsv.
 *
 * Runs the same validation and planning as qsv_load_program but touches no
 * device: it exists so that the host logic (how the lowered instruction stream
 * of a dynamic circuit is cut into tile passes and measurement sub-sites) can
 * be tested on machines without a GPU. Ownership: the caller owns *out.
 * Errors: QSV_ERR_ARG (null pointer or a malformed stream), QSV_ERR_LIMIT
 * (more than 34 qubits).
 */
#ifndef QSV_PLAN_H
#define QSV_PLAN_H

#include "qsv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QSV_PLAN_MAX_STEPS 4096
#define QSV_PLAN_MAX_GATES 65536

enum { QSV_STEP_INIT = 0, QSV_STEP_PASS = 1, QSV_STEP_SITE = 2 };

typedef struct {
  uint32_t n_steps, n_passes, n_sites, n_gates, n_events, max_record;
  uint8_t is_unitary;
  uint8_t init_step;                         /* 1: step 0 writes |0...0> on its own */
  uint8_t reserved[6];
  uint8_t step_kind[QSV_PLAN_MAX_STEPS];     /* QSV_STEP_* per step (first QSV_PLAN_MAX_STEPS) */
  uint64_t step_mask[QSV_PLAN_MAX_STEPS];    /* pass: tile qubit mask; site: histogrammed qubits */
  uint32_t step_count[QSV_PLAN_MAX_STEPS];   /* pass: gates; site: events */
  uint32_t gate_instr[QSV_PLAN_MAX_GATES];   /* instruction index of each planned gate, in order */
  uint64_t gate_regs[QSV_PLAN_MAX_GATES];    /* qubits held in registers while the gate runs
                                                (0: LDS-only pass) */
  uint32_t n_phases;                         /* register phases over all passes */
  uint32_t n_dense_phases;                   /* phases applied as one composed 16x16 matrix */
  uint32_t n_mfma_sweep_passes;              /* passes whose adjoint sweep (qsv_expval_grad) runs on
                                                the matrix cores: all phases dense, 2^10..2^12
                                                amplitudes per tile */
} qsv_plan_stats;

/* tile_bits = 0 uses the default tile width (12 bits). */
qsv_status qsv_plan_inspect(const qsv_program_desc* desc, uint32_t tile_bits, qsv_plan_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* QSV_PLAN_H */
