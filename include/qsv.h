/*
 * qsv.h — C ABI of libqsv: state-vector execution of lowered OpenQASM 3
 * dynamic circuits on one AMD Instinct MI355X (gfx950).
 *
 * The paper (arXiv 2604.11599) transpiles OpenQASM 3 programs with mid-circuit
 * measurement, classical feed-forward (`if`/`else` on bits and multi-bit
 * register predicates) and bounded loops into kernels that a state-vector
 * backend executes, with `input` variables bound at run time so that a
 * program is compiled once and run with many parameter vectors (abstract;
 * Methodology: transpiling dynamic control flow, runtime parameters). This
 * library is that execution side: it takes the lowered instruction stream and
 * runs it shot by shot on the GPU.
 *
 * Conventions used throughout (the paper fixes none of them):
 *   - amplitudes are complex128 (re, im interleaved), index i = sum_q b_q 2^q
 *     (qubit 0 is the least significant bit);
 *   - classical bits form one flat array in declaration order; a register's
 *     integer value is sum_i c[i] 2^i;
 *   - a two-qubit gate's first operand is the control of controlled gates;
 *   - U / u3 carry no extra global phase; rz(t) = exp(-i t Z/2);
 *   - randomness: the e-th measure/reset event of shot s draws the e-th 64-bit
 *     word of Philox4x64-10 with key (seed, shot_offset + s) and block counter
 *     e/4 + 1 (the stream numpy.random.Philox(key=[seed, shot]) produces);
 *     u = (word >> 11) * 2^-53 and the outcome is 0 iff u < p0 / (p0 + p1).
 *
 * Errors: every call returns a qsv_status and never aborts or throws; on error
 * outputs are unspecified and qsv_last_error(ctx) describes the failure.
 * Threading: a context is used by one host thread at a time.
 * Memory: the caller owns every buffer passed in; the library copies what it
 * keeps (programs are deep-copied at load).
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qsv_status;
enum {
  QSV_OK = 0,
  QSV_ERR_ARG = -1,              /* bad argument (null pointer, size mismatch) */
  QSV_ERR_PARSE = -2,            /* reserved for the host-side OpenQASM lowering */
  QSV_ERR_UNSUPPORTED = -3,      /* e.g. expectation value of a dynamic program */
  QSV_ERR_NOMEM = -4,            /* device memory exhausted */
  QSV_ERR_DEVICE = -5,           /* a HIP runtime call failed */
  QSV_ERR_FORCED_ZERO_PROB = -6, /* per-shot: a forced outcome had probability < 2^-60 */
  QSV_ERR_LIMIT = -7             /* a static limit was exceeded (qubits, flags, sizes) */
};

typedef struct qsv_context qsv_context;
typedef struct qsv_program qsv_program;

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */
enum { QSV_FLAG_PROFILE = 1u, QSV_FLAG_DEVICE_PTRS = 2u };

typedef struct {
  int32_t device;      /* HIP device ordinal */
  void* stream;        /* hipStream_t to order all work on; NULL = the library's own stream */
  void* arena;         /* optional device buffer the library sub-allocates from; NULL = hipMalloc */
  size_t arena_bytes;  /* size of `arena` in bytes */
  uint32_t flags;      /* QSV_FLAG_* */
} qsv_config;

/* Creates a context on cfg->device. *out is owned by the caller; free with qsv_destroy
   after every program loaded into it has been freed with qsv_program_free. */
qsv_status qsv_create(const qsv_config* cfg, qsv_context** out);
void qsv_destroy(qsv_context* ctx);
/* Message of the last failed call on ctx; owned by ctx, valid until the next call. */
const char* qsv_last_error(const qsv_context* ctx);

/* ------------------------------------------------------------------------ */
/* Lowered program (the instruction stream)                                  */
/* ------------------------------------------------------------------------ */
/*
 * A program is a straight-line stream of guarded instructions. Structured
 * control flow is lowered by the front end:
 *   if (p) A else B   ->  SETF f_t <- p ; SETF f_e <- !p ; A guarded by f_t ; B by f_e
 *   for i in [a:b] S  ->  SETF f_l <- true ; S unrolled (b - a + 1) times, guarded by f_l
 *   break             ->  CLRF f_l (guarded by the enclosing conditions)
 * Each shot carries 64 flag bits. An instruction is active for a shot iff
 * (flags & guard) == guard. SETF sets flag `flag` to (active && predicate);
 * CLRF clears it when active. Predicates are evaluated when the instruction
 * executes, so a branch condition is latched at its `if` (the paper's feed-
 * forward: the predicate is read from the bits measured so far at run time).
 */
enum {
  QSV_OP_GATE = 1,     /* unitary gate `kind` on q0 (and q1) */
  QSV_OP_MEASURE = 2,  /* measure q0 into classical bit `cbit` (cbit = QSV_NONE: discard) */
  QSV_OP_RESET = 3,    /* reset q0 to |0>: a measurement (one draw) followed by X if 1 */
  QSV_OP_SETF = 4,     /* flag <- active && pred */
  QSV_OP_CLRF = 5,     /* if active: flag <- 0 */
  QSV_OP_SETB = 6,     /* if active: classical bit `cbit` <- 1 (classical assignment) */
  QSV_OP_CLRB = 7      /* if active: classical bit `cbit` <- 0 */
};

enum {
  QSV_G_ID = 0, QSV_G_X, QSV_G_Y, QSV_G_Z, QSV_G_H, QSV_G_S, QSV_G_SDG, QSV_G_T, QSV_G_TDG,
  QSV_G_SX, QSV_G_SXDG,
  QSV_G_RX, QSV_G_RY, QSV_G_RZ, QSV_G_P, QSV_G_U,        /* U(theta, phi, lambda) */
  QSV_G_CX, QSV_G_CY, QSV_G_CZ, QSV_G_CH, QSV_G_SWAP,    /* first operand = control */
  QSV_G_CP, QSV_G_CRX, QSV_G_CRY, QSV_G_CRZ,
  QSV_G_COUNT
};

#define QSV_NONE 0xFFFFFFFFu

typedef struct {
  uint8_t op;          /* QSV_OP_* */
  uint8_t kind;        /* QSV_G_* for gates */
  uint16_t reserved;
  uint32_t q0, q1;     /* qubit operands (q1 = QSV_NONE for one-qubit gates) */
  uint32_t cbit;       /* MEASURE target bit, or QSV_NONE */
  uint32_t pred;       /* SETF: index into the predicate table */
  uint32_t flag;       /* SETF/CLRF: flag bit 0..63 */
  uint64_t guard;      /* guard mask over the flag bits */
  /* gate angle k = scale[k] * theta[param[k]] + offset[k]; param[k] = QSV_NONE -> offset[k] */
  uint32_t param[3];
  uint32_t reserved2;
  double scale[3];
  double offset[3];
} qsv_instr;

enum { QSV_CMP_EQ = 0, QSV_CMP_NE, QSV_CMP_LT, QSV_CMP_GT, QSV_CMP_LE, QSV_CMP_GE, QSV_CMP_TRUE };

typedef struct {
  uint32_t lo, width;  /* classical bits [lo, lo + width) read as an unsigned integer (width <= 64) */
  uint64_t value;      /* right-hand side */
  uint32_t cmp;        /* QSV_CMP_* ; QSV_CMP_TRUE ignores the bits */
  uint32_t reserved;
} qsv_pred;

typedef struct {
  uint32_t n_qubits;   /* 1 .. 34 */
  uint32_t n_clbits;
  uint32_t n_params;   /* length of the theta vector */
  uint32_t n_instr;
  uint32_t n_pred;
  uint32_t reserved;
  const qsv_instr* instr;
  const qsv_pred* pred;
} qsv_program_desc;

/* Validates and deep-copies desc, plans the GPU passes and uploads them.
   Errors: QSV_ERR_ARG (malformed stream: qubit/bit/flag/predicate out of range),
   QSV_ERR_LIMIT (more than 34 qubits). *out is freed with qsv_program_free. */
qsv_status qsv_load_program(qsv_context* ctx, const qsv_program_desc* desc, qsv_program** out);

typedef struct {
  uint32_t n_qubits, n_clbits, n_params;
  uint32_t max_events;   /* upper bound of measure events per shot (record length) */
  uint32_t n_passes;     /* planned tile passes (unconditional count) */
  uint32_t n_sites;      /* planned measurement sites */
  uint8_t is_unitary;    /* no measure/reset/flags: expval/expval_grad allowed */
} qsv_program_info;

qsv_status qsv_program_info_get(const qsv_program* prog, qsv_program_info* out);
void qsv_program_free(qsv_program* prog);

/* ------------------------------------------------------------------------ */
/* Shots                                                                     */
/* ------------------------------------------------------------------------ */
/* QSV_RUN_SHARE_TRAJ: shots whose measurement and reset outcomes (and so
   classical bits, flags and records) are identical so far share one state:
   gate passes run once per distinct history, a site's histogram is taken once
   per history and every shot still draws its own outcome from its own Philox
   stream; a history splits where its shots' outcomes differ. A split copies the
   state only before the next gate pass writes it, so a final measure-all adds
   no copies. Results are bit-identical to running every shot on its own. */
/* QSV_RUN_COMPLEX64: the state is held and evolved in complex64 (single
   precision amplitudes, single-precision matrix-core products), the precision
   of the GPU runs in the paper's experimental setup (Experiments,
   Implementation). Probabilities are summed in double precision from the
   single-precision amplitudes; outcomes, records and feed-forward work as in
   complex128, so results differ from the complex128 run only where a draw
   falls within the single-precision error of its threshold. Gate matrices
   are bound in double precision and rounded once where they are applied.
   state_out is still complex128 (the complex64 amplitudes widened). Applies
   to qsv_run_shots only. */
enum { QSV_RUN_SHARE_TRAJ = 1u, QSV_RUN_COMPLEX64 = 2u };

typedef struct {
  uint64_t seed;         /* Philox key word 0 */
  uint64_t shot_offset;  /* shot s uses Philox key word 1 = shot_offset + s */
  const uint8_t* forced; /* NULL, or [n_shots][forced_len] outcomes for the first
                            forced_len measure events of each shot (resets are never forced) */
  uint32_t forced_len;
  uint32_t flags;        /* QSV_RUN_* */
  double* state_out;     /* NULL, or host [2^n][2] doubles: shot 0's state at program end */
  double readout_error;  /* in [0, 1): after a measurement's outcome is drawn (the state keeps
                            it), the shot's next Philox word u flips the recorded bit (record and
                            classical bit) when u < readout_error; 0: no draw */
  double reset_error;    /* in [0, 1): after a reset, the next word u leaves the qubit flipped
                            when u < reset_error; 0: no draw */
} qsv_run_opts;

typedef struct {
  uint64_t* creg;        /* [n_shots][ceil(n_clbits/64)] classical bits, LSB-first words */
  uint8_t* record;       /* [n_shots][max_events] measure outcomes in execution order, or NULL */
  uint32_t* n_events;    /* [n_shots] Philox words consumed (one per measure or reset event, plus
                            one per error draw), or NULL */
  double* record_prob;   /* [n_shots] product of the outcome probabilities, or NULL */
  int32_t* shot_status;  /* [n_shots] QSV_OK or QSV_ERR_FORCED_ZERO_PROB, or NULL */
} qsv_shot_results;

/* Runs n_shots shots of prog with parameters theta[n_params] (host). Outputs are
   host buffers. A shot whose forced outcome has probability < 2^-60 stops there
   with shot_status QSV_ERR_FORCED_ZERO_PROB; the call still returns QSV_OK. */
qsv_status qsv_run_shots(qsv_context* ctx, const qsv_program* prog, const double* theta,
                         uint64_t n_shots, const qsv_run_opts* opts, qsv_shot_results* out);

/* ------------------------------------------------------------------------ */
/* Shots without device allocation                                           */
/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate device memory: code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc. Same
   arguments, results and errors as qsv_run_shots, and bit-identical results,
   but every device buffer the call needs besides the caller's own (theta and
   gate matrices, states, control blocks, classical bits, records, reduction
   partials, forced outcomes, the state_out staging) is carved from a fixed
   device array of QSV_NOALLOC_SCRATCH_BYTES per device. The library takes that
   array's address when a context is created on the device; the array exists
   from the moment the library is loaded there until the process ends. The
   call makes no hipMalloc, hipFree or other allocating call, and records no
   profiling events. Shots run in batches that fit the array (a 20-qubit
   complex128 shot needs 16 MiB, plus 16 MiB of staging with state_out).
   QSV_ERR_LIMIT when one shot of the program does not fit. Every call on a
   device shares that device's array and leaves the last call's contents in it;
   each call initialises what it reads. Calls that overlap on one device (host
   threads driving contexts of the same device at once) race on the array and
   must be serialised by the caller. */
#define QSV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
qsv_status qsv_run_shots_noalloc(qsv_context* ctx, const qsv_program* prog, const double* theta,
                                 uint64_t n_shots, const qsv_run_opts* opts, qsv_shot_results* out);

/* ------------------------------------------------------------------------ */
/* Batches of requests in one persistent launch                              */
/* ------------------------------------------------------------------------ */
/* A request: every shot of one loaded program with its own parameters, Philox
   key and outputs (sized as for qsv_run_shots; opts.flags and opts.state_out are
   ignored). qsv_run_batch runs the shots of all requests as work items of one
   persistent launch: workgroups take items from a queue, so circuits of
   different widths and trajectories of different lengths (loop exits, taken
   branches) share the GPU. States of up to 12 qubits stay in LDS for the whole
   program; states of 13..20 qubits live in a per-workgroup HBM slot; requests
   with more qubits, and requests of 13..20 qubits with at least 64 shots, run
   through qsv_run_shots (shots sharing the deterministic prefix) after the
   launch. The path is chosen from the request alone. Every item is
   computed the same way whatever else is in the batch, so a request's results
   do not depend on the batch it is part of. Errors: QSV_ERR_ARG for a null or
   foreign program or missing outputs, QSV_ERR_NOMEM when the slots do not fit. */
typedef struct {
  const qsv_program* prog;
  const double* theta;     /* host [n_params], may be NULL when n_params == 0 */
  uint64_t n_shots;
  qsv_run_opts opts;
  qsv_shot_results out;
} qsv_request;

qsv_status qsv_run_batch(qsv_context* ctx, const qsv_request* reqs, uint32_t n_reqs);

/* ------------------------------------------------------------------------ */
/* Expectation values and gradients (unitary programs only)                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t n_terms;
  uint32_t reserved;
  const double* coeff;   /* [n_terms] real coefficients */
  const uint8_t* pauli;  /* [n_terms][n_qubits] 0 = I, 1 = X, 2 = Y, 3 = Z */
} qsv_pauli_sum;

/* energy[b] = sum_j coeff_j Re <psi(theta_b)| P_j |psi(theta_b)> for b < batch.
   theta is [batch][n_params]. With QSV_FLAG_DEVICE_PTRS set on the context,
   theta and energy are device pointers ordered on the context stream. */
qsv_status qsv_expval(qsv_context* ctx, const qsv_program* prog, const double* theta, uint32_t batch,
                      const qsv_pauli_sum* h, double* energy);

/* As qsv_expval, plus grad[b][k] = dE_b / dtheta_b[k] by the adjoint method. */
qsv_status qsv_expval_grad(qsv_context* ctx, const qsv_program* prog, const double* theta,
                           uint32_t batch, const qsv_pauli_sum* h, double* energy, double* grad);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of requests                                  */
/* ------------------------------------------------------------------------ */
/* A server owns a queue of requests. qsv_server_step runs one scheduling tick:
   waiting requests are admitted in arrival order while the HBM footprint of
   the admitted set stays within the budget (footprint of a shots request =
   its per-tick shot slice x 16 x 2^n bytes, where the slice is shots_per_tick
   for n <= 16 and shots_per_tick / 2^(n-16) (at least 1) above; of an
   energy+gradient request 2 x 16 x 2^n bytes); then one slice of every admitted shots request runs in
   a single persistent launch (qsv_run_batch) and every admitted
   energy+gradient request is evaluated; requests that finish are retired and
   their memory is released, so requests that arrive while others run join at
   the next tick. A shot's results depend only on (program, theta, seed, shot
   index), never on the other requests. Programs must stay loaded until their
   requests are fetched. */
typedef struct qsv_server qsv_server;

qsv_status qsv_server_create(qsv_context* ctx, size_t hbm_budget, uint32_t shots_per_tick, qsv_server** out);
void qsv_server_destroy(qsv_server* srv);
/* Shots request: n_shots shots of prog with theta (copied), Philox seed. */
qsv_status qsv_submit(qsv_server* srv, const qsv_program* prog, const double* theta, uint64_t n_shots,
                      uint64_t seed, uint64_t* ticket);
/* Energy + gradient request for one parameter vector (theta and h are copied). */
qsv_status qsv_submit_expval_grad(qsv_server* srv, const qsv_program* prog, const double* theta,
                                  const qsv_pauli_sum* h, uint64_t* ticket);
/* One tick; reports how many requests are admitted (running) and waiting. */
qsv_status qsv_server_step(qsv_server* srv, uint32_t* n_running, uint32_t* n_waiting);
/* done = 1 once the request has finished (its results can be fetched). */
qsv_status qsv_poll(qsv_server* srv, uint64_t ticket, int32_t* done);
/* Copies a finished request's results (buffers sized as for qsv_run_shots /
   energy[1] and grad[n_params]) and forgets the request. */
qsv_status qsv_fetch_shots(qsv_server* srv, uint64_t ticket, qsv_shot_results* out);
qsv_status qsv_fetch_expval_grad(qsv_server* srv, uint64_t ticket, double* energy, double* grad);

/* ------------------------------------------------------------------------ */
/* Profiling (contexts created with QSV_FLAG_PROFILE)                        */
/* ------------------------------------------------------------------------ */
/* Kernel time is measured with HIP events recorded on the context stream
   around every launch. "Algorithmic" bytes and flops count what the method
   needs, not what the hardware moved: a tile pass over S shots of n qubits
   reads and writes 2 * 16 * 2^n * S bytes (the pass that also prepares
   |0...0> only writes, 16 * 2^n * S bytes); its flops are the gate arithmetic
   (14 per amplitude for a dense 2x2 gate, 6 for a diagonal one, 7 for a
   controlled 2x2, 1.5 for a controlled phase, 0 for permutations). Only passes
   whose gates are unconditional are counted in the *_uncond figures, since a
   guarded pass skips shots at run time. */
typedef struct {
  uint64_t pass_launches;        /* all tile-pass launches */
  double pass_ms;                /* their summed kernel time */
  uint64_t pass_uncond_launches; /* launches of passes without guarded gates */
  double pass_uncond_ms;
  double pass_uncond_bytes;      /* algorithmic HBM bytes of those launches */
  double pass_uncond_flops;      /* algorithmic flops of those launches */
  uint64_t site_launches;        /* measurement reduce + finalize launches */
  double site_ms;
  uint64_t other_launches;       /* init, bind, compose, reductions and copies */
  double other_ms;
  uint64_t ham_launches;         /* lambda = H psi and the energy partials */
  double ham_ms;
  double ham_bytes;              /* 16 B per amplitude read (psi), 16 written (lambda, gradients only) */
  uint64_t sweep_launches;       /* adjoint sweeps over the passes (backward gate passes) */
  double sweep_ms;
  double sweep_bytes;            /* 64 B per amplitude: psi and lambda, each read and written */
  uint64_t persistent_launches;  /* persistent batch launches (qsv_run_batch) */
  double persistent_ms;
  double persistent_bytes;       /* 32 B per amplitude of every streamed (13..20-qubit) state per
                                    pass it runs, 16 per measurement site reduction; states in LDS
                                    move no HBM bytes */
} qsv_profile;

/* Copies the counters accumulated since the last reset. QSV_ERR_ARG if ctx was
   created without QSV_FLAG_PROFILE. */
qsv_status qsv_profile_read(qsv_context* ctx, qsv_profile* out);
qsv_status qsv_profile_reset(qsv_context* ctx);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H */
