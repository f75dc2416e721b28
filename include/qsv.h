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
/* QSV_FLAG_PROFILE: time every launch (qsv_profile_read).
   QSV_FLAG_DEVICE_PTRS: theta, energy and grad of qsv_expval / qsv_expval_grad are
   device pointers, read and written in the order of the context's stream.
   QSV_FLAG_NULL_STREAM: with stream = NULL, order all work on the device's null
   stream (the default stream of a framework that uses it) instead of a stream
   of the library's own.
   QSV_FLAG_TUNED_PLANS: qsv_load_program plans with the options the autotuner
   found fastest for this device architecture and qubit count (complex128),
   when it has measured them (qsv_autotune, qsv_tune_import); else defaults. */
enum { QSV_FLAG_PROFILE = 1u, QSV_FLAG_DEVICE_PTRS = 2u, QSV_FLAG_NULL_STREAM = 4u, QSV_FLAG_TUNED_PLANS = 8u };

typedef struct {
  int32_t device;      /* HIP device ordinal */
  void* stream;        /* hipStream_t to order all work on; NULL = the library's own non-blocking
                          stream, or the null stream with QSV_FLAG_NULL_STREAM */
  void* arena;         /* optional device buffer the library sub-allocates from; NULL = hipMalloc */
  size_t arena_bytes;  /* size of `arena` in bytes */
  uint32_t flags;      /* QSV_FLAG_* */
} qsv_config;

/* Creates a context on cfg->device: the GPU state-vector backend that executes
   transpiled kernels (Background, CUDA-Q and high-performance simulation; the
   paper's backends are a GPU and a CPU state-vector simulator, Experiments,
   Implementation). *out is owned by the caller; free with qsv_destroy after
   every program loaded into it has been freed with qsv_program_free.
   Errors: QSV_ERR_ARG (null out, device ordinal out of range), QSV_ERR_DEVICE. */
qsv_status qsv_create(const qsv_config* cfg, qsv_context** out);
void qsv_destroy(qsv_context* ctx);
/* Message of the last failed call on ctx; owned by ctx, valid until the next call. */
const char* qsv_last_error(const qsv_context* ctx);
/* A second context on parent's device with a non-blocking stream and scratch
   of its own, driven from another host thread while the parent or other forks
   work, so their device work overlaps on the GPU. A context and its forks form
   one family: each may run (qsv_run_shots, qsv_run_batch, qsv_expval*) the
   programs any of them loaded; a program stays owned by the context that
   loaded it (replan and free it there, before that context is destroyed).
   Destroy forks before the parent. Forks cannot be forked. */
qsv_status qsv_context_fork(qsv_context* parent, qsv_context** out);

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
  QSV_OP_CLRB = 7,     /* if active: classical bit `cbit` <- 0 */
  QSV_OP_CSTORE = 8,   /* if active: classical bits [cbit, cbit + flag) <- the low `flag` bits of
                          the classical expression that starts at code[pred] */
  QSV_OP_NOISE = 9     /* if active and the call's depolarizing rate p > 0: qubit q0 takes X, Y or
                          Z with probability p/3 each, decided by the Philox word with counter
                          (noise[pred].ctr[0..2], 1) (see qsv_run_opts.depolarizing) */
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
  /* gate angle k = scale[k] * theta[param[k]] + offset[k]; param[k] = QSV_NONE -> offset[k];
     param[k] >= n_params names derived parameter param[k] - n_params */
  uint32_t param[3];
  uint32_t reserved2;
  double scale[3];
  double offset[3];
} qsv_instr;

/* QSV_CMP_EXPR: the predicate holds iff the classical expression that starts
   at code[value] is nonzero (lo and width unused). */
enum { QSV_CMP_EQ = 0, QSV_CMP_NE, QSV_CMP_LT, QSV_CMP_GT, QSV_CMP_LE, QSV_CMP_GE, QSV_CMP_TRUE, QSV_CMP_EXPR };

typedef struct {
  uint32_t lo, width;  /* classical bits [lo, lo + width) read as an unsigned integer (width <= 64) */
  uint64_t value;      /* right-hand side */
  uint32_t cmp;        /* QSV_CMP_* ; QSV_CMP_TRUE ignores the bits */
  uint32_t reserved;
} qsv_pred;

/* Classical integer expressions (OpenQASM 3 classical types and operators on
   registers and variables: the classical registers of the paper's symbol
   table, Methodology, parsing and semantic analysis) as postfix code run on a
   stack of at most 16 signed 64-bit values. An expression is a run of ops
   ending with QSV_C_END, which yields the top of the stack. Every result wraps
   to 64-bit two's complement; comparisons and logical operators give 0 or 1;
   division truncates toward zero and x / 0 = x % 0 = 0; a shift by a count
   outside 0..63 gives 0 (a right shift of a negative value then gives -1);
   right shifts are arithmetic. */
enum {
  QSV_C_END = 0,
  QSV_C_IMM,      /* push imm */
  QSV_C_BITS,     /* push classical bits [lo, lo + width) as an integer (two's complement if sgn) */
  QSV_C_NEG, QSV_C_NOT, QSV_C_LNOT,                       /* unary: -a, ~a, !a */
  QSV_C_ADD, QSV_C_SUB, QSV_C_MUL, QSV_C_DIV, QSV_C_MOD,  /* binary: a op b, b on top */
  QSV_C_AND, QSV_C_OR, QSV_C_XOR, QSV_C_SHL, QSV_C_SHR,
  QSV_C_EQ, QSV_C_NE, QSV_C_LT, QSV_C_GT, QSV_C_LE, QSV_C_GE, QSV_C_LAND, QSV_C_LOR,
  QSV_C_COUNT
};

typedef struct {
  uint8_t op;          /* QSV_C_* */
  uint8_t sgn;         /* QSV_C_BITS: 1 = signed */
  uint16_t width;      /* QSV_C_BITS: 1..64 */
  uint32_t lo;         /* QSV_C_BITS: first classical bit */
  int64_t imm;         /* QSV_C_IMM */
} qsv_cop;

typedef struct {
  uint32_t out;        /* derived parameter index (< n_derived) */
  uint32_t in;         /* input parameter index (< n_params) */
  double coef;
} qsv_lin;

/* The first three Philox counter words of one depolarizing draw (QSV_OP_NOISE).
   The lowering sets them to (gate statement index, loop code, 64 j + k): the
   statement among those outside gate definitions in source order, sum over
   the enclosing for loops of iteration ordinal << (16 * depth), application j
   of the statement (register broadcast) and operand k. */
typedef struct {
  uint64_t ctr[3];
} qsv_noise;

typedef struct {
  uint32_t n_qubits;   /* 1 .. 34 */
  uint32_t n_clbits;
  uint32_t n_params;   /* length of the theta vector */
  uint32_t n_instr;
  uint32_t n_pred;
  uint32_t reserved;
  const qsv_instr* instr;
  const qsv_pred* pred;
  uint32_t n_code;     /* classical expression code (QSV_OP_CSTORE, QSV_CMP_EXPR) */
  uint32_t reserved2;
  const qsv_cop* code;
  /* Derived parameters, for gate angles that combine several inputs: derived
     parameter k (k < n_derived) is sum of coef * theta[in] over the entries
     with out == k; a gate angle's param index n_params + k reads it. */
  uint32_t n_lin;
  uint32_t n_derived;
  const qsv_lin* lin;
  /* counters of the depolarizing slots (QSV_OP_NOISE pred indexes them) */
  uint32_t n_noise;
  uint32_t reserved3;
  const qsv_noise* noise;
} qsv_program_desc;

/* Validates and deep-copies desc, plans the GPU passes and uploads them: the
   compile step of compile-once, run-many (Background, parameter passing and
   VQE; Methodology, handling runtime parameters: `input` angles stay symbolic
   and are bound per call from theta). The stream itself is what the paper's
   AST visitor emits, with gates, measurements, resets and the feed-forward of
   `if` statements on bits and registers (Methodology, kernel generation via
   AST visitor; transpiling dynamic control flow). A program without
   parameters also has its gate matrices bound and its dense phases composed
   here, on ctx's stream (the call waits for them), once for every later call.
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
/* QSV_RUN_GRAPH: the call's launch sequence (parameter binding, phase
   composition, control-block set-up, every gate pass and measurement site,
   state materialisation) is captured once in a HIP graph and replayed by later
   calls of the same program with the same shot count, flags, forced-record
   length, error rates and state_out request; seed, shot_offset, theta and the
   forced outcomes may differ between replays (they are copied to the device
   ahead of the replay). Results are bit-identical to the uncaptured call.
   Applies when the call's shots fit one batch, without QSV_RUN_SHARE_TRAJ
   (whose host decisions between launches cannot be captured), on a context
   with a stream other than the null stream; elsewhere the flag is ignored.
   One captured sequence is kept per program (a different call replaces it);
   it refers to the context's scratch buffers and is captured again when those
   have moved. */
enum { QSV_RUN_SHARE_TRAJ = 1u, QSV_RUN_COMPLEX64 = 2u, QSV_RUN_GRAPH = 4u };

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
  double depolarizing;   /* in [0, 1]: the rate p of the program's depolarizing slots
                            (QSV_OP_NOISE; the paper's future-work depolarization, as quantum
                            trajectories): an active slot draws the word w of its own counter
                            (key (seed, shot)), u = (w >> 11) 2^-53, and applies X if u < p/3,
                            Y if u < 2p/3, Z if u < p. The draws never touch the measurement
                            stream. p > 0 needs a program with slots; each shot then binds its
                            own gate matrices, and QSV_RUN_SHARE_TRAJ has no effect.
                            qsv_run_shots only (qsv_run_batch rejects programs with slots). */
} qsv_run_opts;

typedef struct {
  uint64_t* creg;        /* [n_shots][ceil(n_clbits/64)] classical bits, LSB-first words */
  uint8_t* record;       /* [n_shots][max_events] measure outcomes in execution order, or NULL */
  uint32_t* n_events;    /* [n_shots] Philox words consumed (one per measure or reset event, plus
                            one per error draw), or NULL */
  double* record_prob;   /* [n_shots] product of the outcome probabilities, or NULL */
  int32_t* shot_status;  /* [n_shots] QSV_OK or QSV_ERR_FORCED_ZERO_PROB, or NULL */
} qsv_shot_results;

/* Runs n_shots shots of prog with parameters theta[n_params] (host): per shot,
   gate application, mid-circuit measurement (outcome drawn from the shot's
   stream, collapse, renormalisation), reset and classical feed-forward, as in
   the dynamic circuits the paper validates over repeated shots (Background,
   dynamic circuit testing; Experiments, dynamic control flow validation: the
   conditional reset run over 1000 and 10^4 shots). Outputs are host buffers.
   A shot whose forced outcome has probability < 2^-60 stops there with
   shot_status QSV_ERR_FORCED_ZERO_PROB; the call still returns QSV_OK.
   Errors: QSV_ERR_ARG (null program/creg, foreign program, theta missing,
   forced_len without forced, error rates outside [0, 1)), QSV_ERR_NOMEM,
   QSV_ERR_DEVICE. */
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
   with more qubits, requests of 18..20 qubits, and requests of 13..17 qubits
   with at least 64 shots run through qsv_run_shots with shared trajectories.
   When a batch has both kinds, those calls run on up to 12 contexts forked from
   ctx (created on first use, with scratch of their own, and destroyed with
   ctx), each driven from a host thread of its own while the persistent
   launches run, so all of them overlap on the GPU; ctx itself must not be a
   fork, use an arena, or be capturing, else they run after the launch on ctx.
   The call returns when all are done. The path is chosen from the request
   alone. Every item is
   computed the same way whatever else is in the batch, so a request's results
   do not depend on the batch it is part of. The paper runs whole suites of
   circuits of 2..20 qubits and the dynamic circuits over many shots
   (Experiments, benchmark suites; dynamic control flow validation); running
   them as one launch is this library's. Errors: QSV_ERR_ARG for a null or
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

/* energy[b] = sum_j coeff_j Re <psi(theta_b)| P_j |psi(theta_b)> for b < batch:
   the energy expectation value of the paper's VQE runs, for many parameter
   vectors of one compiled ansatz (Background, parameter passing and VQE;
   Methodology, validation framework: energies swept over input parameters;
   Experiments, hybrid compilation efficiency). theta is [batch][n_params]
   (row-major); coeff and pauli stay host arrays. With QSV_FLAG_DEVICE_PTRS set
   on the context, theta and energy are device pointers ordered on the context
   stream. Errors: QSV_ERR_ARG (null arguments, Pauli code > 3),
   QSV_ERR_UNSUPPORTED (the program measures, resets or branches). */
qsv_status qsv_expval(qsv_context* ctx, const qsv_program* prog, const double* theta, uint32_t batch,
                      const qsv_pauli_sum* h, double* energy);

/* As qsv_expval_grad with one Hamiltonian per parameter vector: h is [batch]
   (h[b] for theta row b), so requests with different Hamiltonians share one
   sweep over the batch. */
qsv_status qsv_expval_grad_each(qsv_context* ctx, const qsv_program* prog, const double* theta,
                                uint32_t batch, const qsv_pauli_sum* h, double* energy, double* grad);

/* As qsv_expval, plus grad[b][k] = dE_b / dtheta_b[k] ([batch][n_params]) by the
   adjoint method: one backward sweep that undoes the gates on psi and on
   lambda = H psi and reads each angle's derivative on the way. The paper
   binds the parameters; the gradient is this library's addition for the
   optimiser loop around them. With QSV_FLAG_DEVICE_PTRS, grad is a device
   pointer too. */
qsv_status qsv_expval_grad(qsv_context* ctx, const qsv_program* prog, const double* theta,
                           uint32_t batch, const qsv_pauli_sum* h, double* energy, double* grad);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of requests                                  */
/* ------------------------------------------------------------------------ */
/* Serving is this library's addition (the paper runs one program at a time).
   A server owns a queue of requests and three worker threads ("lanes"), each
   driving a context forked from ctx, so their device work overlaps on the GPU:
   the persistent lane runs shots requests whose states fit the persistent
   launch (up to 20 qubits with fewer than 64 shots, or up to 12 qubits), one
   slice of shots of every request it holds per launch (shots_per_tick shots
   for up to 16 qubits, all shots above), requests handed over meanwhile
   joining the next launch; the wide lane runs the other shots requests on the
   tile passes with shared trajectories, one at a time in arrival order; the
   energy lane runs energy+gradient requests, one sweep per program over every
   vector it holds (qsv_expval_grad_each). qsv_server_step retires finished
   requests (their memory returns to the budget) and admits waiting requests
   in arrival order while the HBM footprint of the admitted set stays within
   the budget (a shots request is charged 16 x 2^n bytes per state resident at
   once: its slice in the persistent lane, at most 16 shared histories in the
   wide lane; an energy request 2 x 16 x 2^n bytes; a request larger than the
   whole budget is admitted alone); it never waits for device work, so
   requests that arrive while others run are admitted at the next step. A
   request's results depend only on (program, theta, seed, shot index) or
   (program, theta, Hamiltonian), never on the other requests. Programs must
   stay loaded until their requests are fetched; server calls come from one
   host thread (the lanes never call back). */
typedef struct qsv_server qsv_server;

qsv_status qsv_server_create(qsv_context* ctx, size_t hbm_budget, uint32_t shots_per_tick, qsv_server** out);
void qsv_server_destroy(qsv_server* srv);
/* Shots request: n_shots shots of prog with theta (copied), Philox seed. */
qsv_status qsv_submit(qsv_server* srv, const qsv_program* prog, const double* theta, uint64_t n_shots,
                      uint64_t seed, uint64_t* ticket);
/* Energy + gradient request for one parameter vector (theta and h are copied). */
qsv_status qsv_submit_expval_grad(qsv_server* srv, const qsv_program* prog, const double* theta,
                                  const qsv_pauli_sum* h, uint64_t* ticket);
/* Retires finished requests and admits waiting ones (non-blocking); reports how
   many are admitted and not yet retired (running) and how many wait. */
qsv_status qsv_server_step(qsv_server* srv, uint32_t* n_running, uint32_t* n_waiting);
/* done = 1 once the request has finished (its results can be fetched). */
qsv_status qsv_poll(qsv_server* srv, uint64_t ticket, int32_t* done);
/* Copies a finished request's results (buffers sized as for qsv_run_shots /
   energy[1] and grad[n_params]) and forgets the request. */
qsv_status qsv_fetch_shots(qsv_server* srv, uint64_t ticket, qsv_shot_results* out);
qsv_status qsv_fetch_expval_grad(qsv_server* srv, uint64_t ticket, double* energy, double* grad);

/* ------------------------------------------------------------------------ */
/* Plan autotuning                                                           */
/* ------------------------------------------------------------------------ */
/* The planner's tunable choices (this library's; the paper leaves execution to
   its backends). tile_bits: qubits of the largest amplitude tile a gate pass
   holds in LDS (1..12); low_bits: qubits 0..low_bits-1 that every tile holds,
   so each global access is a contiguous run of 2^low_bits amplitudes;
   dense_min_cost: a register phase whose gates cost at least this much (a
   dense one-qubit gate costs 1) is composed into one 16x16 product applied on
   the matrix cores, cheaper ones apply gate by gate (0: never). */
typedef struct {
  uint32_t tile_bits, low_bits;
  double dense_min_cost;
} qsv_plan_options;

typedef struct {
  qsv_plan_options best;   /* the options installed in the program */
  qsv_plan_options deflt;  /* the default options (the first candidate) */
  double best_ms;          /* one call of the measured shape with best, wall time */
  double default_ms;       /* the same with the default options */
  uint32_t n_candidates;   /* plans measured */
  uint32_t reserved;
  char arch[64];           /* device architecture name the result is cached under */
} qsv_tune_report;

/* Plans prog with every candidate (tile_bits 12/11/10, low_bits 4/5,
   dense_min_cost 0.5/0/3, the default first), times qsv_run_shots(n_shots,
   run_flags & (SHARE_TRAJ | COMPLEX64)) on the device for each (one warm-up,
   best of two), installs the fastest plan in prog and records it in the
   process-wide cache under (architecture, n_qubits, precision). Every plan
   computes the same results up to floating-point rounding order. Takes about
   18 x 3 calls of that shape. Errors as qsv_run_shots. */
qsv_status qsv_autotune(qsv_context* ctx, qsv_program* prog, const double* theta, uint64_t n_shots,
                        uint32_t run_flags, qsv_tune_report* out);
/* The options prog's current plan was built with. */
qsv_status qsv_program_plan_get(const qsv_program* prog, qsv_plan_options* out);
/* Re-plans prog with explicit options (QSV_ERR_ARG when out of range). */
qsv_status qsv_program_replan(qsv_context* ctx, qsv_program* prog, const qsv_plan_options* opts);
/* Cached options for (ctx's device architecture, n_qubits, run_flags' precision):
   *found = 1 and *out set, or *found = 0 and *out the defaults. */
qsv_status qsv_tune_lookup(qsv_context* ctx, uint32_t n_qubits, uint32_t run_flags, qsv_plan_options* out,
                           int32_t* found);
/* The cache as text, one entry per line:
   "<arch> <n_qubits> <c64|c128> <tile_bits> <low_bits> <dense_min_cost> <best_ms> <default_ms>".
   *len = bytes needed including the terminating NUL; buf may be NULL to query;
   QSV_ERR_LIMIT when cap is too small. Host only. */
qsv_status qsv_tune_export(char* buf, size_t cap, size_t* len);
/* Adds entries in that format (later entries replace equal keys); lines that
   start with '#' are skipped. QSV_ERR_ARG on a malformed line (nothing is
   added then). Host only. */
qsv_status qsv_tune_import(const char* text);

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
/* Sum of a server's lane profiles (server on a context created with
   QSV_FLAG_PROFILE; the lanes' contexts inherit the flag). */
qsv_status qsv_server_profile(qsv_server* srv, qsv_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H */
