/*
 * qs.h -- C ABI of the CZ-partition circuit simulator for MI355X (gfx950).
 *
 * Method (Chen et al., "64-qubit quantum circuit simulation", arXiv 1802.06952):
 * every CZ gate that crosses a chosen cut of the qubits is rewritten as
 * P0 x I + P1 x Z (Sec. 2.1, Eq. 1; Supp. A, Eq. 2), so a circuit with c such
 * gates is the sum of 2^c copies, each the tensor product of an upper and a
 * lower half circuit with no entangling gate between them (Supp. A, Eq. 7-8).
 * The amplitude of an output bitstring x is the sum over copies k of
 * U_k[u(x)] * L_k[l(x)], where u(x) and l(x) are the bits of x on the upper and
 * lower qubits (Sec. 2.3.1: sample each half, take the tensor product, add).
 *
 * Conventions shared by every call:
 *   - A circuit is a sequence of layers ("cycles"); each layer holds gates on
 *     disjoint qubits (Supp. A, the layer graphs G_t = (V_t, E_t)).  Gates:
 *     h, t, sx (square root of X), sy (square root of Y), cz, and the
 *     controlled gates cx and cy (control first; Supp. Eq. 1).
 *   - Bit q of a bitstring (uint64) is the outcome of qubit q.  Bits >= n must
 *     be zero.
 *   - Cut j is the j-th crossing CZ ordered by (layer, upper endpoint id); copy
 *     k carries bit s_j = (k >> (c-1-j)) & 1 (earliest cut = most significant).
 *     P_{s_j} acts on the upper endpoint and Z^{s_j} on the lower endpoint.
 *   - Inside a half, qubits are numbered in ascending global id.
 *   - Amplitudes are complex64 pairs (re, im) of float; the half states are
 *     complex64 with FP32 arithmetic on the GPU.
 *
 * Errors: every call returns a qs_status; no exception crosses the ABI.  On
 * failure out-parameters are left untouched, handles stay valid, and
 * qs_last_error() returns a message for the calling thread.
 * Ownership: handles are created by qs_* calls and released by the matching
 * qs_*_free; every input array belongs to the caller and is copied before the
 * call returns; output arrays belong to the caller.  Device memory belongs to
 * the plan, comes from qs_options.alloc, and is released by qs_plan_free.
 * Threads: a plan is not thread-safe; different plans may be used from
 * different threads and streams at the same time.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QS_OK = 0,
  QS_ERR_ARG = -1,          /* invalid argument (range, null pointer, size) */
  QS_ERR_PARSE = -2,        /* malformed circuit text */
  QS_ERR_UNSUPPORTED = -3,  /* valid request this library does not handle */
  QS_ERR_OOM = -4,          /* device or host allocation failed / over budget */
  QS_ERR_HIP = -5,          /* a HIP runtime call failed */
  QS_ERR_STATE = -6         /* call out of order (e.g. bitstrings not registered) */
} qs_status;

typedef enum {
  QS_PREC_FP32 = 0,        /* assembly GEMM on FP32 MFMA, FP32 accumulation */
  QS_PREC_SPLIT_BF16 = 1   /* each FP32 operand split into bf16 hi + lo; hi*hi + hi*lo + lo*hi
                              on BF16 MFMA with FP32 accumulation */
} qs_precision;

typedef struct qs_circuit qs_circuit; /* opaque, host memory */
typedef struct qs_plan qs_plan;       /* opaque, owns device buffers */

/* Device memory for a plan's buffers.  alloc returns `bytes` of device memory
 * on the current device, aligned to 256 bytes, or NULL on failure (the call
 * that needed it then fails with QS_ERR_OOM); free releases a pointer that
 * alloc returned.  ctx is passed back unchanged.  The library calls them only
 * from inside qs_* calls, on the calling thread, and frees a buffer only when
 * no queued kernel uses it any more (after a device synchronisation).  Both
 * NULL: hipMalloc and hipFree.  The Python binding passes PyTorch's caching
 * allocator here. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} qs_allocator;

/* Tuning knobs; a zero field means "choose automatically". */
typedef struct {
  int tile_bits;          /* largest tile of a full-state pass, in qubits (7..11 for halves of
                             7+ qubits: 6 over the lanes of a wavefront, the rest in registers) */
  int coalesce_bits;      /* low qubits always inside a tile (contiguous runs of 2^b amplitudes) */
  int tail_max_qubits;    /* largest light cone the leaf evaluation accepts (0..10) */
  int materialize_level;  /* force the last materialised tree level (-1 = cost model) */
  int plain;              /* 1 = the paper's flat per-copy form, for comparison: every copy
                             simulated from |0> on its own (no shared prefix), one gate per
                             full-state pass, full leaf states then a gather */
  size_t mem_budget;      /* bytes of device memory the plan may hold for states; 0 = 80 % of
                             the device's memory.  Fixed once per plan (the first run), and
                             shared by whatever runs at the same time (the two halves on two
                             streams, the t parts of a chain), so the same inputs always give
                             the same schedule */
  int one_stream;         /* 1 = run the two halves one after the other on hip_stream; 0 = the
                             lower half on a stream of the plan (default priority), ordered
                             after the work queued on hip_stream by an event and joined back
                             into hip_stream by another before the assembly */
  uint64_t copies_per_launch; /* most copies one block of qs_run_halves holds (a power of two,
                             0 = as many as the range allows): each block's passes and leaf
                             evaluation run over all of its copies in one launch each, and
                             blocks run one after another */
  int max_stages;         /* tree levels one full-state pass may descend at once (1..2, 0 = 2):
                             a pass reads a level, branches through the next levels' cut bits
                             and gates in registers and writes only the deepest one; the
                             planner picks where each pass lands */
  int min_tile_bits;      /* smallest tile of a full-state pass (7..tile_bits, 0 = 8): a pass's
                             tile holds its gates' qubits, padded up to this many */
  int no_exchange;        /* 1: every full-state pass is a launch of its own; 0: runs of passes
                             without a branch whose register bits fit in 3 more bits run as
                             one launch on workgroup tiles that pass through LDS between the
                             passes (one HBM read and write per run; same results) */
  qs_allocator alloc;     /* every device buffer of the plan (states, gathered half amplitudes,
                             descriptors, copy tables, assembly workspace) comes from here */
} qs_options;

/* Message describing the last failed call on this thread ("" if none). */
const char* qs_last_error(void);

/* Parse circuit text (format: "qubits <n>" then one gate per line,
 * "<layer> <gate> <q> [<q2>]", '#' comments).  The text is the layered circuit
 * of Supp. A: layer t holds the gates of G_t = (V_t, E_t), each CZ an edge of
 * E_t, no qubit in two gates of one layer; the one-qubit gates are those of
 * the random circuits of Sec. 2.2 (H, square roots of X and Y, T).  Layers
 * must not decrease.  n <= 64.  On success *out owns a new circuit (host
 * memory).  Errors: QS_ERR_ARG (null pointers), QS_ERR_PARSE (unknown gate,
 * qubit out of range, a qubit twice in a layer, decreasing layers). */
qs_status qs_load_circuit(const char* text, size_t len, qs_circuit** out);

/* Number of qubits and gates of a parsed circuit (either pointer may be NULL). */
qs_status qs_circuit_info(const qs_circuit* circ, int* n_qubits, int* n_gates);

void qs_circuit_free(qs_circuit* circ);

/* Build a plan for the bipartition given by upper_mask (bit q set = qubit q in
 * the upper half V1; Supp. A).  Classifies the crossing CZ gates (the set
 * E_int of Supp. A), builds the two half programs and uploads nothing yet.
 * opts may be NULL.  The plan keeps its own copy of the circuit.
 * Errors: QS_ERR_ARG (mask empty, full, or naming qubits >= n; a half with
 * more than 32 qubits), QS_ERR_UNSUPPORTED (more than 40 cut gates). */
qs_status qs_partition(const qs_circuit* circ, uint64_t upper_mask, const qs_options* opts,
                       qs_plan** out);

/* Sizes of a plan: qubits per half and number of cut gates (copies = 1 << n_cuts). */
qs_status qs_plan_info(const qs_plan* plan, int* n_upper, int* n_lower, int* n_cuts);

/* JSON description of the plan for the first copy block of [copy_begin,
 * copy_end) as qs_run_halves would split the range (cuts, half programs, tree
 * levels, passes, light-cone qubits, cost estimate), for tests.  Host only.
 * Writes at most cap bytes including the terminating NUL; *needed receives
 * the full size including the NUL.  buf may be NULL when cap is 0.
 * Errors: QS_ERR_ARG (null pointers, range outside [0, 2^c)). */
qs_status qs_plan_dump(const qs_plan* plan, uint64_t copy_begin, uint64_t copy_end, char* buf,
                       size_t cap, size_t* needed);

void qs_plan_free(qs_plan* plan);

/* Cost of a bipartition, before any simulation (host only).  The paper
 * estimates a partition's time by Eq. 2 (Sec. 2.2: gates per layer times the
 * number of half circuits) and its memory by the equivalent qubits N_e
 * (Sec. 3); this library's own schedule is cheaper than that flat count. */
typedef struct {
  int n_cuts;            /* c: CZ gates between the halves (copies = 2^c) */
  int n_upper, n_lower;  /* qubits of the halves */
  int equivalent_qubits; /* N_e (Sec. 3): the larger half plus c + 1 */
  double flat_updates;   /* Eq. 2's work in gate-amplitude updates: every copy runs every gate of
                            each half on its full state, 2^c (G_up 2^n_upper + G_lo 2^n_lower),
                            G counting the half's H, one-qubit and internal CZ gates plus one per
                            cut gate */
  double plan_cost;      /* this library's schedule of all 2^c copies with n_values requested
                            values per half: the planner's estimate in HBM byte-equivalents
                            (full-state passes, leaf evaluation, launches; both halves) plus
                            the product-set assembly of n_values x n_values amplitudes
                            (FP32 MFMA flops at 8 TB/s per 157.3 TFLOP/s) */
} qs_cut_score;

/* Score the bipartition upper_mask of circ for n_values requested values per
 * half (>= 1).  Errors: QS_ERR_ARG (null pointers, n_values < 1, and the mask
 * errors of qs_partition), QS_ERR_UNSUPPORTED (more than 40 cut gates, or no
 * schedule the kernels can run). */
qs_status qs_score_cut(const qs_circuit* circ, uint64_t upper_mask, int n_values,
                       qs_cut_score* out);

/* Choose among n_masks candidate bipartitions the one with the smallest
 * criterion (0: flat_updates, the paper's Eq. 2 accounting; 1: plan_cost, this
 * library's schedule); masks that qs_score_cut rejects are skipped, ties go to
 * the first.  *best receives the index into masks, *best_score (may be NULL)
 * its score.  Errors: QS_ERR_ARG (null pointers, n_masks 0, n_values < 1,
 * unknown criterion), QS_ERR_UNSUPPORTED (no candidate can be scored). */
qs_status qs_choose_cut(const qs_circuit* circ, const uint64_t* masks, size_t n_masks,
                        int n_values, int criterion, size_t* best, qs_cut_score* best_score);

/* Simulate the copies k in [copy_begin, copy_end) of both halves on the GPU
 * and keep, for each, the half amplitudes at the upper and lower parts of the
 * m bitstrings (host array).  The first call registers the bitstrings (they
 * must form, up to a factor 4, a product set of upper x lower values: Sec.
 * 2.3.1 samples the halves and takes their tensor product); later calls pass
 * the same set (same values, same order) or bitstrings = NULL and m = 0 for
 * the registered set, and add further copy ranges; a copy range may not be run
 * twice.  Asynchronous on hip_stream (a hipStream_t, NULL = default stream)
 * once the plan has seen the same copy blocks before; the first call of a
 * block plans it and uploads its descriptors (host work, one stream sync).
 * Assembly: when the distinct upper values times the distinct lower values
 * are at most 4m + 1024 (the product sets of Sec. 2.3.1: sample each half,
 * take the tensor product) the sum over copies is a GEMM over the whole
 * value grid; otherwise every bitstring gets its own sum over copies (FP32
 * accumulation for either precision).
 * Errors: QS_ERR_ARG (range outside [0, 2^c), empty, bits >= n, no
 * bitstrings), QS_ERR_STATE (different bitstrings, overlapping range),
 * QS_ERR_UNSUPPORTED (a tree the kernels cannot hold), QS_ERR_OOM, QS_ERR_HIP. */
qs_status qs_run_halves(qs_plan* plan, uint64_t copy_begin, uint64_t copy_end,
                        const uint64_t* bitstrings, size_t m, void* hip_stream);

/* Amplitudes of the m bitstrings summed over every copy run so far (the whole
 * circuit when all 2^c copies were run, a partial sum for a slice): the sum
 * over copies k of U_k[u(x)] L_k[l(x)] of Supp. A, Eq. (8), i.e. the tensor
 * products of the sampled half amplitudes added up as in Sec. 2.3.1.  If no
 * copy has been run yet, runs all copies first with these bitstrings.  The
 * bitstrings must be the registered set.  out_c64 receives 2*m floats (re, im)
 * in host memory.  out_stats (nullable, host) receives three doubles computed
 * in FP64 on the GPU: sum |a|^2, 2^n * mean |a|^2, 2^(2n) * mean |a|^4.
 * Synchronises hip_stream.  out_c64 and out_stats are written only when the
 * call succeeds.  Errors: QS_ERR_ARG, QS_ERR_STATE, QS_ERR_OOM, QS_ERR_HIP. */
qs_status qs_amplitudes(qs_plan* plan, const uint64_t* bitstrings, size_t m, qs_precision prec,
                        float* out_c64, double* out_stats, void* hip_stream);

/* Per-copy half amplitudes of an already run copy range [copy_begin,
 * copy_end) (exactly one qs_run_halves range or a block of one): side 0 =
 * upper, 1 = lower.  out_c64 (host) receives (copy_end - copy_begin) * S
 * complex64 values, row k - copy_begin holding the half amplitudes of copy k
 * at the S distinct registered half values (ascending packed half index:
 * bit i = the i-th qubit of the half in ascending global id); *n_values
 * receives S.  cap is the capacity of out_c64 in complex values.  These are
 * the U_k[u] (side 0) and L_k[l] (side 1) of Supp. A, Eq. (8), whose sum over
 * k of products is the amplitude.  Synchronises hip_stream.
 * Errors: QS_ERR_ARG (null pointers, side, cap too small), QS_ERR_STATE
 * (range not run as one block), QS_ERR_HIP. */
qs_status qs_half_amplitudes(qs_plan* plan, int side, uint64_t copy_begin, uint64_t copy_end,
                             float* out_c64, size_t cap, size_t* n_values, void* hip_stream);

/* Device-resident variant of qs_amplitudes for the registered bitstrings:
 * d_out_c64 (device, 2*m floats in registration order) and d_out_sums (device,
 * nullable, 2 doubles: sum |a|^2 and sum |a|^4 in FP64) are written on
 * hip_stream without any host transfer or synchronisation.  Copies must have
 * been run.  Errors: QS_ERR_ARG, QS_ERR_STATE, QS_ERR_HIP. */
qs_status qs_amplitudes_device(qs_plan* plan, qs_precision prec, float* d_out_c64,
                               double* d_out_sums, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as qs_amplitudes_device, with every temporary buffer of the assembly (the
 * value grid, split-K partial products, split-BF16 operand planes, FP64
 * partial sums) taken from a static region of 256 MiB per device that the
 * library holds until the process ends, instead of from the plan's
 * allocator.  The call allocates nothing and creates no event (timing, if
 * enabled, skips it); it still needs the plan's run copies and its
 * registered bitstrings, as qs_amplitudes_device does.  Every call on one
 * device shares that device's region: calls that overlap on one device (on
 * different streams, or from different threads) race and must not be made.
 * Errors: QS_ERR_ARG, QS_ERR_STATE (no copies run), QS_ERR_UNSUPPORTED (the
 * assembly needs more than 256 MiB of scratch; about 56 MiB in FP32 and
 * 190 MiB in split-BF16 for 1024 x 1024 values over 2^14 copies), QS_ERR_HIP. */
qs_status qs_amplitudes_device_static(qs_plan* plan, qs_precision prec, float* d_out_c64,
                                      double* d_out_sums, void* hip_stream);

/* Forget every run copy of the plan.  keep_bitstrings = 1 keeps the
 * registered bitstrings (a new round of qs_run_halves may pass NULL);
 * 0 forgets them too.  Device buffers and cached block plans are kept. */
qs_status qs_plan_reset(qs_plan* plan, int keep_bitstrings);

/* Device time in milliseconds, measured with HIP events on the plan's stream,
 * accumulated since qs_set_timing(plan, 1), by kernel family:
 * out[0] full-state passes, out[1] leaf evaluation, out[2] assembly GEMM,
 * out[3] gather and FP64 reductions; out[4..7] the number of launches of each
 * family; out[8] the algorithmic bytes of the full-state passes (reads and
 * writes of the half states), out[9] the assembly flops (8 M N K per block,
 * FP32-equivalent), out[10] the 2x2-gate flops of the leaf evaluation (14 per
 * amplitude per gate on the light-cone subspaces).  Synchronises with the
 * recorded events.  out has 11 doubles. */
qs_status qs_get_timing(qs_plan* plan, double* out11);
/* enable: 0 off, 1 per kernel family (events around each family's launches),
 * 2 also around every full-state pass launch (qs_get_pass_timing).  Clears the
 * totals.  Timing adds events to the stream; leave it off when capturing a
 * graph.  Errors: QS_ERR_ARG. */
qs_status qs_set_timing(qs_plan* plan, int enable);

/* Every full-state pass launch timed since qs_set_timing(plan, 2), in launch
 * order, as 8 doubles: half (0 upper, 1 lower), index in that half's schedule
 * of the launch's first pass, input tree level, branch stages (tree levels
 * descended), wavefront tiles (or workgroups) of one pass, algorithmic bytes
 * (8 B per amplitude of every state read and written; the last pass only its
 * listed tiles), milliseconds (HIP events on the launch stream), and the
 * number of passes the launch ran (more than one for a group of passes that
 * exchange their tiles through LDS).  Writes min(n, cap_records) records to
 * out (caller-owned, 8 * cap_records doubles) and the total count to
 * *n_records.  Synchronises with the recorded events.  Errors: QS_ERR_ARG,
 * QS_ERR_HIP. */
qs_status qs_get_pass_timing(qs_plan* plan, double* out, size_t cap_records, size_t* n_records);

/* One step of the hot path as a HIP graph: every copy in [copy_begin,
 * copy_end) of both halves (qs_run_halves on the registered bitstrings) and
 * the assembly with its FP64 sums (qs_amplitudes_device), launched as one
 * graph on hip_stream.  The batching of Sec. 2.3.1 (many copies, many layer
 * passes) then costs one launch per step.  The first call, and any call whose
 * arguments or stream differ from the captured ones, runs one eager step
 * (planning and filling the plan's buffer pool), captures the next step and
 * launches it; later calls only launch the graph (asynchronous).  The graph
 * is captured again after the plan released device memory (a new bitstring
 * set, a full buffer pool).  Results are those of the eager calls, bit for
 * bit.  Needs registered bitstrings (QS_ERR_STATE otherwise: call
 * qs_run_halves with them once); d_out_c64 / d_out_sums as in
 * qs_amplitudes_device (device memory, 2m floats / 2 doubles or NULL).
 * hip_stream must not be the null stream (it cannot be captured).  Timing
 * events are not recorded inside the graph.  Errors: QS_ERR_ARG, QS_ERR_STATE,
 * QS_ERR_OOM, QS_ERR_HIP (capture or instantiation failed). */
qs_status qs_run_graph(qs_plan* plan, uint64_t copy_begin, uint64_t copy_end, qs_precision prec,
                       float* d_out_c64, double* d_out_sums, void* hip_stream);

/* ---------------------------------------------------------------- chain partitions
 *
 * Partitions into t parts (Sec. 3, Fig. 3): part_masks[0..t-1] are disjoint,
 * non-empty, at most 32 qubits each and cover the circuit; every cut gate
 * (a two-qubit gate with its endpoints in two parts) must join parts i and
 * i+1, as row bands of a grid do.  A cut CZ is rewritten by Eq. (1) with P_b
 * on its endpoint in the even-numbered part and Z^b on the one in the
 * odd-numbered part; the 2^c copies are the products of t part circuits and
 * an amplitude is the sum over copies of the product of the t part
 * amplitudes, computed as a chain of t - 1 complex FP32 products over the
 * cut bits that neighbouring parts share.  Each part runs the same kernels as
 * a half of qs_partition (copy tree, full-state passes, leaf evaluation).
 * Cut gates are numbered by (layer, endpoint in the lower-numbered part);
 * part p sees only the cuts of links p-1 and p.
 *
 * The plan holds host copies of the circuit and masks and owns its device
 * buffers; it is not thread-safe.  Errors: QS_ERR_ARG (null pointers, t
 * outside 2..8, masks that overlap, leave a qubit out, are empty or exceed 32
 * qubits), QS_ERR_UNSUPPORTED (a cut gate joins parts that are not
 * neighbours, more than 30 cuts touch one part: a part's 2^c_p copies run as
 * one block). */
typedef struct qs_mplan qs_mplan;
qs_status qs_partition_chain(const qs_circuit* circ, const uint64_t* part_masks, int t,
                             const qs_options* opts, qs_mplan** out);

/* *t, part_qubits[p] (t entries) and link_cuts[i] (t - 1 entries: cuts between
 * parts i and i+1); any of them may be NULL. */
qs_status qs_chain_info(const qs_mplan* plan, int* t, int* part_qubits, int* link_cuts);

/* Register m >= 1 host bitstrings (bit q = qubit q).  The products run over
 * the grid of distinct part values, which must stay within 2^28 amplitudes
 * (QS_ERR_UNSUPPORTED otherwise): product sets over the parts fit best.
 * Registering a different set on the same plan: QS_ERR_STATE. */
qs_status qs_chain_register(qs_mplan* plan, const uint64_t* bitstrings, size_t m);

/* All copies of every part, the chain of products, the gather of the m
 * registered amplitudes into d_out_c64 (2m floats, device) and the FP64 sums
 * [sum p, sum p^2] into d_out_sums (2 doubles, device, may be NULL), on
 * hip_stream; asynchronous.  QS_ERR_STATE if nothing is registered. */
qs_status qs_chain_amplitudes_device(qs_mplan* plan, float* d_out_c64, double* d_out_sums,
                                     void* hip_stream);

/* Register bitstrings (as qs_chain_register), compute, and copy the amplitudes
 * to out_c64 (2m floats, host) and, when out_stats is not NULL, [sum p,
 * 2^n mean p, 2^2n mean p^2] to out_stats; synchronises hip_stream. */
qs_status qs_chain_amplitudes(qs_mplan* plan, const uint64_t* bitstrings, size_t m,
                              float* out_c64, double* out_stats, void* hip_stream);

void qs_chain_free(qs_mplan* plan);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
