/*
 * tcx.h - C ABI of an MI355X (gfx950) tensor-network circuit contraction
 * executor.
 *
 * What it computes (arXiv:2205.10091, TensorCircuit):
 *   - section "Tensor network engine": a parameterised circuit's diagram is a
 *     tensor network (gate tensors plus product-state boundary vectors); an
 *     amplitude or an expectation value is obtained by contracting its edges
 *     until a single node remains, in an order chosen by a path finder, and
 *     the contraction itself is a sequence of pairwise einsum/matmul steps
 *     ("Schematic of the quantum circuit components" figure: path search
 *     first, backend contraction second);
 *   - section "Basic circuits and outputs": amplitudes <bits|U|0...0>;
 *   - sections "Pauli string expectation" and "Explicit loop with
 *     c.expectation_ps": E = sum_j alpha_j <psi|P_j|psi>, each Pauli term
 *     contracted as one network (the reuse=False form of section "Custom
 *     contraction settings");
 *   - section "Gradients, optimization and variational algorithms": dE/dtheta;
 *   - section "vmap and vectorized_value_and_grad / Batched VQE": many
 *     parameter vectors evaluated against one compiled plan.
 *
 * Conventions.  Qubit 0 is the most significant position of a bitstring
 * and of a gate's matrix index (section "Circuits and gates /
 * Preliminaries").  Rotation gates are R_G(t) = exp(-i t G / 2).  Complex
 * numbers crossing the ABI are pairs of doubles (re, im).
 *
 * Errors.  Every call returns a tc_status.  Outputs are written only when
 * TC_OK is returned.  tc_last_error() gives a thread-local message for the
 * most recent failure on the calling thread.  No C++ exception crosses the
 * ABI.
 *
 * Ownership.  Objects returned through an out-pointer (tc_network, tc_path,
 * tc_plan, tc_server) belong to the library and are released with the
 * matching *_free call; freeing NULL is a no-op.  Caller arrays passed in
 * (circuits, observables, parameters) are copied or consumed before the call
 * returns unless stated otherwise.
 *
 * Threads.  Distinct objects may be used from distinct threads.  A plan
 * accepts one contraction call at a time (TC_ERR_BUSY otherwise).
 */
#ifndef TCX_H
#define TCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TC_OK = 0,
  TC_ERR_INVALID_ARG = 1,   /* malformed input: bad qubit, size, pointer */
  TC_ERR_UNSUPPORTED = 2,   /* unknown gate kind, option not available   */
  TC_ERR_OUT_OF_MEMORY = 3, /* host or device allocation failed          */
  TC_ERR_TOO_LARGE = 4,     /* plan needs more device memory than allowed */
  TC_ERR_DEVICE = 5,        /* a HIP call failed                         */
  TC_ERR_BUSY = 6,          /* object already has a call in flight       */
  TC_ERR_STATE = 7          /* call not valid in the object's state      */
} tc_status;

const char* tc_status_string(tc_status s);
const char* tc_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t tc_version(void);

/* ------------------------------------------------------------------ circuit
 * Gate kinds (section "Circuits and gates": standard gates, exp1-type
 * rotations, arbitrary unitaries).  Matrices are indexed with q[0] the
 * more significant qubit.  Not in the paper, standard definitions:
 *   SQRT_X/Y/W = ((1+i)/2) I + ((1-i)/2) G with W = (X+Y)/sqrt 2;
 *   FSIM(t, p) = [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],
 *                 [0,0,0,exp(-i p)]].
 * Channels with externalised randomness (sections "Externalizing the
 * randomness", "Batched Monte Carlo trajectory noise simulation" and
 * "Demonstration of barren plateaus"): the random number ("status", in
 * [0,1)) is an angle argument, so a parameter slot per batch row makes each
 * row one trajectory or one circuit structure.  [0,1) is cut into intervals
 * in the listed order, and the operator of the interval holding the status
 * is applied (a unitary: the channel's Kraus operators are multiples of
 * unitaries).  The cuts are computed and compared in float32.
 *   DEPOL   angle 0 = status; matrix = 3 doubles (px, py, pz), each >= 0,
 *           sum <= 1; applies I, X, Y, Z with probabilities
 *           1 - px - py - pz, px, py, pz (cuts p0 = ((1 - px) - py) - pz,
 *           p0 + px, (p0 + px) + py).
 *   RSWITCH angle 0 = t, angle 1 = status; applies RX(t), RY(t), RZ(t) for
 *           status < 1/3, < 2/3, else.
 * The gradient of a status is 0 (the choice is piecewise constant).
 */
typedef enum {
  TC_GATE_H = 0, TC_GATE_X = 1, TC_GATE_Y = 2, TC_GATE_Z = 3, TC_GATE_S = 4,
  TC_GATE_SQRT_X = 5, TC_GATE_SQRT_Y = 6, TC_GATE_SQRT_W = 7,
  TC_GATE_RX = 8, TC_GATE_RY = 9, TC_GATE_RZ = 10,
  TC_GATE_U1 = 11,                       /* caller 2x2 matrix             */
  TC_GATE_CNOT = 12, TC_GATE_CZ = 13,
  TC_GATE_RZZ = 14, TC_GATE_RXX = 15, TC_GATE_RYY = 16,
  TC_GATE_FSIM = 17,                     /* two angles (theta, phi)       */
  TC_GATE_U2 = 18,                       /* caller 4x4 matrix             */
  TC_GATE_DEPOL = 19,                    /* Monte Carlo depolarizing      */
  TC_GATE_RSWITCH = 20                   /* RX / RY / RZ chosen per row   */
} tc_gate_kind;

typedef struct {
  int32_t kind;        /* tc_gate_kind                                     */
  int32_t q[2];        /* target qubits; q[1] ignored for 1-qubit gates    */
  int32_t param[2];    /* slot in the parameter vector per angle, or -1    */
  double fixed[2];     /* angle used where param[i] == -1                  */
  const double* matrix;/* U1: 8 doubles, U2: 32 doubles, (re,im) pairs,
                          row-major; NULL otherwise.  Copied at build.     */
} tc_gate;

typedef struct {
  int32_t n_qubits;    /* 1 .. 4096                                        */
  int32_t n_params;    /* length of one parameter vector (>= 0)            */
  int32_t n_gates;
  const tc_gate* gates;/* applied in order to |0...0>                      */
} tc_circuit;

/* --------------------------------------------------------------- observable
 * AMPLITUDE: <bits|U|0...0> (section "Basic circuits and outputs").
 * PAULI_SUM: sum_j weights[j] <psi|P_j|psi> with structure vectors
 * structures[j*n_qubits + q] in {0=I,1=X,2=Y,3=Z} (section "Pauli structures
 * and weights").  The weighted sum is reduced in FP64 in a fixed order.
 * MPO: <psi|M|psi> for an operator given as a matrix product operator
 * (sections "Expectations of Hamiltonians via operator_expectation", MPO
 * input, and "QuOperator as the operator to be measured"):
 *   M[i_1..i_n; j_1..j_n] = sum over bonds of prod_k T_k[b_{k-1}, b_k, i_k, j_k]
 * contracted as ONE network (ket, the n site tensors, conjugated ket)
 * instead of one network per Pauli term.  Site k is a D_{k-1} x D_k x 2 x 2
 * array (left bond, right bond, row = out index, column = in index) of
 * (re, im) doubles, row-major; the sites are concatenated in `mpo`;
 * mpo_bonds[k-1] = D_k for the n-1 inner bonds, each in 1..8 (D_0 = D_n = 1).
 * A bond of dimension D becomes ceil(log2 D) legs of dimension 2, the
 * padded entries zero.  No light cone applies (M acts on every qubit).
 * STATE: the network <psi|psi> (ket and conjugated ket joined on every
 * wire); contracted it gives the squared norm, and it is the network of
 * the geometric tensor (tc_plan_opts.qgt, tc_contract_qgt).
 */
typedef enum { TC_OBS_AMPLITUDE = 0, TC_OBS_PAULI_SUM = 1, TC_OBS_MPO = 2,
               TC_OBS_STATE = 3 } tc_obs_kind;

typedef struct {
  int32_t kind;               /* tc_obs_kind                               */
  const uint8_t* bits;        /* AMPLITUDE: n_qubits entries in {0,1}, or
                                 NULL for all zeros                        */
  int32_t n_terms;            /* PAULI_SUM: number of terms (>= 1)         */
  const uint8_t* structures;  /* PAULI_SUM: n_terms * n_qubits             */
  const double* weights;      /* PAULI_SUM: n_terms                        */
  const int32_t* mpo_bonds;   /* MPO: n_qubits - 1 inner bond dimensions   */
  const double* mpo;          /* MPO: the site tensors (copied at build)   */
} tc_observable;

/* ------------------------------------------------------------------ network
 * tc_build_network: translate circuit + observable into one tensor network
 * per term (section "Tensor network engine").  An expectation term is the
 * network <0|U^dagger P_j U|0>: ket gate tensors, Pauli matrices on the
 * measured qubits, and entrywise-conjugated gate tensors for the bra.
 *
 * Options:
 *   split_2q   split RZZ/RXX/RYY/CNOT/CZ into two three-leg tensors joined
 *              by a bond of dimension 2 (exact rank-2 operator-Schmidt
 *              form; section "Very large circuit simulation", gate split);
 *   lightcone  drop gates outside the backward light cone of each Pauli
 *              term (exact: a gate that does not touch the support of the
 *              conjugated operator cancels with its mirror image; a run of
 *              consecutive diagonal gates (Z, S, RZ, CZ, RZZ) commutes, so
 *              only its gates touching the support at the run's end are
 *              kept and the support grows by their qubits only; U1/U2
 *              matrices may be non-unitary and are always kept);
 *   absorb_1q  before path search, contract every tensor of rank <= 2 into
 *              a neighbour (section "Custom contraction settings",
 *              preprocessing=True).  Applied by tc_greedy_path.
 * A NULL opts pointer means {split_2q=1, lightcone=1, absorb_1q=1}.
 * Errors: INVALID_ARG for out-of-range or repeated qubits, bad structure
 * values, negative sizes, param slots >= n_params; UNSUPPORTED for unknown
 * gate kinds.
 */
typedef struct tc_network tc_network;

typedef struct {
  int32_t split_2q;
  int32_t lightcone;
  int32_t absorb_1q;
} tc_build_opts;

tc_status tc_build_network(const tc_circuit* circuit,
                           const tc_observable* observable,
                           const tc_build_opts* opts, tc_network** out);
void tc_network_free(tc_network* net);

typedef struct {
  int32_t n_qubits;
  int32_t n_params;
  int32_t n_terms;        /* 1 for an amplitude                            */
  int32_t max_leaves;     /* largest number of leaf tensors of a term      */
  int64_t total_leaves;
} tc_network_info;

tc_status tc_network_info_get(const tc_network* net, tc_network_info* out);

/* Leaf tensors of one term, for inspection and host-side checks.  For leaf
 * i: kind[i] (0 gate, 1 |0> vector, 2 <bit| vector, 3 Pauli matrix, 4 MPO
 * site), gate[i] (gate index, the bit / Pauli value for kinds 1-3, the site
 * for kind 4), part[i]
 * (0 whole gate, 1 first split factor, 2 second split factor), conj[i] (1
 * for bra copies), rank[i] and legs[4*i + r] (leg labels, most significant
 * first).  Element e of a leaf is the entry whose r-th leg has value
 * (e >> (rank-1-r)) & 1.  Whole gates have legs (out..., in...); split
 * factors have legs (bond, out, in) and equal P_k (first) and c_k P_k
 * (second) with P_0 = I, P_1 = the gate's Pauli (Z for CZ, X for CNOT's
 * target) and c_k from the gate; MPO sites have legs (left bond bits...,
 * right bond bits..., out, in).  Arrays have max_leaves entries (legs:
 * 8*max_leaves, unused entries -1); *n_leaves receives the count. */
tc_status tc_network_term_leaves(const tc_network* net, int32_t term,
                                 int32_t* n_leaves, int32_t* kind,
                                 int32_t* gate, int32_t* part, int32_t* conj,
                                 int32_t* rank, int32_t* legs);

/* --------------------------------------------------------------------- path
 * tc_greedy_path: host-side pairwise greedy path per term (section "Custom
 * contraction settings": the default greedy finder; FLOPs / WRITE / SIZE
 * metrics).  Each step contracts the pair of tensors sharing a leg that
 * minimises size(out) - size(a) - size(b); ties go to fewer flops, then to
 * smaller ids.  With n_trials > 1 each further trial perturbs that cost with
 * seeded Gumbel noise of the given temperature and the tree with the best
 * score is kept.  Deterministic for a fixed seed.
 *
 * score: 0 flops, 1 write, 2 size, 3 combo = flops + 64 * write (the
 * default combination named in the contractor table of that section),
 * 4 time = an execution-time estimate on this executor: flops at
 * 10 TFLOP/s, written elements at 2 TB/s and 6 us per tree level (levels
 * are dependent launches).  Beside the greedy trials two candidates are
 * scored: a sweep in time order (ket gates, observable, conjugated gates)
 * and, for networks whose leaves sit on wires, per-wire column tensors
 * merged left to right or as a balanced binary tree over wires.
 * flops count 8 real operations per complex multiply-add.
 */
typedef struct tc_path tc_path;

typedef enum { TC_SCORE_FLOPS = 0, TC_SCORE_WRITE = 1, TC_SCORE_SIZE = 2,
               TC_SCORE_COMBO = 3, TC_SCORE_TIME = 4 } tc_score;

typedef struct {
  uint64_t seed;
  int32_t n_trials;      /* >= 1                                          */
  int32_t score;         /* tc_score                                      */
  double temperature;    /* noise scale for trials after the first        */
  int32_t reconf_k;      /* 0 = off; 3..10: subtree reconfiguration of the
                            chosen tree, frontiers of up to reconf_k inputs
                            re-contracted optimally (exact dynamic program
                            over subsets, flops/8 + 64 write), kept when
                            the score improves                           */
  int32_t max_depth;     /* 0 = off; > 0: each term's tree is the best-
                            scoring candidate with at most max_depth tree
                            levels (the shallowest candidate when none has
                            so few).  The deepest term sets the number of
                            dependent level launches of a plan, so a cap on
                            the few deepest terms trades their flops for
                            fewer launches.  -1 = the cap that minimises
                            4 us per level of the deepest term plus 0.45 ps
                            per flop of all terms (a launch-bound small-node
                            time model), over the depths the candidates of
                            all terms reach                              */
} tc_path_opts;

tc_status tc_greedy_path(const tc_network* net, const tc_path_opts* opts,
                         tc_path** out);
/* A path from caller SSA pairs for one term: pairs[2*s], pairs[2*s+1] are
 * ids of tensors alive before step s (leaves 0..n_leaves-1, step s creates
 * id n_leaves+s); n_steps must be n_leaves-1.  Other terms keep the greedy
 * path of `base` (required, same network). */
tc_status tc_path_replace_term(tc_path* base, int32_t term,
                               const int32_t* pairs, int32_t n_steps);
void tc_path_free(tc_path* path);

/* tc_slice: a network contracted as a sum of smaller ones (section
 * "Outlook and concluding remarks": slicing, to go past memory limits and
 * to spread one contraction over devices).  For every term whose tree in
 * `path` has an intermediate above 2^max_log2_size elements, bond labels
 * are chosen on that tree (the label carried by the most of its largest
 * intermediates, repeatedly) until every intermediate fits; the term then
 * becomes 2^s terms of the same weight, each with the s bonds cut and
 * capped by the basis vectors of one assignment of their values, and its
 * path is the original tree with the caps absorbed first.  Contracting the
 * new network (with the new path) gives the same value and gradient.
 * Returns a new network and path (library-owned, freed with *_free) and
 * the largest s over the terms.  TOO_LARGE if more than max_labels (<= 16)
 * labels would be needed; INVALID_ARG for a path of another network. */
tc_status tc_slice(const tc_network* net, const tc_path* path, int32_t max_log2_size,
                   int32_t max_labels, tc_network** out_net, tc_path** out_path,
                   int32_t* n_sliced_labels);

typedef struct {
  double log10_flops;    /* over all terms                                */
  double log2_write;     /* total elements written by contraction steps   */
  double log2_size;      /* largest intermediate (elements)               */
  double flops;
  double write;
  double size;
  int32_t n_steps;       /* pairwise contractions over all terms          */
  int32_t max_depth;     /* deepest tree                                  */
} tc_path_stats;

tc_status tc_path_stats_get(const tc_path* path, int32_t term /* -1: all */,
                            tc_path_stats* out);
/* The SSA pairs of one term (2*(n_leaves-1) ints). */
tc_status tc_path_term_pairs(const tc_path* path, int32_t term,
                             int32_t* pairs, int32_t* n_steps);

/* --------------------------------------------------------------------- plan
 * tc_plan_create compiles network + path into device work: leaf materialisation
 * from parameters, the contraction tree as level-ordered batched kernels
 * (small nodes: a gather-contraction kernel; wide nodes: coalesced permute
 * plus MFMA complex GEMM), the FP64 root reduction and, with want_grad, the
 * reverse sweep.  Host-only: no device memory is touched until
 * tc_plan_bind (or the first contraction call, which binds with
 * library-allocated memory).
 *
 *   precision   0 = complex64 with FP32 MFMA (default); 1 = split-BF16
 *               (hi+lo, three BF16 MFMA products, FP32 accumulation) on
 *               wide nodes, complex64 elsewhere;
 *   batch       number of parameter vectors B evaluated per call (>= 1);
 *   want_grad   keep intermediates and compile the reverse sweep;
 *   mem_budget_bytes  0 = no limit; otherwise the plan is made to fit it:
 *               when the terms' intermediates, all live at once under
 *               level-by-level execution, would exceed it, the terms run
 *               in groups (level by level within a group, one group after
 *               another, sized to about 80 % of the budget), and with
 *               want_grad, if that is not enough, with checkpointed
 *               segments; TOO_LARGE if the workspace still exceeds it;
 *   stream      hipStream_t to run on (NULL = the library's own stream);
 *   gemm_min_k  nodes with K >= gemm_min_k contracted indices (K = product
 *               of their dimensions) and M, N >= 16 run on the MFMA GEMM,
 *               the rest on the gather kernels; 0 = default (8), a value
 *               above every K keeps all nodes on the gather kernels;
 *   gemm_min_macs  a node also needs at least this many complex
 *               multiply-adds (M N K times its batch rows) to go to the GEMM:
 *               below it the gather kernels finish sooner; 0 = default
 *               (2^20), 1 = no floor;
 *   exec_mode   how tree levels (steps) run.  Level launch: all terms'
 *               nodes at one step as a GEMM kernel and a gather kernel over
 *               the whole chip.  Term launch: one workgroup per term runs
 *               the term's nodes of a run of consecutive steps with
 *               workgroup barriers in between (gather path only; each term
 *               gets its own arena region).  1 = level launches only; 2 =
 *               term launches only (the leaves and all forward steps in
 *               one kernel, the reverse sweep in another); 3 = resident
 *               term launches: one kernel runs each term's leaves, forward
 *               pass and reverse sweep in one workgroup, with tensors the
 *               planner places in the workgroup's LDS arena (sized from
 *               the device's shared memory) read and written there
 *               (batch 1, every node on the gather path, one term group;
 *               TC_ERR_UNSUPPORTED otherwise); 0 = term launches for runs
 *               of at least two light steps (batch 1, no node for the GEMM
 *               path, at most two gather items per thread of each term's
 *               workgroup; the forward runs as resident term launches when
 *               the device has an LDS arena), level launches for the other
 *               steps.
 *   tile_mode   0 = GEMM nodes whose operands are stored dense, A as
 *               [m][k] and B as [k][n] (the planner stores intermediates
 *               that feed GEMM nodes so), with at least 256 tiles of
 *               128 x 128 run such tiles, the others 64 x 64 tiles; 1 =
 *               64 x 64 tiles only; 2 = 128 x 128 tiles for every such
 *               node whatever its tile count (for tests).  The wide tiles
 *               read the operands as planes written once per evaluation
 *               (FP32 re/im, or split-BF16 hi/lo: 8 bytes per element of
 *               workspace); under mem_budget_bytes a plan that fits only
 *               without them is built with 64 x 64 tiles.
 * GEMM nodes whose output tiles cannot fill the chip have K cut into
 * slices (split-K): every slice writes a partial tile to the workspace and
 * a reduction kernel adds the slices in slice order, so results do not
 * depend on the order in which slices finish.  Gather nodes with a sum too
 * long for one wavefront and few outputs (a final inner product) have
 * their sum cut into slices the same way.
 *   checkpoint_every  with want_grad: 0 = keep every intermediate for the
 *               reverse sweep unless mem_budget_bytes is exceeded, in which
 *               case the segment length with the smallest workspace is
 *               chosen; c >= 2 = always checkpoint with segments of c tree
 *               levels (values consumed inside their own segment are freed
 *               after the forward pass and recomputed segment by segment
 *               during the reverse sweep); -1 = never.
 *   qgt         geometric tensor (section "Advanced automatic
 *               differentiation": the quantity <d_i psi|d_j psi> -
 *               <d_i psi|psi><psi|d_j psi> behind the QFI and the quantum
 *               natural gradient).  The plan contracts the <psi|psi>
 *               network once per gate use u of a parameter (batch row u
 *               takes that gate's derivative on the ket side), which gives
 *               <psi|d_u psi>; its reverse sweep toward the bra leaves
 *               gives <d_i psi|d_u psi> for every slot i in the same pass;
 *               a last kernel sums the uses of each slot and subtracts the
 *               product term.
 */
typedef struct tc_plan tc_plan;

typedef enum { TC_PREC_C64 = 0, TC_PREC_BF16X3 = 1 } tc_precision;

typedef struct {
  int32_t precision;
  int32_t batch;
  int32_t want_grad;
  int32_t device;            /* HIP device ordinal                        */
  uint64_t mem_budget_bytes;
  void* stream;              /* hipStream_t                               */
  int32_t gemm_min_k;
  int32_t checkpoint_every;
  uint64_t gemm_min_macs;
  int32_t exec_mode;
  int32_t tile_mode;
  int32_t qgt;               /* 1: the plan computes the geometric tensor
                                (tc_contract_qgt) of the circuit's state;
                                needs a TC_OBS_STATE network and batch 1   */
} tc_plan_opts;

tc_status tc_plan_create(const tc_network* net, const tc_path* path,
                         const tc_plan_opts* opts, tc_plan** out);
void tc_plan_free(tc_plan* plan);

typedef struct {
  double flops;              /* forward contraction flops (8 per c-MAC),
                                times batch where batched               */
  double alg_bytes;          /* forward algorithmic bytes: operands read
                                plus results written, once per node     */
  double grad_flops;         /* reverse-sweep flops (0 without grad)    */
  double grad_alg_bytes;
  uint64_t workspace_bytes;  /* device memory the plan needs             */
  uint64_t peak_tensor_bytes;/* largest single intermediate              */
  int32_t n_nodes;           /* contraction steps over all terms        */
  int32_t n_levels;          /* forward launch levels                   */
  int32_t n_gemm_nodes;      /* nodes sent to the MFMA GEMM path         */
  int32_t n_launches;        /* kernels per forward call                 */
  int32_t n_grad_launches;
  int32_t batch;
  int32_t n_params;
  int32_t n_terms;
  int32_t checkpoint_every;  /* segment length used, 0 = none            */
  int32_t exec_mode;         /* 1 level launches only, 2 term launches
                                only, 3 both, 4 resident term launches   */
  int32_t n_split_nodes;     /* GEMM nodes whose K is cut into slices    */
  int32_t n_split_sums;      /* gather nodes (long sums, few outputs)
                                whose K is cut into slices               */
  int32_t n_wide_nodes;      /* GEMM nodes in 128 x 128 tiles            */
  int32_t n_term_groups;     /* terms run in this many groups, one group's
                                forward pass and reverse sweep after the
                                other's, so that the live intermediates
                                fit mem_budget_bytes (1 = all together)  */
  int32_t n_qgt_rows;        /* qgt plans: gate uses of parameters, one
                                contraction row each (0 otherwise)        */
} tc_plan_info;

tc_status tc_plan_info_get(const tc_plan* plan, tc_plan_info* out);

/* Bind device memory: `workspace` must be a device pointer with at least
 * workspace_bytes bytes, 256-byte aligned, owned by the caller and kept
 * alive until tc_plan_free; NULL asks the library to allocate (hipMalloc)
 * and own it.  Uploads the op tables and captures the launch sequence as a
 * HIP graph.  TOO_LARGE if the budget is exceeded, DEVICE on HIP errors. */
tc_status tc_plan_bind(tc_plan* plan, void* workspace, uint64_t bytes);

/* ----------------------------------------------------------------- contract
 * tc_contract: params is a DEVICE pointer to B*n_params floats (row b =
 * parameter vector b).  out is a HOST pointer to 2*B doubles receiving
 * (re, im) of sum_j alpha_j T_j for each b (the amplitude itself for
 * AMPLITUDE).  Synchronous on the plan's stream.
 *
 * tc_contract_grad: requires want_grad.  value (HOST, B doubles) receives
 * Re E; grad (HOST, B*n_params doubles) receives dE/dparams, slots no gate
 * uses are exactly 0.  Either may be NULL to skip its copy.
 *
 * *_device variants write to DEVICE buffers of the same shapes (out_dev:
 * 2*B doubles; value_dev: B doubles; grad_dev: B*n_params doubles) and do
 * not synchronise; the caller orders later work on the plan's stream.
 * tc_contract_grad_device with both outputs (and n_params > 0) reads params
 * and writes value_dev and grad_dev in place: the plan keeps one extra
 * graph captured for the last (params, value_dev, grad_dev) triple and
 * captures it again when a call passes other pointers (so a loop over the
 * same buffers pays no staging copies); the three buffers must not overlap
 * each other.  While the plan's stream is being captured by the caller, the
 * call takes the staging path instead (copies around the plan's graph).
 */
tc_status tc_contract(tc_plan* plan, const float* params, double* out);
tc_status tc_contract_grad(tc_plan* plan, const float* params, double* value,
                           double* grad);
tc_status tc_contract_device(tc_plan* plan, const float* params,
                             double* out_dev);
tc_status tc_contract_grad_device(tc_plan* plan, const float* params,
                                  double* value_dev, double* grad_dev);

/* tc_contract_qgt: for a plan made with qgt = 1.  params is a DEVICE
 * pointer to n_params floats (one vector); qgt is a HOST pointer to
 * 2 * n_params * n_params doubles receiving G[i][j] = <d_i psi|d_j psi> -
 * <d_i psi|psi><psi|d_j psi> as (re, im), row-major (i the bra slot, j the
 * ket slot); slots no gate uses give zero rows and columns.  The QFI is
 * 4 Re G.  Synchronous.  STATE for plans without qgt (and the other
 * contraction calls return STATE for qgt plans). */
tc_status tc_contract_qgt(tc_plan* plan, const float* params, double* qgt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * tc_contract_grad_device computation run in a static device array of
 * TC_NOALLOC_MAX_BYTES per GPU, reserved when the library is loaded and
 * held until the process ends, instead of the plan's bound workspace.  It
 * calls no hipMalloc/hipFree and never binds the plan (the plan may also be
 * bound; its workspace is not touched).  Each call uploads the plan's tables
 * and params into the array, enqueues the forward and reverse sweeps
 * kernel by kernel (no graph) on the plan's stream (opts.stream; NULL = the
 * null stream), and copies value (B doubles) and grad (B*n_params doubles)
 * to the caller's DEVICE buffers; either may be NULL.  Does not
 * synchronise.  The array is shared by every plan on that GPU and keeps
 * the last call's contents: calls that overlap on one GPU (two streams,
 * two threads) race and give wrong results.
 * Errors: STATE without want_grad; TOO_LARGE when the plan's
 * workspace_bytes exceed TC_NOALLOC_MAX_BYTES; BUSY as for the other
 * contraction calls; DEVICE on HIP errors. */
#define TC_NOALLOC_MAX_BYTES (64ull << 20)
tc_status tc_contract_grad_device_noalloc(tc_plan* plan, const float* params,
                                          double* value_dev, double* grad_dev);

/* Profiling.  Runs the plan's kernels eagerly (not as a graph), one after
 * another on the plan's stream, `reps` times; every kernel's start and end
 * are stamped by its own dispatch (hipExtLaunchKernel events), so a
 * duration holds no queueing gap.  params is a DEVICE pointer as for
 * tc_contract.  For kernel i <
 * *n_launches (at most `cap` are written) it reports the kernel class
 * kinds[i] (0 leaf materialisation, 2 MFMA GEMM tiles of one tree level,
 * 3 gather contractions of one tree level, 4 FP64 root sum, 5 FP64
 * gradient sum, 6 term mode: all terms' trees, forward pass with the leaves
 * or reverse sweep, 7 MFMA GEMM nodes of one tree level in 128 x 128
 * tiles with their split pass, 8 row tiles of one tree level (batched small
 * nodes), 9 split sums of one tree level with their reduction), the mean
 * duration ms[i], and the kernel's algorithmic
 * flops[i] and bytes[i] (operands read once plus results written once).
 * which: 0 the forward sequence, 1 forward plus reverse sweep (needs
 * want_grad).  A level's GEMM and gather parts run one after the other
 * here (in the graph they overlap); a part of several kernels (split-K and
 * its reduction) is timed from its first kernel's start to its last's end. */
tc_status tc_plan_profile(tc_plan* plan, const float* params, int32_t which,
                          int32_t reps, int32_t cap, int32_t* n_launches,
                          int32_t* kinds, double* ms, double* flops,
                          double* bytes);

/* ------------------------------------------------------------------ serving
 * Continuous-batching request loop (not a method of the paper: a serving
 * form of the same executor).  Requests are admitted while the sum of their
 * workspace sizes stays within pool_bytes and fewer than max_active are
 * live; admitted requests advance one contraction level per engine step and
 * the steps of all live requests are launched together, so requests that
 * arrive while others run join the next step.  Plans are cached by circuit
 * structure and observable; each request gets its own region of the pool.
 *
 *   tc_serve_submit  copies the request; params are HOST floats
 *                    (n_params); returns an id.  A request whose plan does
 *                    not fit max_request_bytes even with its terms in
 *                    groups is sliced (tc_slice, every intermediate within
 *                    an eighth of the cap) and its slices run as terms.
 *                    TOO_LARGE if it still does not fit, or needs more
 *                    than max_request_flops (it is not queued).
 *   tc_serve_step    admits what fits, launches one step for every live
 *                    request, and collects finished ones; *n_live receives
 *                    the number still queued or running.
 *   tc_serve_result  TC_OK with value (Re E), value_im and, if requested,
 *                    grad (HOST, n_params doubles) once finished;
 *                    TC_ERR_BUSY while pending.  A fetched result is
 *                    released.
 */
typedef struct tc_server tc_server;

typedef struct {
  int32_t device;
  uint64_t pool_bytes;        /* device memory shared by live requests    */
  uint64_t max_request_bytes; /* per-request workspace cap                */
  int32_t max_active;         /* live request slots                       */
  int32_t path_trials;        /* greedy trials per new structure          */
  void* stream;               /* hipStream_t, NULL = own stream           */
  double max_request_flops;   /* 0 = no limit; else requests whose plan
                                 needs more flops are rejected (TOO_LARGE) */
} tc_serve_opts;

typedef struct {
  int64_t id;
  double value;
  double value_im;
  double submit_to_done_s;    /* library-measured latency                 */
  int32_t want_grad;
  int32_t status;             /* tc_status of the request                 */
  double plan_s;              /* of which host planning (network, path,
                                 plan; ~0 on a plan-cache hit)            */
  double admit_to_done_s;     /* of which from admission (pool memory and
                                 a slot granted) to the result            */
} tc_serve_result;

tc_status tc_serve_create(const tc_serve_opts* opts, tc_server** out);
tc_status tc_serve_submit(tc_server* srv, const tc_circuit* circuit,
                          const tc_observable* observable,
                          const float* params, int32_t want_grad,
                          int64_t* id);
tc_status tc_serve_step(tc_server* srv, int32_t* n_live);
tc_status tc_serve_result_get(tc_server* srv, int64_t id,
                              tc_serve_result* out, double* grad);
void tc_serve_free(tc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* TCX_H */
