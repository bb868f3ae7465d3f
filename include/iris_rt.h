/*
 * iris_rt.h -- C ABI of the MI355X 13CO(2-1) position-position-velocity (PPV)
 * radiative-transfer library.
 *
 * The library synthesises spectral-line cubes from a gridded snapshot by
 * solving the radiative-transfer equation along every sightline (paper: "The
 * Radiative Transfer Equation", eqs. Total/Continuum Radiative Transfer;
 * "Transfer Solution: Formal and Smooth Integration of Optically Thick and
 * Selectively Thin Transfer", the formal step, or the smooth TR/BDF2
 * integrator selected by iris_line.integrator). Level populations are
 * LTE (Boltzmann, as in "Synthetic Observation Versus Density-Tracing"), the
 * line profile is a thermal plus microturbulent Gaussian ("Line Emission and
 * Absorption", eq. Thermal Broadening Profile), dust is a kappa*rho absorber
 * with a blackbody source ("Dust Emission and Absorption") and the CMB enters
 * as the background intensity at the far side of each sightline ("Transfer
 * Solution: Overview"). Outputs are Rayleigh-Jeans brightness temperatures
 * ("Intensity Versus Temperature"), split into five components:
 *
 *   [T] total            march of line + dust from the background,
 *   [C] continuum        march of dust only from the background,
 *   [L] line             [T] - [C], continuum subtraction in intensity
 *                        (equivalently T_RJ) space ("Continuum Subtraction"),
 *   [B] background       background intensity attenuated by the dust column,
 *   [D] dust             dust emission marched from zero intensity,
 *                        so that [C] = [D] + [B].
 *
 * The continuum ([C], [D], [B]) is evaluated at the line rest frequency, so it
 * is the same in every channel; it is nevertheless written for every channel.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers on the current HIP device; the
 *    caller owns them. The library never allocates on the forward/adjoint
 *    path: scratch comes from a caller-provided workspace. Batched plans own
 *    their scratch, allocated at creation and freed at destruction.
 *  - `stream` is a hipStream_t (NULL = the default stream). Calls are
 *    asynchronous on that stream.
 *  - Arguments are validated on the host before anything is launched. A bad
 *    argument returns IRIS_E_INVALID_ARG and launches nothing; the reason is
 *    available from iris_last_error() (thread-local, valid until the next
 *    call on that thread). HIP failures return IRIS_E_HIP.
 *  - Grids are C-ordered [nx][ny][nz] (z fastest). A sightline runs along
 *    `axis`; its position 0 is the far side (where the background enters)
 *    and the observer lies beyond the last cell. Pixels enumerate the two
 *    remaining axes in C order: axis 0 -> pixel = y*nz + z, axis 1 ->
 *    pixel = x*nz + z, axis 2 -> pixel = x*ny + y.
 *  - Channel k (0-based) is centred at v_lo + (k + 1/2) dv km/s (radio
 *    velocity). A cell with line-of-sight velocity v (positive = receding)
 *    has its profile centred at v; the profile is evaluated at channel
 *    centres.
 *  - Cube outputs and cotangents are FP32 [n_pix][n_chan], channel fastest.
 */
#ifndef IRIS_RT_H
#define IRIS_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IRIS_OK = 0,
  IRIS_E_INVALID_ARG = 1, /* null pointer, bad size or parameter; nothing launched */
  IRIS_E_UNSUPPORTED = 2, /* valid request outside what is built (e.g. too many channels) */
  IRIS_E_WORKSPACE = 3,   /* workspace null or smaller than iris_rt_workspace_bytes() */
  IRIS_E_HIP = 4,         /* a HIP runtime call failed */
  IRIS_E_NONFINITE = 5    /* iris_rt_check_fields found values the march cannot use */
} iris_status;

typedef enum { IRIS_F64 = 0, IRIS_F32 = 1, IRIS_BF16 = 2, IRIS_F16 = 3 } iris_dtype;

/* Units of the output cubes ("Intensity Versus Temperature"). Every unit is
 * evaluated at the rest frequency nu0, where [C], [D] and [B] are taken.
 *  - IRIS_UNITS_TRJ: Rayleigh-Jeans brightness temperature, K (default).
 *  - IRIS_UNITS_INTENSITY: specific intensity, erg s^-1 cm^-2 Hz^-1 sr^-1
 *    (T_RJ * 2 k nu0^2 / c^2 for every component).
 *  - IRIS_UNITS_TB: Planck brightness temperature T0 / ln(1 + T0 / T_RJ),
 *    T0 = h nu0 / k, for [T], [C] and [B] (0 where T_RJ is 0); [L] and [D],
 *    which are not intensities of a blackbody, stay in T_RJ. The adjoint does
 *    not support these units. */
typedef enum { IRIS_UNITS_TRJ = 0, IRIS_UNITS_INTENSITY = 1, IRIS_UNITS_TB = 2 } iris_units;

/* Integrator of the transfer equation ("Transfer Solution: Formal and Smooth
 * Integration of Optically Thick and Selectively Thin Transfer").
 *  - IRIS_INTEGRATOR_FORMAL: the exponential (formal) step of each cell with
 *    its coefficients held constant across it (default).
 *  - IRIS_INTEGRATOR_SMOOTH: the implicit trapezoidal rule for the first
 *    step and the two-step backward differentiation formula (BDF2) after it,
 *    each solved in closed form and clamped at zero intensity. The nodes are
 *    the cells, each with its own coefficients, and the background is the
 *    intensity at node 0 (the far cell): a sightline of n cells takes n - 1
 *    steps, and a single cell returns the background. [C], [D] and [B] are
 *    integrated the same way, from the background, from zero and (with no
 *    emission) from the background. Forward only: checkpoints, the adjoint,
 *    adjoint plans and autotuning are not built for it (IRIS_E_UNSUPPORTED;
 *    forward plans are), and the marched velocities must not exceed
 *    iris_smooth_max_channels(). */
typedef enum { IRIS_INTEGRATOR_FORMAL = 0, IRIS_INTEGRATOR_SMOOTH = 1 } iris_integrator;

/* Transfer mode ("Transfer Solution: Optically Thick Transfer" / "... Optically
 * Thin Transfer").
 *  - IRIS_TRANSFER_THICK: the full transfer equation with line and dust
 *    absorption (default).
 *  - IRIS_TRANSFER_THIN: absorption and stimulated emission are ignored;
 *    every component is the background plus the path integral of its
 *    emission, and the line profile is replaced by its mean over each
 *    channel, (1/dv) (1/2) [erf(x_hi) - erf(x_lo)], x = (v_edge - v)/b. The
 *    formal integrator sums every cell; the smooth one takes Simpson panels
 *    of two cells over the nodes 0 .. 2P, P = floor((n_los - 1)/2) (the last
 *    cell of an even count is left out). [B] is the unattenuated background.
 *  - IRIS_TRANSFER_SELECTIVE ("Transfer Solution: Selectively Thin
 *    Transfer"): the line absorbs the continuum but not itself. Each cell's
 *    continuum step is solved first; the total then takes the formal step
 *    with the dust absorption only and the emission
 *    jbar_L + j_D - alphabar_L I_C, I_C the continuum after that cell, with
 *    the channel-averaged profile, and is clamped at zero after every step
 *    (a line colder than the continuum it absorbs could otherwise drive it
 *    negative; the paper applies its ReLU to each selective step). Under the
 *    smooth integrator the same
 *    substitution enters the TR and BDF2 steps: I_C is the continuum of the
 *    same node (solved first), the absorption is the dust's, and every step
 *    of the total is clamped at zero; up to iris_smooth_max_channels()
 *    channels.
 *    For both thin modes velocity subsampling does not apply (simpson_f must
 *    be 0: IRIS_E_INVALID_ARG); checkpoints, adjoint plans and autotuning are
 *    not built for them (IRIS_E_UNSUPPORTED; forward plans are). Optically
 *    thin transfer has an adjoint (both integrators): nothing is marched, so
 *    iris_rt_adjoint takes ckpt_K = 0 and any workspace of
 *    iris_rt_workspace_bytes(fields, channels, 0) bytes (it rebuilds its
 *    tables); the selectively thin mode has none (IRIS_E_UNSUPPORTED). */
typedef enum {
  IRIS_TRANSFER_THICK = 0,
  IRIS_TRANSFER_THIN = 1,
  IRIS_TRANSFER_SELECTIVE = 2
} iris_transfer;

/* Per-cell fields of one cube, all in the same storage type, device memory,
 * [nx][ny][nz] each. Arithmetic is FP32 whatever the storage type. */
typedef struct {
  int32_t nx, ny, nz; /* grid shape, each >= 1 */
  int32_t axis;       /* sightline axis, 0..2 */
  double cell_cm;     /* cell length along the sightline, cm, > 0 */
  iris_dtype dtype;   /* storage type of every field below */
  const void* ln_nh2; /* natural log of the H2 number density, ln(cm^-3) */
  const void* t_kin;  /* gas kinetic temperature, K, > 0 */
  const void* v_los;  /* line-of-sight velocity, km/s, positive = receding */
  const void* x_tracer; /* tracer abundance n(13CO)/n(H2) */
  const void* t_dust; /* dust temperature, K; NULL means T_dust = T_kin */
} iris_fields;

/* Uniform channel grid: n_chan channels of width dv_kms starting at v_lo_kms.
 * simpson_f sets the velocity subsampling ("Transfer Solution: Optically
 * Thick Transfer"): 0 evaluates the profile at channel centres; f >= 1
 * marches a fine grid of 2 f n_chan + 1 velocities v_lo + j dv / (2f) (the
 * channel edges and 2f - 1 points inside each channel) and reports each
 * channel's composite-Simpson average over its 2f steps. Outputs and
 * cotangents keep n_chan channels; 2 f n_chan + 1 must not exceed
 * iris_max_channels(). */
typedef struct {
  int32_t n_chan;    /* 1 .. iris_max_channels() */
  int32_t simpson_f; /* 0 .. 64 */
  double v_lo_kms;
  double dv_kms; /* > 0 */
} iris_channels;

/* Grid of non-LTE level populations (iris_levels_create, below). */
typedef struct iris_levels iris_levels;

/* Line, dust and background constants ("Line Emission and Absorption",
 * "Einstein Coefficients ...", "Dust Emission and Absorption", Table of
 * synthetic-observation parameters). */
typedef struct {
  double nu0_hz;         /* rest frequency of the transition, Hz */
  double a_ul;           /* Einstein A of the transition, s^-1 */
  double e_u_k;          /* upper-level energy / k, K (energy_mode 1 only) */
  int32_t j_u;           /* upper rotational level; lower level is j_u - 1 */
  int32_t j_max;         /* partition function summed over J = 0..j_max */
  double m_tracer_amu;   /* tracer molecular mass, amu */
  double sigma_turb_kms; /* 1-D microturbulent dispersion: b^2 = 2kT/m + 2 sigma^2 */
  double kappa_dust_cm2g; /* dust opacity per gram of dust, cm^2/g */
  double dust_to_gas;    /* dust-to-gas mass ratio */
  double mu_amu_per_h2;  /* gas mass per H2 molecule, amu */
  double t_bg_k;         /* background blackbody temperature (CMB), K, >= 0 */
  double t_inf_k;        /* no line emission or absorption above this T_kin, K */
  int32_t energy_mode;   /* 0: level energies of a rigid rotor with
                            E_u - E_l = h nu0 / k exactly; 1: rigid rotor
                            through the literal e_u_k */
  int32_t units;         /* iris_units of the output cubes (0 = T_RJ) */
  int32_t integrator;    /* iris_integrator (0 = formal) */
  int32_t transfer;      /* iris_transfer (0 = optically thick) */
  /* Level populations of the observed transition: NULL for LTE (Boltzmann at
   * T_kin); else the optically thin level balance, interpolated per cell in
   * a grid built by iris_levels_create for this transition (its frequency,
   * Einstein A and level weights must be nu0_hz, a_ul, 2 j_u + 1 and
   * 2 j_u - 1, to 1e-6). The adjoint differentiates through the grid's
   * interpolation (its slopes on the interval a cell falls in). The grid
   * must outlive every call that uses it. */
  const iris_levels* levels;
  /* Molecular fraction chi = 2 n_H2 / n_H of every cell, (0, 1] (0 means 1:
   * all hydrogen in H2), for the collision partners of the level balance. */
  double h2_frac;
} iris_line;

/* Five output cubes, FP32 [n_pix][n_chan] in line->units (Rayleigh-Jeans K
 * by default), device; any pointer may be NULL to skip that component.
 * Cotangents of the adjoint are with respect to the same units. */
typedef struct {
  float* T;
  float* C;
  float* D;
  float* L;
  float* B;
} iris_outputs;

/* Cotangents dLoss/d[X] for each output cube, FP32 [n_pix][n_chan], device;
 * NULL means zero. */
typedef struct {
  const float* gT;
  const float* gC;
  const float* gD;
  const float* gL;
  const float* gB;
} iris_cotangents;

/* Gradients of the loss with respect to the stored field values, FP64
 * [nx][ny][nz], device, overwritten: d/d(ln n_H2), d/dT_kin, d/dv_los
 * (per km/s), d/dX. g_t_dust is used only when fields->t_dust is non-NULL.
 * The gradient with respect to n_H2 itself is g_ln_nh2 / n_H2. */
typedef struct {
  double* g_ln_nh2;
  double* g_t_kin;
  double* g_v_los;
  double* g_x_tracer;
  double* g_t_dust;
} iris_gradients;

/* Library identification and limits. */
const char* iris_version(void);
int32_t iris_max_channels(void);
/* Largest marched velocity count (2 f n_chan + 1 when subsampled, else
 * n_chan) of the smooth integrator, which keeps two intensities per marched
 * velocity in registers. */
int32_t iris_smooth_max_channels(void);
const char* iris_status_string(iris_status s);
const char* iris_last_error(void);

/* Field ingest ("Physical Tensors": per-cell channels on a lattice marched
 * along one axis). Copies the four fields (five with t_dust) into sightline-
 * major order, [field][n_pix][n_los] in the storage type, so that each
 * sightline is contiguous. dst must hold iris_rt_layout_bytes(fields) bytes.
 * Bit-exact copy; no arithmetic. */
size_t iris_rt_layout_bytes(const iris_fields* fields);
iris_status iris_rt_layout(const iris_fields* fields, void* dst, size_t dst_bytes, void* stream);

/* Optional scan of the fields before a synthesis: counts values the march
 * cannot use (non-finite values in any field, T_kin or T_dust not above zero,
 * negative abundance) into *bad and returns IRIS_E_NONFINITE if there are any.
 * The physical tensors of the paper ("Physical Tensors") carry finite,
 * positive temperatures and non-negative abundances; the march itself does
 * not test every value. Uses 8 bytes of device scratch (caller-owned) and
 * synchronises the stream. */
iris_status iris_rt_check_fields(const iris_fields* fields, void* scratch, size_t scratch_bytes,
                                 void* stream, int64_t* bad);

/* Workspace needed by iris_rt_forward/iris_rt_adjoint for these fields and
 * checkpoint interval (ckpt_K = 0: forward only, no adjoint checkpoints):
 * the temperature tables of the per-cell setup ("Observability
 * Determination"), the erfc pieces of the thin modes, a sightline-major copy
 * of the fields when IRIS_RT_FIELD_LAYOUT=transpose asks for one, and for
 * ckpt_K > 0 the checkpoints of the intensity state every ckpt_K cells that
 * the adjoint recomputes from (the paper's memory bound on these tensors,
 * "Observability Determination", is what the checkpoints trade against
 * recomputation). The adjoint needs the workspace of the forward that wrote
 * the checkpoints: a workspace-free adjoint that recomputes everything would
 * have to allocate its own checkpoints, which the single-cube calls never do.
 * Returns 0 for invalid arguments. */
size_t iris_rt_workspace_bytes(const iris_fields* fields, const iris_channels* channels,
                               int32_t ckpt_K);

/* Forward synthesis. Writes the requested output cubes. When ckpt_K > 0 the
 * intensity state is also saved every ckpt_K cells into the workspace so
 * that iris_rt_adjoint can run afterwards on the same workspace. ckpt_K must
 * be 0 or one of 8, 16, 32, 64. */
iris_status iris_rt_forward(const iris_fields* fields, const iris_channels* channels,
                            const iris_line* line, const iris_outputs* out, int32_t ckpt_K,
                            void* workspace, size_t workspace_bytes, void* stream);

/* Forward synthesis that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts that
 * forbid hipMalloc). Same outputs as iris_rt_forward with ckpt_K = 0, from the
 * same kernels; the scratch that iris_rt_forward takes from its workspace (the
 * temperature tables and the erfc pieces of the thin modes) lives instead in a
 * static device array of iris_rt_forward_static_max_bytes() bytes that each GPU
 * holds until the process ends. No checkpoints (hence no adjoint after it). A
 * call that would need more scratch than the array holds (a sightline-major
 * copy of the fields, which IRIS_RT_FIELD_LAYOUT=transpose asks for, of all
 * but the smallest cubes) returns IRIS_E_WORKSPACE and launches nothing.
 * Every call on one GPU
 * uses that GPU's one array: two calls that may run at the same time on one GPU
 * (different streams, or different host threads) race on it and must be
 * ordered by the caller. The array keeps the last call's contents; every call
 * rewrites what it reads before reading it. */
size_t iris_rt_forward_static_max_bytes(void);
iris_status iris_rt_forward_static(const iris_fields* fields, const iris_channels* channels,
                                   const iris_line* line, const iris_outputs* out, void* stream);

/* Reverse-mode gradient ("differentiability modes" in "Synthetic Observation
 * Implementation and Algorithms") of Loss = sum over cubes of cot.gX * [X],
 * with respect to every stored field value (g_t_dust too when fields->t_dust
 * is given: the line and dust source functions apart, as in energy_mode 1).
 * Requires a preceding iris_rt_forward with the same fields, channels, line
 * and ckpt_K (> 0) on the same workspace, stream-ordered before this call;
 * the workspace must not be modified in between. Thick transfer, formal
 * steps, LTE populations, T_RJ or intensity units; other lines return
 * IRIS_E_UNSUPPORTED. */
iris_status iris_rt_adjoint(const iris_fields* fields, const iris_channels* channels,
                            const iris_line* line, const iris_cotangents* cot, int32_t ckpt_K,
                            void* workspace, size_t workspace_bytes,
                            const iris_gradients* grads, void* stream);

/* ---- Autotuning -----------------------------------------------------------
 * The forward march packs G = 1, 2 or 4 sightlines into one wavefront (64/G
 * lanes each). iris_rt_autotune times the three on the given cube (writing
 * its outputs), records the fastest for cubes of the same shape class
 * (channel count and width, storage type, sightline length, line source
 * variant) and returns it in *groups. Later iris_rt_forward calls and plans
 * of that class use the recorded choice; without one, a rule based on the
 * Doppler width in channels is used. When the environment variable
 * IRIS_RT_TUNE_CACHE names a file, choices are loaded from and appended to it.
 * Arguments as for iris_rt_forward (ckpt_K = 0). Synchronises the stream. */
iris_status iris_rt_autotune(const iris_fields* fields, const iris_channels* channels,
                             const iris_line* line, const iris_outputs* out, void* workspace,
                             size_t workspace_bytes, void* stream, int32_t* groups);

/* The adjoint's reverse march ("differentiability modes" in "Synthetic
 * Observation Implementation and Algorithms") packs G = 1, 2 or 4 sightlines
 * per wavefront too; each packing holds its own tape of K cells in LDS, so the
 * packings that fit depend on n_chan and ckpt_K. iris_rt_autotune_adjoint
 * times those that fit on the given cube (each timing runs the full adjoint
 * and overwrites the gradients), records the fastest for the class (the
 * forward's class plus ckpt_K; same cache file) and returns it in *groups;
 * the gradients on return are those of the chosen packing. Later
 * iris_rt_adjoint calls of the class use it (plans do not: their launches
 * share the GPU between cubes, and follow their own rule). Without a recorded
 * choice the adjoint takes the widest packing whose Doppler window at 100 K
 * spans at most 64/G channels, narrowed until its tape fits; the environment
 * variable IRIS_RT_ADJOINT_SIGHTLINES_PER_WAVE
 * (1, 2 or 4) overrides every rule. Arguments and preconditions as for
 * iris_rt_adjoint (a forward with the same ckpt_K on the same workspace
 * first). Synchronises the stream. */
iris_status iris_rt_autotune_adjoint(const iris_fields* fields, const iris_channels* channels,
                                     const iris_line* line, const iris_cotangents* cot,
                                     int32_t ckpt_K, void* workspace, size_t workspace_bytes,
                                     const iris_gradients* grads, void* stream, int32_t* groups);

/* ---- Batched plans ---------------------------------------------------------
 * The paper iterates observability determination and transfer over batches
 * of rays so that the observability tensors fit in GPU memory
 * ("Observability Determination"), and notes that iterating over sky-plane
 * chunks deflates its measured speed ("Speed Testing"). A plan does the
 * opposite: it binds many cubes (each with its own grid, sightline axis, storage
 * type and channel grid; one line) to one persistent launch per phase: a
 * work queue of (cube, sightlines) items, longest sightlines first, drained
 * by as many workgroups as the device keeps resident. Each phase is captured
 * once in a hipGraph (queue reset, batched field layout, persistent march;
 * for the adjoint also the batched gradient layout) and replayed by
 * iris_plan_forward / iris_plan_adjoint. The plan keeps the pointers it was
 * created with: to process new data, write it into the same buffers.
 * The plan owns its scratch (allocated at creation, freed by
 * iris_plan_destroy). Calls are asynchronous on `stream`; two phases of one
 * plan must not overlap.
 * Adjoint plans with cubes that carry a t_dust field (separate line and dust
 * source functions) run those cubes in launches of their own and need
 * grads.g_t_dust. The smooth integrator and the thin transfer modes have no
 * persistent kernel: their plans capture the single-cube forward of every cube, in
 * order, into the forward graph (outputs identical to iris_rt_forward).
 * They are forward only: IRIS_PLAN_ADJOINT and IRIS_PLAN_AUTOTUNE return
 * IRIS_E_UNSUPPORTED; iris_plan_info reports one forward item per cube and
 * no persistent grid. */
typedef struct {
  iris_fields fields;
  iris_channels channels;
  iris_outputs out;       /* forward outputs */
  iris_cotangents cot;    /* adjoint inputs (IRIS_PLAN_ADJOINT) */
  iris_gradients grads;   /* adjoint outputs (IRIS_PLAN_ADJOINT) */
} iris_cube;

typedef struct iris_plan iris_plan;

enum {
  IRIS_PLAN_FORWARD = 1,  /* always implied */
  IRIS_PLAN_ADJOINT = 2,  /* forward writes checkpoints every ckpt_K cells; adjoint phase built */
  IRIS_PLAN_AUTOTUNE = 4  /* time the forward's sightline packing per cube class at
                             creation (writes the cubes' outputs). With IRIS_PLAN_ADJOINT
                             and ckpt_K = 0, the checkpoint interval is chosen too: forward
                             + adjoint timed at K = 8, 16, 32, 64 on the cube with the most
                             cells (writes its gradients; iris_plan_info.ckpt_K). The
                             adjoint's packing in plans follows the plan rule, which beat
                             choices timed cube by cube */
};

typedef struct {
  int64_t scratch_bytes;   /* device memory owned by the plan */
  int64_t samples;         /* sum over cubes of cells x channels */
  int32_t n_cubes;
  int32_t n_fwd_items, n_adj_items;
  int32_t fwd_blocks, adj_blocks; /* persistent grid sizes */
  int32_t layout_tiles;    /* tiles of the batched field layout (0: none needed) */
  int32_t ckpt_K;          /* checkpoint interval of the adjoint (0: forward-only plan) */
} iris_plan_info;

iris_status iris_plan_create(const iris_cube* cubes, int32_t n_cubes, const iris_line* line,
                             int32_t flags, int32_t ckpt_K, void* stream, iris_plan** plan);
iris_status iris_plan_forward(iris_plan* plan, void* stream);
iris_status iris_plan_adjoint(iris_plan* plan, void* stream);
iris_status iris_plan_get_info(const iris_plan* plan, iris_plan_info* info);
/* Sightlines per wavefront chosen for cube i (1, 2 or 4) by a persistent
 * plan; 0 for a plan of one launch per cube (smooth integrator, thin modes),
 * whose captured single-cube forwards choose their own, and 0 if out of range. */
int32_t iris_plan_groups(const iris_plan* plan, int32_t cube);
/* Sightlines per wavefront of the adjoint's reverse march for cube i (1, 2 or
 * 4); 0 for a plan without IRIS_PLAN_ADJOINT, and 0 if out of range. */
int32_t iris_plan_adjoint_groups(const iris_plan* plan, int32_t cube);
void iris_plan_destroy(iris_plan* plan);

/* ---- Non-LTE level populations ------------------------------------------------
 * The optically thin (OT) level balance ("Level Populations: The Optically
 * Thin Assumption", "... Mathematical Solution", eq. OT Levels System): the
 * statistical equilibrium of every level under collisions, spontaneous
 * emission, and absorption and stimulated emission of a blackbody background
 * at t_bar_k (no self-absorption of the line), with the ground-state equation
 * replaced by the conservation sum n_i = N. Collision rates
 * C_ij = sum_s K_ij^[s] N_s over the partners H2 (ortho and para when the
 * file lists them separately, else combined), atomic H and He; the excitation
 * rates follow from the tabulated de-excitation rates by detailed balance
 * ("Einstein Coefficients, Collisions, and the Detailed Balance"); tabulated
 * rates are interpolated linearly in T and held at the table's end values
 * beyond it. Partner densities: n_H = 2 n_H2 / chi, atomic H (1 - chi) n_H,
 * He he_per_h n_H, and n_H2 split ortho_para : 1.
 *
 * Molecular data come from a text file in the LAMDA .dat convention
 * ("Spectral-Line Configuration"): levels (energy in cm^-1, weight), radiative
 * transitions (upper, lower, A in s^-1, frequency in GHz), collision partners
 * (LAMDA partner code, temperatures, de-excitation rates in cm^3 s^-1 per
 * transition). At most 63 levels, 8 partners, 64 temperatures per partner;
 * electrons and H+ are read and not used. */
typedef struct iris_molecule iris_molecule;
typedef struct {
  int32_t n_levels, n_transitions, n_partners;
  int32_t partner_code[8];          /* LAMDA partner codes, file order */
  int32_t partner_transitions[8];   /* collisional transitions per partner */
  int32_t partner_temperatures[8];  /* tabulated temperatures per partner */
} iris_molecule_info;

/* Reads and checks a molecular data file (host only; no GPU work).
 * IRIS_E_INVALID_ARG with the line at fault on a malformed file. The caller
 * frees it with iris_molecule_destroy. */
iris_status iris_molecule_read(const char* path, iris_molecule** mol);
iris_status iris_molecule_get_info(const iris_molecule* mol, iris_molecule_info* info);
void iris_molecule_destroy(iris_molecule* mol);

typedef struct {
  int32_t transition;     /* 1-based radiative transition of the observed line */
  double t_bar_k;         /* background temperature of the balance, K, >= 0 (0: none) */
  double ortho_para;      /* ortho:para H2 ratio, > 0 */
  double he_per_h;        /* He per H nucleus, >= 0 */
  int32_t n_n, n_chi, n_t; /* nodes per axis, 1..4096 each, product <= 2^24 */
  double ln_nh2_lo, ln_nh2_hi; /* density axis, uniform in ln n_H2 (cm^-3) */
  double chi_lo, chi_hi;       /* molecular-fraction axis, uniform, within (0, 1] */
  double t_lo_k, t_hi_k;       /* temperature axis, uniform in ln T, K, > 0 */
} iris_levels_config;

/* Grid precomputation ("Grid Precomputation"): solves the OT level balance of
 * `mol` at every node of the (ln n_H2, chi, ln T) grid on the GPU (one
 * wavefront per node, FP64 Gaussian elimination with partial pivoting) and
 * keeps, per node, the population factors of the observed transition per
 * unit tracer density, FU = (g_l/g_u) f_u and FL = f_l - FU, as FP32 pairs
 * [n_chi][n_t][n_n] in device memory owned by the grid. Per-abundance line
 * coefficients follow as j/N = (h nu / 4 pi) A (g_u/g_l) FU and
 * alpha/N = (h nu / 4 pi) B_lu FL; the line source function is
 * (h nu / k) FU / FL in Rayleigh-Jeans kelvin. The march interpolates FU and
 * FL multilinearly in (ln n_H2, chi, ln T), extended linearly beyond the
 * grid ("Observability Determination"); where the interpolated FL is not
 * positive the cell carries no line. Allocates device memory (set-up, not
 * the hot path); the solve is queued on `stream` and the grid is ready for
 * work ordered after it on that stream. */
iris_status iris_levels_create(const iris_molecule* mol, const iris_levels_config* cfg,
                               void* stream, iris_levels** levels);
/* Copies the grid to host memory, (FU, FL) pairs [n_chi][n_t][n_n]; n_floats
 * must be 2 n_chi n_t n_n. Synchronises the device. */
iris_status iris_levels_copy_grid(const iris_levels* levels, float* host, size_t n_floats);
void iris_levels_destroy(iris_levels* levels);

/* ---- Post-transfer products -------------------------------------------------
 * Operate on one FP32 cube [n1][n2][n_chan] (device, channel fastest) whose two
 * sky axes are n1 and n2: an output cube of iris_rt_forward is such a cube
 * with (n1, n2) the two axes other than the sightline axis, in C order.
 *
 * Gaussian beam convolution ("Beam Convolution"): every channel map is
 * convolved with a Gaussian of full width at half maximum fwhm_pix pixels
 * (sigma = FWHM / (2 sqrt(2 ln 2))), sampled at pixel offsets, truncated at
 * |offset| <= ceil(4 sigma) <= 128 along each axis and normalised to unit
 * sum; the sky beyond the map is empty (zero padding). An angular beam (the
 * paper's 30 arcsec) is given in pixels by the caller, who knows the pixel's
 * angular size. `out` may be `cube`; the workspace (iris_beam_workspace_bytes)
 * must not overlap either. Two passes along n2 then n1, asynchronous on
 * `stream`. */
size_t iris_beam_workspace_bytes(int32_t n1, int32_t n2, int32_t n_chan);
iris_status iris_beam_convolve(const float* cube, float* out, int32_t n1, int32_t n2,
                               int32_t n_chan, double fwhm_pix, void* workspace,
                               size_t workspace_bytes, void* stream);

/* l,v projection: the mean over sky axis `axis` (0: over n1, out [n2][n_chan];
 * 1: over n2, out [n1][n_chan]), summed in FP64. `out` must not overlap `cube`. */
iris_status iris_lv_mean(const float* cube, float* out, int32_t n1, int32_t n2, int32_t n_chan,
                         int32_t axis, void* stream);

/* ---- Diagnostics -------------------------------------------------------------
 * Measured issue rates of the device's FP32 units, for roofline figures:
 * base-2 exponentials (v_exp_f32) and FMAs per second, each from eight
 * independent chains per lane over a grid filling the current device (best
 * of three timed runs after one warm-up). Not on the synthesis path:
 * allocates and frees a small buffer, creates and destroys its own stream,
 * and synchronises. */
iris_status iris_probe_issue_rates(double* exp_per_s, double* fma_per_s);

#ifdef __cplusplus
}
#endif

#endif /* IRIS_RT_H */
