/*
 * corr.h -- C ABI of libcorr, an FX correlator for AMD Instinct MI355X (gfx950).
 *
 * The library implements the real-time correlator data path of Roy et al.,
 * "A real-time software backend for the GMRT" (arXiv:0910.1517):
 *
 *   F-engine   integer-sample delay by read-pointer offset (section 2.1 and
 *              the overlap scheme of section 2.3.2), real-to-complex FFT
 *              channelisation (section 2.1, FX design; section 3.1), post-FFT
 *              fractional-sample-time correction and fringe stopping with the
 *              phase of Eq. 2 (section 2.1), requantisation (the fixed-point
 *              pipeline of section 4.1) and the corner turn into the X layout.
 *   X-engine   all signal-pair products per channel, self and cross
 *              polarisation (RR*, RL*, LR*, LL* of section 2.1), accumulated
 *              over time (the MAC of sections 2.3.2 and 3.4).
 *   integrate  long-term accumulation in floating point (section 4.1) and
 *              dump of the visibilities.
 *   RFI        the MAD statistic of section 5 (Eq. 3 and 4) on power tiles
 *              with zeroing and exact pair counts, a learned flagger, and
 *              the time-domain voltage blanker with noise replacement.
 *   B-engine   incoherent and coherent array beams (section 2.2).
 *
 * Conventions used everywhere below
 *   S   number of signals (antenna a, polarisation pol -> s = 2a + pol)
 *   N   FFT length (power of two), C = N/2 channels (DC kept, Nyquist bin
 *       dropped), channel k centred at nu_BB + k fs / N
 *   T   spectra per call (T_call of the plan)
 *   P   S(S+1)/2 signal pairs; pair (i <= j) has index p = j(j+1)/2 + i and
 *       holds V_ij = sum_m Y_i[m] * conj(Y_j[m])
 *
 * Every function is extern "C", never throws, and returns a corr_status
 * (0 = success, < 0 = error; see corr_status_string).  All device pointers are
 * caller-owned device memory (for example torch tensors); the library never
 * allocates device memory itself: a plan's device tables and scratch live in a
 * workspace the caller binds.  "stream" is a hipStream_t (NULL = the null
 * stream); every call only enqueues work on it.  A plan must be used by one
 * stream at a time.  Device-side argument errors (a delay outside
 * [0, max_delay]) are recorded in the workspace and reported by
 * corr_check_device_errors.
 */
#ifndef CORR_H
#define CORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t corr_status;

#define CORR_OK 0
#define CORR_ERR_INVALID (-1)     /* an argument value is out of range          */
#define CORR_ERR_NULL (-2)        /* a required pointer is NULL                 */
#define CORR_ERR_ALIGN (-3)       /* a pointer or stride is misaligned          */
#define CORR_ERR_UNSUPPORTED (-4) /* shape / precision not built for this GPU   */
#define CORR_ERR_WORKSPACE (-5)   /* no workspace bound, or too small           */
#define CORR_ERR_OVERFLOW (-6)    /* int32 accumulator bound would be exceeded  */
#define CORR_ERR_DEVICE (-7)      /* HIP runtime error (message in last_error)  */
#define CORR_ERR_NOMEM (-8)       /* host allocation failed                     */
#define CORR_ERR_STATE (-9)       /* call sequence not allowed in this state    */
#define CORR_ERR_DEVICE_ARG (-10) /* a device-resident argument was invalid     */
#define CORR_ERR_IO (-11)         /* file could not be opened, read or written  */

/* Arithmetic of the spectra handed from the F- to the X-engine. */
#define CORR_FP32 0     /* complex64 spectra, FP32 MFMA X-engine                */
#define CORR_INT8 1     /* int8 (re, im) in [-127, 127], int8 MFMA, int32 sums  */
#define CORR_FP8_E4M3 2 /* OCP e4m3 (re, im), FP8 MFMA, FP32 sums               */

/* Requantisation scale handling (INT8 / FP8 only). */
#define CORR_SCALE_HOLD 0    /* use the scales passed in d_scale (set once,      */
                             /* like the paper's gain table, section 2.3.2)     */
#define CORR_SCALE_COMPUTE 1 /* measure sigma on this call's spectra first and   */
                             /* write the scales to d_scale (two passes)        */

/* corr_integrate flags */
#define CORR_DUMP 1u  /* write the accumulated visibilities to d_vis_out         */
#define CORR_RESET 2u /* zero the FP64 state after the (optional) dump          */

/* Plan description. */
typedef struct {
    int32_t n_signals;    /* S, 1..64                                            */
    int32_t fft_len;      /* N, power of two, 512..16384                         */
    int64_t n_spectra;    /* T, spectra per call, multiple of 32, >= 32          */
    int32_t max_delay;    /* largest integer delay D in samples (>= 0); the      */
                          /* rows of the input carry T*N + max_delay samples    */
    int32_t precision;    /* CORR_FP32 / CORR_INT8 / CORR_FP8_E4M3               */
    int32_t sideband;     /* sigma of Eq. 2: +1 (nu_RF >= nu_LO) or -1           */
    int32_t scale_mode;   /* CORR_SCALE_HOLD / CORR_SCALE_COMPUTE                */
    double sample_rate;   /* fs in Hz (> 0)                                      */
    double nu_bb;         /* baseband frequency of the band's lower edge (Hz)    */
    int32_t x_split;      /* X-engine K-splits (0 = library choice)              */
    int32_t phase_lut;    /* 0: FSTC/fringe phase evaluated directly (FP32     */
                          /* sincos); 1: the paper's 1440-step sin/cos table    */
                          /* (section 2.3.2): the phase k f/N + c_m of Eq. 2 is */
                          /* formed in FP64 per channel and spectrum, rounded   */
                          /* to the nearest 0.25 degree step, and that step's   */
                          /* FP32 cos and sin are used (error <= 0.125 deg)     */
    int32_t power_fp16;   /* power cells of corr_fengine / corr_mad_flag: 0 FP32 */
                          /* |X|^2; 1 FP16 |X|^2 / N^2 (half the bytes; real    */
                          /* int8 input keeps |X| <= 127 N, so no overflow)     */
    int32_t reserved[5];  /* must be zero                                        */
} corr_desc_t;

/*
 * Per-signal geometry of one call (section 2.1, Eq. 2), device-resident so
 * that captured graphs read fresh values:
 *   D     integer delay in samples; window m of signal s starts at sample
 *         m*N + D of its row (read-pointer advance, section 2.3.2)
 *   frac  fractional delay f in samples, [0, 1): tau_frac = f / fs
 *   psi0  fringe phase (cycles) at the call's reference epoch
 *   rate  fringe rate (Hz)
 * Spectrum m (absolute index spectrum0 + m) is phase-corrected by
 *   exp(+2 pi i [ (nu_BB + k fs/N) f/fs + sideband (psi0 + rate t_m) ]),
 *   t_m = (spectrum0 + m + 1/2) N / fs  (window centre).
 * 24 bytes, 8-byte aligned.
 */
typedef struct {
    int32_t D;
    float frac;
    double psi0;
    double rate;
} corr_geom_t;

typedef struct corr_plan corr_plan_t;

/*
 * Geometry of one call from an antenna-based delay model (section 2.1, Eq. 1
 * and Eq. 2; host arithmetic in FP64, like the per-slice delay parameters of
 * section 2.3.2).  The total delay of signal s at stream time t (seconds
 * since sample 0 of its row) is
 *   tau_s(t) = h_tau0[s] + h_taudot[s] (t - t0)        (seconds, s/s)
 * and the call's geometry is
 *   D_s + f_s = tau_s(t_delay) * sample_rate, D_s = floor(.), f_s in [0, 1):
 *       the integer delay (read-pointer advance) and the fractional sample
 *       time correction, held for the whole call (t_delay is normally the
 *       call's centre);
 *   psi0_s + rate_s t_m = nu_lo * tau_s(t_m + tau_s(t_delay)): the fringe
 *       term (nu_RF - nu_BB) tau_tot of Eq. 2, nu_lo = nu_RF - nu_BB >= 0 the
 *       local-oscillator frequency, at the time the samples of spectrum m
 *       arrived -- its aligned time stamp t_m (corr_geom_t) plus the delay
 *       the read pointer skips (rate * tau is up to 6.4e-4 cycles at 5 Hz and
 *       128 us).  So rate_s = nu_lo * h_taudot[s] (Hz) and psi0_s =
 *       nu_lo * (tau_s(0) + h_taudot[s] tau_s(t_delay)) reduced mod 1
 *       (cycles).  Its sign is the plan's sideband, which the F-engine
 *       applies.
 * f_s is stored as float: a fraction that rounds up to 1 is carried into D_s.
 * nu_lo * tau_s(0) is formed with error-free transforms (the rounding errors
 * of its products and difference are kept and added after the reduction mod
 * 1), so psi0 carries ~1e-16 cycles of error for any nu_lo tau below 2^50
 * cycles -- 1.4 GHz x 128 us is 179200 cycles.
 *   n_signals >= 1; h_tau0, h_taudot: double[n_signals]; h_geom: corr_geom_t
 *   [n_signals] (host).  max_delay >= 0 bounds D_s (pass the plan's).
 * Errors: NULL, INVALID (n_signals < 1, a non-finite input, sample_rate <= 0,
 * nu_lo < 0, or a signal whose D_s falls outside [0, max_delay]); the message
 * names the signal, via corr_last_error(NULL).  Nothing is written on error.
 */
corr_status corr_geom_from_model(int32_t n_signals, const double *h_tau0, const double *h_taudot, double t0,
                                 double t_delay, double sample_rate, double nu_lo, int32_t max_delay,
                                 corr_geom_t *h_geom);

/* ----------------------------------------------------------------- plans */

/* Validate desc and build host tables.  Errors: NULL, INVALID (shape, rate,
 * sideband, reserved fields), UNSUPPORTED (no gfx950 device current), NOMEM. */
corr_status corr_plan_create(const corr_desc_t *desc, corr_plan_t **out);
void corr_plan_destroy(corr_plan_t *plan);

/* Bytes of device workspace the plan needs (twiddle and pair tables,
 * calibration partial sums, device error word).  0 on a NULL plan. */
size_t corr_plan_workspace_bytes(const corr_plan_t *plan);
/* Sizes of the caller-owned buffers of the data path (bytes):
 *   spectra  F-engine output / X-engine input, layout below
 *   acc      X-engine accumulator, [splits][C][P][2] int32 (INT8) or float
 *   state    integrator state, [C][P][2] double
 *   vis      dumped visibilities, [C][P][2] float (complex64) */
size_t corr_plan_spectra_bytes(const corr_plan_t *plan);
size_t corr_plan_acc_bytes(const corr_plan_t *plan);
size_t corr_plan_state_bytes(const corr_plan_t *plan);
size_t corr_plan_vis_bytes(const corr_plan_t *plan);
int32_t corr_plan_x_splits(const corr_plan_t *plan);
/* Name of the F-engine kernel the plan's corr_fengine launches for its data
 * (as a profiler lists it: "fengine4_kernel<log2 M, mode>" for the four-step
 * one, "fengine_kernel<...>" for the LDS-radix one; mode 0 FP32, 1 int8, 2
 * e4m3, plus 4 in table mode), for a call without power cells (with them the
 * four-step kernel's mode adds 4 for FP32 and 8 for FP16 cells).  The string
 * is valid until the calling thread's next call; "" for a NULL plan. */
const char *corr_plan_fengine_kernel(const corr_plan_t *plan);

/* Attach caller-owned device workspace (>= workspace_bytes, 256-byte
 * aligned) and upload the tables on `stream`.  The workspace must stay
 * allocated while the plan is used.  Errors: NULL, ALIGN, WORKSPACE, DEVICE. */
corr_status corr_plan_bind_workspace(corr_plan_t *plan, void *d_ws, size_t bytes,
                                     void *stream);

/* --------------------------------------------------------------- F-engine */

/*
 * Channelise T spectra of all S signals.
 *   d_x        int8 samples, row s at d_x + s*row_stride; 16-byte aligned;
 *              row_stride a multiple of 16 and >= T*N + max_delay
 *   d_geom     corr_geom_t[S] (device)
 *   spectrum0  absolute index of this call's first spectrum (fringe time)
 *   d_spec     output spectra, corr_plan_spectra_bytes, 256-byte aligned,
 *              in 16-byte chunks indexed [g][k/8][s][k mod 8] (the chunks of
 *              8 consecutive channels of one signal form one 128-byte line):
 *                FP32: chunk g of channel k, signal s = spectra 2g, 2g+1 as
 *                      two complex64
 *                INT8 / FP8: chunk g = bytes 0..7 the real parts of spectra
 *                      8g..8g+7, bytes 8..15 their imaginary parts
 *   d_scale    [S][C] float; INT8: q = clamp(rne(Y / scale), -127, 127)
 *              (Y / scale + 128 is formed in FP32 before the rounding, so a
 *              code may differ from that of the exact quotient only within
 *              2^-16 of a .5 boundary), FP8: q = e4m3_rne_satfinite(Y /
 *              scale).  Read in HOLD mode,
 *              written (scale = 4 sigma / 127 or 4 sigma / 448, sigma the RMS
 *              of one component of Y over this call) in COMPUTE mode.
 *              Unused (may be NULL) for FP32.
 *   d_power    optional (NULL: not written) power of every cell, [S][T][C]
 *              -- the dynamic spectra the flaggers below read
 *              (corr_plan_power_bytes): FP32 |X|^2, or with the plan's
 *              power_fp16 FP16 |X|^2 / N^2 (the FP32 value times the exact
 *              power of two, rounded to nearest even); X before phase
 *              rotation and requantisation (the rotation keeps |X|).  4-byte
 *              (FP32) or 2-byte (FP16) aligned.
 * Errors: NULL, ALIGN, INVALID (row_stride), WORKSPACE, DEVICE.
 */
corr_status corr_fengine(corr_plan_t *plan, const int8_t *d_x, int64_t row_stride,
                         const corr_geom_t *d_geom, int64_t spectrum0, void *d_spec,
                         float *d_scale, void *d_power, void *stream);

/* Corner turn of externally produced spectra into the X layout above.
 *   d_in: [S][T][C][2] elements (float for FP32, int8 for INT8, e4m3 bytes
 *   for FP8), 16-byte aligned.  Errors: NULL, ALIGN, DEVICE. */
corr_status corr_xpack(corr_plan_t *plan, const void *d_in, void *d_spec, void *stream);

/* Requantisation of externally produced FP32 spectra with the F-engine's own
 * encoders' definitions (section 4.1: a fixed-point format with a per-channel
 * level ahead of the MAC): per component q = enc(v * (1 / d_scale[s][k])), enc the INT8
 * plan's clamp(rne(.), +-127) or the FP8 plan's OCP e4m3 (nearest even,
 * saturating at +-448, +0 for values that round to zero; NaN gives -127 or
 * -448).  d_in: float [S][T][C][2], 8-byte aligned; d_scale: float [S][C];
 * d_out: codes [S][T][C][2] (int8 or e4m3 bytes), 2-byte aligned, ready for
 * corr_xpack.  Errors: NULL, ALIGN, UNSUPPORTED (an FP32 plan), DEVICE. */
corr_status corr_requantize(corr_plan_t *plan, const float *d_in, const float *d_scale, void *d_out, void *stream);

/* --------------------------------------------------------------- X-engine */

/*
 * d_acc[split][k][p] += sum over this split's spectra of Y_i conj(Y_j), for
 * every channel k and pair p (section 2.1's cross-multiplication of every
 * pair, integrated over time; int32 exact for INT8; float for FP32/FP8).
 *   d_spec   the X layout above, 256-byte aligned; not modified.
 *   d_keep   optional flag mask (section 5: flagged data take no part in the
 *            products) as the bit-packed keep words of corr_apply_flags,
 *            [C/8][T/32][S][8] uint32 (channel k's word w of signal s at
 *            ((k/8 * T/32 + w) S + s) 8 + k mod 8), bit i of word w =
 *            spectrum 32 w + i kept;
 *            a cleared bit zeroes that cell of Y inside the X-engine, so the
 *            result equals corr_apply_flags' zeroing followed by this call
 *            without d_keep (bit-exact), without writing the spectra.  NULL:
 *            every cell.  4-byte aligned.
 *   d_acc    corr_plan_acc_bytes, 256-byte aligned, zeroed once before the
 *            first call (corr_integrate zeroes it afterwards).
 *   d_counts optional (needs d_keep and the bound workspace): += the exact
 *            per-pair unflagged counts, as corr_pair_counts (int32 [C][P]),
 *            4-byte aligned.
 * INT8: rejects with OVERFLOW a call that would take the spectra accumulated
 * since the last corr_integrate above 66572 (2 * 127^2 * T < 2^31).  COMPUTE
 * scale mode: rejects with STATE a second call before corr_integrate, since
 * the scales change per call.  Errors: NULL (also d_counts without d_keep),
 * ALIGN, WORKSPACE (d_counts without a bound workspace), OVERFLOW, STATE,
 * DEVICE.
 */
corr_status corr_xengine(corr_plan_t *plan, const void *d_spec, const uint32_t *d_keep, void *d_acc,
                         int32_t *d_counts, void *stream);

/* ------------------------------------------------------- gated correlator */

/* Gated correlator (section 5: the pulsar-gated mode, for off-pulse emission
 * and pulsars as phase calibrators): accumulator set b sums only the spectra
 * whose gate is b,
 *   d_acc_b[split][k][p] += sum over m with gate[m] == b of Y_i conj(Y_j),
 * for b = 0 .. n_bins-1, in one launch that reads the spectra once (every
 * product's second operand is masked per spectrum in registers).  The sum of
 * all sets is the ungated corr_xengine result (exactly for INT8).
 *   d_gate   uint8 [T], the bin of each spectrum of the call; a value
 *            >= n_bins leaves the spectrum out of every set.  16-byte aligned.
 *   d_acc    n_bins consecutive accumulators of corr_plan_acc_bytes each
 *            (set b at d_acc + b * corr_plan_acc_bytes), 256-byte aligned,
 *            zeroed before the first call like corr_xengine's.
 * Integrate each set with corr_integrate.  The INT8 bound and the COMPUTE
 * scale rule are those of corr_xengine, counted per call: integrate every set
 * before 66572 spectra have accumulated.
 * Errors: NULL, ALIGN, INVALID (n_bins outside [1, CORR_MAX_GATE_BINS]),
 * OVERFLOW, STATE, DEVICE. */
#define CORR_MAX_GATE_BINS 255
corr_status corr_xengine_gated(corr_plan_t *plan, const void *d_spec, const uint8_t *d_gate, int32_t n_bins,
                               void *d_acc, void *stream);

/* Gates of spectra spectrum0 .. spectrum0 + n_spectra - 1 from a pulsar's
 * period (host arithmetic, FP64, like the delay model): spectrum m is taken
 * at its window centre t = (m + 1/2) fft_len / sample_rate (the time stamp of
 * the fringe phase), its pulse phase is frac((t - t0) / period), and
 * h_gate[m - spectrum0] = floor(phase * n_bins) (at most n_bins - 1).
 * h_counts (optional, int64 [n_bins], host) gets each bin's spectra added.
 * Errors: NULL, INVALID (negative counts, fft_len < 1, non-finite or
 * non-positive rate or period, n_bins); messages via corr_last_error(NULL). */
corr_status corr_pulsar_gates(int64_t spectrum0, int64_t n_spectra, int32_t fft_len, double sample_rate, double t0,
                              double period, int32_t n_bins, uint8_t *h_gate, int64_t *h_counts);

/* ------------------------------------------------------------- beamformer */

/*
 * Array beams from X-layout spectra: the two beamformer modes of section 2.2,
 * on the F-engine output as in section 2.3.2 (one incoherent and coherent beams
 * at the raw FFT time resolution, optionally summed over a few spectra).
 * Per spectrum m, channel k and polarisation pol (signals s = 2a + pol; an
 * odd S leaves the last antenna with polarisation 0 only), with Y_s the
 * spectra (INT8 / FP8 codes times d_scale[s][k]; FP32 as stored):
 *   incoherent     I_pol = sum_s w_s |Y_s|^2 over the signals of pol
 *                  (d_w[S] >= 0; 0 leaves a signal out)
 *   coherent b     V_b,pol = sum_s c_b,s Y_s over the signals of pol
 *                  (d_c[n_beams][S] complex as (re, im) float pairs: gain and
 *                  antenna-based phase of beam b)
 * Coherent outputs by mode:
 *   CORR_BEAM_INTENSITY  2 planes: |V_b,0|^2, |V_b,1|^2
 *   CORR_BEAM_FULLPOL    4 planes: |V_b,0|^2, |V_b,1|^2, Re and Im of
 *                        V_b,0 conj(V_b,1) (every product the Stokes
 *                        parameters need)
 *   CORR_BEAM_VOLTAGE    2 planes of complex64: V_b,0, V_b,1 (tint = 1)
 * Every plane is [T/tint][C], summed over tint = 1, 2, 4 or 8 consecutive
 * spectra.  d_inc: [2][T/tint][C] float (NULL: no incoherent beam; d_w is
 * then unused).  d_coh: [n_beams][planes][T/tint][C] (unused if n_beams = 0).
 * n_beams 0..CORR_MAX_BEAMS; at least one beam of either kind.  d_scale is
 * required for INT8 / FP8 and ignored for FP32.  d_spec 256-byte aligned,
 * the rest 4-byte aligned (d_coh 8-byte aligned for VOLTAGE).
 * Errors: NULL, ALIGN, INVALID, DEVICE.
 */
#define CORR_MAX_BEAMS 4
#define CORR_BEAM_INTENSITY 0
#define CORR_BEAM_FULLPOL 1
#define CORR_BEAM_VOLTAGE 2
corr_status corr_beamform(corr_plan_t *plan, const void *d_spec, const float *d_scale, const float *d_w,
                          float *d_inc, const float *d_c, int32_t n_beams, int32_t mode, float *d_coh,
                          int32_t tint, void *stream);

/* -------------------------------------------------------------- integrate */

/*
 * d_state[k][p] += (INT8/FP8: scale_i[k] * scale_j[k] *) sum_split d_acc,
 * in FP64 (the paper's float long-term accumulation, section 4.1), then
 * zero d_acc.  CORR_DUMP: d_vis_out[k][p] = (complex64) d_state[k][p].
 * CORR_RESET: d_state = 0 afterwards.  d_scale is ignored for FP32.
 * Errors: NULL, ALIGN, DEVICE.
 */
corr_status corr_integrate(corr_plan_t *plan, void *d_acc, const float *d_scale,
                           double *d_state, float *d_vis_out, uint32_t flags, void *stream);

/* ---------------------------------------- 16-bit fixed-point emulation */

/* The 16-bit fixed-point numerics of the paper's real-time pipeline, beside
 * the FP32, INT8 and FP8 paths for the precision comparison of section 4.1:
 * the FFT output held as 16-bit integers (section 3.1's 16-bit fixed-point
 * real FFT, whose butterflies run in floating point), the fringe stop and
 * FSTC by an integer multiply with the phase table scaled so that the result
 * keeps 16 bits (section 4.1), and exact correlation products of the 16-bit
 * data (32-bit products, section 4.1) accumulated in integers, then floating
 * point.
 *
 * corr_fix16_spectra reads the spectra an FP32 plan's corr_fengine wrote with
 * a geometry whose frac, psi0 and rate are zero (the integer delay applied,
 * the FFT output unrotated; nu_BB of the plan then plays no part in it), and
 * per signal s, spectrum m, channel k and component:
 *   q = sat16(round-half-even(X / d_scale[s][k]))   the 16-bit FFT output
 *   j = nearest of the 1440 steps of section 2.3.2 to the Eq. 2 phase of
 *       d_geom (formed in FP64 as in phase_lut mode, spectrum0 + m absolute)
 *   y = sat16(floor((q w_j + 2^13) / 2^14))         (complex product; w_j =
 *       rint(2^14 cos, 2^14 sin) of the step: rounded, not truncated)
 * with sat16 clamping to [-32767, 32767].  d_y16 (and d_q16 if not NULL):
 * int16 [S][T][C][2], 4-byte aligned.  d_scale: float [S][C] (the level of
 * each signal and channel; 4 sigma / 32767 uses the 16-bit range as the int8
 * path uses its own).  Errors: NULL, INVALID (not an FP32 plan, spectrum0),
 * ALIGN, WORKSPACE, DEVICE. */
corr_status corr_fix16_spectra(corr_plan_t *plan, const void *d_spec, const corr_geom_t *d_geom, int64_t spectrum0,
                               const float *d_scale, int16_t *d_q16, int16_t *d_y16, void *stream);

/* d_acc[k][p] = sum over the plan's T spectra of y_i conj(y_j) (int64, [C][P]
 * [2]; each product exact in 32 bits, the sums exact), and, if d_vis is not
 * NULL, d_vis[k][p] = d_acc * scale_i[k] * scale_j[k] in FP64 ([C][P][2]).
 * d_y16 as corr_fix16_spectra writes it.  Writes (does not accumulate).
 * Errors: NULL, ALIGN, DEVICE. */
corr_status corr_fix16_xengine(corr_plan_t *plan, const int16_t *d_y16, const float *d_scale, int64_t *d_acc,
                               double *d_vis, void *stream);

/* --------------------------------------------------------------- flagging */

/* RFI flags from the MAD statistic of section 5 (Eq. 3: MAD = median
 * |x - median(x)|; Eq. 4: flag when |x - median(x)| > M MAD / 0.6745), taken
 * per signal on tiles of 64 spectra x 256 channels of d_power: the row
 * statistic (mean power of a spectrum over the tile's channels) exposes
 * broadband bursts, the column statistic (mean power of a channel over the
 * tile's spectra) persistent tones; a cell is flagged (1) when its row or its
 * column is.  Median of an even count = mean of the two middle values.
 *   d_power  [S][T][C], the plan's power type (FP32, or FP16 with
 *            power_fp16: the statistics are taken in FP32 either way and do
 *            not depend on the scale), 16-byte aligned.
 *   d_flags  [S][T][C] uint8 (corr_plan_flags_bytes), 16-byte aligned.
 * Needs T % 64 == 0 (C = N/2 >= 256 is always a multiple of 256).
 * Errors: NULL, ALIGN, INVALID (shape, M <= 0), DEVICE. */
corr_status corr_mad_flag(corr_plan_t *plan, const void *d_power, float M, uint8_t *d_flags,
                          void *stream);

/* Zero the flagged cells of X-layout spectra in place (both components;
 * d_spec NULL: leave the spectra alone), and optionally (d_keep != NULL) write
 * bit-packed keep masks [C/8][T/32][S][8] uint32 (channel k's word w of
 * signal s at ((k/8 * T/32 + w) S + s) 8 + k mod 8: the order in which the
 * X-engine reads them; bit i of word w = spectrum
 * 32 w + i not flagged; corr_plan_keep_bytes), which corr_xengine can apply
 * itself instead of the zeroing.  d_flags may come from corr_mad_flag or from
 * any other flagger.  Errors: NULL (also d_spec and d_keep both NULL), ALIGN,
 * DEVICE. */
corr_status corr_apply_flags(corr_plan_t *plan, const uint8_t *d_flags, void *d_spec,
                             uint32_t *d_keep, void *stream);

/* d_counts[k][p] += n_ij[k] = sum_m (1 - F_i[m,k]) (1 - F_j[m,k]): the number
 * of spectra in which neither signal of pair p was flagged (int32 [C][P],
 * exact; zero it before the first call).  Divide an integrated visibility by
 * it for a flag-corrected mean.  Errors: NULL, ALIGN, WORKSPACE, DEVICE. */
corr_status corr_pair_counts(corr_plan_t *plan, const uint32_t *d_keep, int32_t *d_counts,
                             void *stream);

size_t corr_plan_power_bytes(const corr_plan_t *plan);
size_t corr_plan_flags_bytes(const corr_plan_t *plan);
size_t corr_plan_keep_bytes(const corr_plan_t *plan);

/* ------------------------------------------------- coherent dedispersion */

/* Coherent dedispersion of phased-array voltages (section 4.3: the coherent
 * beam's pre-detected voltages converted to a broadband series by inverse
 * FFT, multiplied by the inverse of the interstellar dispersion kernel in the
 * Fourier domain, detected, polarisations added, integrated).
 *   d_v      complex64 [npol][T][C]: the channel voltages of one beam (for
 *            example corr_beamform's CORR_BEAM_VOLTAGE output of one beam),
 *            upper sideband, channel k at sky frequency nu0 + k fs/N, N = 2C.
 *            Not modified.  8-byte aligned.
 *   Steps: z[m C + n] = sum_k V[m][k] exp(+2 pi i k n / C) (complex baseband
 *   at fs/2); its L = T C point transform times
 *   exp(-2 pi i K DM f^2 / (nu0^2 (nu0 + f))), f = q fs / (2L), K =
 *   4.148808e15 Hz^2 s / (pc cm^-3) (group delay K DM (nu^-2 - nu0^-2): every
 *   frequency is aligned to its arrival at nu0); the inverse transform / L;
 *   I[j] = sum over polarisations and samples j n_int .. j n_int + n_int - 1
 *   of |z|^2.
 *   The transform is circular: the first K DM (nu0^-2 - (nu0 + fs/2)^-2) fs/2
 *   output samples (the sweep across the band) are not valid; consecutive
 *   blocks should overlap by that many samples.
 *   npol     1 or 2.  C a power of two in [16, 8192]; T a power of two;
 *            T C in [4096, 2^28].  n_int a power of two <= T C.
 *   d_work   corr_dedisperse_workspace_bytes(npol, T, C) bytes, 8-byte
 *            aligned, not d_v; holds the dedispersed voltages afterwards.
 *   d_out    float [T C / n_int].
 * FP32 transforms (error about 1e-6 of the rms at T C = 2^24), the chirp
 * phase in FP64 reduced mod 1.  Errors: NULL, ALIGN, INVALID, DEVICE;
 * messages via corr_dedisperse_last_error. */
corr_status corr_dedisperse(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate, double nu0,
                            double dm, int32_t n_int, float *d_work, float *d_out, void *stream);
size_t corr_dedisperse_workspace_bytes(int32_t npol, int64_t T, int32_t C);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): corr_dedisperse
 * without d_work.  Its work buffer is a file-scope device array of
 * CORR_DEDISPERSE_NOALLOC_MAX complex samples (32 MiB) that the library holds
 * on every GPU it runs on until the process ends; the call itself allocates
 * nothing.  Same arguments, results and errors as corr_dedisperse, plus
 * INVALID when npol * T * C exceeds CORR_DEDISPERSE_NOALLOC_MAX, and
 * UNSUPPORTED on a device id of 64 or more.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race, and each call's transform overwrites the previous one's. */
#define CORR_DEDISPERSE_NOALLOC_MAX ((int64_t)1 << 22)
corr_status corr_dedisperse_noalloc(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate,
                                    double nu0, double dm, int32_t n_int, float *d_out, void *stream);
const char *corr_dedisperse_last_error(void);

/* ------------------------------------------------------------- ADC input */

/* Demultiplex and unpack the raw streams of the acquisition cards (sections
 * 2.3.2 and 3.3): each card digitises four inputs, 8-bit (16 MHz mode) or
 * 4-bit (33 MHz mode), and the compute side separates the four streams and
 * unpacks 4-bit samples to 8 bits before the FFT.
 *   d_raw       card c's stream at d_raw + c*raw_stride, time-major with the
 *               four inputs of a time sample together: 8-bit, byte 4t + i is
 *               input i; 4-bit, byte 2t + i/2, nibble i mod 2 (low nibble
 *               first).  Two's complement.  16-byte aligned; raw_stride a
 *               multiple of 16 and >= n*bits/2.
 *   n           time samples per card (0 enqueues nothing; at most 2^40).
 *   d_x         int8 rows, row 4c + i (input i of card c) at
 *               d_x + (4c + i)*row_stride, n samples each: the layout
 *               corr_fengine reads.  4-bit samples are sign-extended (value
 *               kept, -8..7).  16-byte aligned; row_stride a multiple of 16
 *               and >= n.  Must not overlap d_raw.  Bytes of a row past n are
 *               not written.
 * Errors: NULL, ALIGN, INVALID (bits not 4 or 8, n_cards outside
 * [1, 16383], n, strides), DEVICE; messages via corr_adc_last_error. */
corr_status corr_adc_unpack(const uint8_t *d_raw, int64_t raw_stride, int32_t n_cards, int64_t n, int32_t bits,
                            int8_t *d_x, int64_t row_stride, void *stream);

/* Message of the last failed corr_adc_unpack call on this thread. */
const char *corr_adc_last_error(void);

/* ------------------------------------------------------- voltage blanker */

/* Time-domain RFI blanker on the pre-detected voltages (section 5, Eq. 3 and
 * Eq. 4).  It runs on the int8 sample rows corr_fengine reads, before the FFT.
 * Each block of `block` consecutive samples of a row is handled on its own
 * (the last block of a row may be shorter): x~ = median, MAD = median
 * |x - x~| (median of an even count = mean of the two middle values).  A
 * sample with |x - x~| > M MAD / 0.6745 is replaced by
 * rint(x~ + (MAD / 0.6745) z), clamped to [-128, 127] (rint: nearest, ties to
 * even).  z is entry (sample0 + i) mod table_len of the signal's row of a
 * precomputed Gaussian noise table (corr_blank_noise_table), so the
 * replacements are independent between antennas.  A block with MAD = 0 has
 * no scale estimate and passes unchanged.  The median and the MAD are exact,
 * and the threshold and the replacements are evaluated in FP64, so the
 * output is one definite array.
 *   d_x        S rows of int8 samples, row s at d_x + s*row_stride, n samples
 *              each; row_stride a multiple of 16 and >= n; 16-byte aligned.
 *              Whole 16-byte chunks are read, so each row must be addressable
 *              up to n rounded up to 16 (true for S full rows of row_stride).
 *   block      multiple of 16 in [16, 65536] (the paper leaves the block
 *              length to the user; a few thousand samples suit impulsive RFI).
 *   M          threshold, finite and > 0 (2.5 to 3.0 in the paper).
 *   d_table    [S][table_len] float, table_len a power of two <= 2^31.
 *   sample0    absolute index of each row's first sample (>= 0), so that
 *              consecutive calls on a stream draw consecutive table entries.
 *   d_out      same layout as d_x.  Either d_x itself (in place: only 16-byte
 *              chunks holding a blanked sample are written), or a buffer that
 *              does not overlap it (every sample is written).
 *   d_counts   optional [S][ceil(n / block)] int32: samples blanked per block.
 *   d_stats    optional [S][ceil(n / block)][2] int32: (2 x~, 4 MAD) per block,
 *              both integers for int8 data.
 * n == 0 enqueues nothing.  Calls that overlap on the same buffers race.
 * Errors: NULL, ALIGN, INVALID (S outside [1, 65535], n < 0, row_stride,
 * block, M, table_len, sample0 < 0 or sample0 + n above 2^63 - 1, more than
 * 2^31 - 1 blocks), DEVICE;
 * messages via corr_blank_last_error. */
corr_status corr_blank_voltages(const int8_t *d_x, int64_t row_stride, int32_t S, int64_t n, int32_t block,
                                float M, const float *d_table, int64_t table_len, int64_t sample0, int8_t *d_out,
                                int32_t *d_counts, int32_t *d_stats, void *stream);

/* Fill d_table [S][L] (float, 4-byte aligned; L a power of two <= 2^31) with
 * the blanker's precomputed Gaussian noise (section 5): entry j of signal s is
 * the sum of twelve uniforms (U + 1/2) / 65536 minus 6 (mean 0, variance 1,
 * the Irwin-Hall approximation of a normal deviate, |z| < 6).  The U are the
 * 16-bit halves, low then high, of words 0..3 of Philox4x32-10 (Salmon et al.,
 * SC'11) at counter (j mod 2^32, j / 2^32, s, 0) and words 0..1 at counter
 * (.., s, 1), with key (seed mod 2^32, seed / 2^32).  One row per signal makes
 * the replacements of different antennas independent.  Every value is exact
 * in float.  Errors: NULL, ALIGN, INVALID (S outside [1, 65535], L), DEVICE. */
corr_status corr_blank_noise_table(uint64_t seed, int32_t S, int64_t L, float *d_table, void *stream);

/* Message of the last failed blanker call on this thread ("" after success). */
const char *corr_blank_last_error(void);

/* ------------------------------------------------------------------ batch */

/* Several correlations of different shapes (the paper runs sub-arrays and
 * modes side by side, and sizes each compute node's time slice to its
 * capability, section 2.3.2) driven as one unit: the F-engines of the
 * sub-arrays run concurrently on forked streams, one X-engine launch covers
 * the tasks (channel block x split) of every sub-array, then each sub-array
 * is integrated.  INT8 with held scales only; up to 8 sub-arrays, each with
 * T <= 66572 (one integration per run).  The whole run can be captured once
 * into a HIP graph and replayed with a single launch; geometry, scales and
 * data are read from the recorded device pointers at every replay. */
typedef struct corr_batch corr_batch_t;

typedef struct {
    const int8_t *x;         /* input rows, as corr_fengine                   */
    int64_t row_stride;
    const corr_geom_t *geom; /* corr_geom_t[S]                                */
    int64_t spectrum0;
    void *spec;              /* X-layout spectra (corr_plan_spectra_bytes)     */
    float *scale;            /* held int8 scales [S][C]                        */
    void *acc;               /* accumulator (corr_plan_acc_bytes), zeroed      */
    double *state;           /* integrator state                               */
    float *vis;              /* dump (NULL unless flags has CORR_DUMP)         */
    uint32_t flags;          /* corr_integrate flags                           */
} corr_batch_io_t;

/* Errors: NULL, INVALID (count, scale mode), UNSUPPORTED (non-INT8), OVERFLOW
 * (an entry with more than 66572 spectra: one run sums its whole call in the
 * int32 accumulator before integrating it), DEVICE, NOMEM. */
corr_status corr_batch_create(const corr_desc_t *descs, int n, corr_batch_t **out);
void corr_batch_destroy(corr_batch_t *batch);
/* Sub-plan i (owned by the batch): query its sizes and bind its workspace. */
corr_plan_t *corr_batch_plan(corr_batch_t *batch, int i);
/* Record the buffers of sub-array i.  Errors: NULL, INVALID, ALIGN, WORKSPACE. */
corr_status corr_batch_set_io(corr_batch_t *batch, int i, const corr_batch_io_t *io);
/* Enqueue one batch pass on `stream`.  Errors: STATE (missing io), DEVICE. */
corr_status corr_batch_run(corr_batch_t *batch, void *stream);
/* Capture corr_batch_run into a HIP graph (stream must be non-NULL).
 * Errors: NULL, INVALID, STATE, DEVICE. */
corr_status corr_batch_capture(corr_batch_t *batch, void *stream);
/* Replay the captured graph.  Errors: STATE (not captured), DEVICE. */
corr_status corr_batch_launch(corr_batch_t *batch, void *stream);
const char *corr_batch_last_error(const corr_batch_t *batch);

/* --------------------------------------------------------------- autotune */

/* Time the X-engine of desc for every K-split in 1..64 that divides T/32
 * (each the median of 5 launches after one warm-up launch) and return the
 * fastest in *best_split (its median time in *best_ms when non-NULL); the
 * split goes into corr_desc_t.x_split.  The tile body is fixed by S (one
 * 32-signal tile up to 32 signals, two above: the two-tile body on fewer
 * signals does more matrix work on the same bytes).  Uses caller scratch of
 * corr_autotune_scratch_bytes(desc) (256-byte aligned; contents ignored) and
 * synchronises `stream`.  Errors: NULL, ALIGN, WORKSPACE, INVALID, DEVICE. */
size_t corr_autotune_scratch_bytes(const corr_desc_t *desc);
corr_status corr_autotune_x_split(const corr_desc_t *desc, void *d_scratch, size_t bytes, void *stream,
                                  int32_t *best_split, float *best_ms);

/* ---------------------------------------------------------- learned flagger */

/* A convolutional RFI flagger trained on the GPU against the MAD flags above
 * (the paper's MAD filter of section 5, Eq. 3 and Eq. 4, is the teacher; the
 * paper itself notes that better filtering has room to improve).  It works on
 * the same 64 x 256 (spectra x channels) tiles of one signal's power, each
 * tile its own zero-padded image:
 *   x  = log(1 + P / m), m = median over the tile's 256 channels of each
 *        channel's mean power over the tile's 64 spectra (1 if not > 0)
 *   z1 = conv3x3(x; 1 -> 16), a1 = ReLU(z1)
 *   z2 = conv3x3(a1; 16 -> 16), a2 = ReLU(z2)
 *   z3 = conv3x3(a2; 16 -> 1), the logit; a cell is flagged when
 *        sigmoid(z3) > threshold
 * conv3x3(a)[o][r][c] = b[o] + sum_{i,u,v} w[o][i][u][v] a[i][r+u-1][c+v-1]
 * with a = 0 outside the tile.  Training minimises the mean binary
 * cross-entropy of sigmoid(z3) against the labels with Adam (Kingma & Ba
 * 2015, Algorithm 1).
 *
 * Parameters: CORR_CNN_PARAMS floats on the device, layer by layer, each
 * layer's weights [Cout][Cin][3][3] then its biases [Cout].  Tiles of power
 * [S][T][C] (T a multiple of 64, C of 256) are numbered
 * tile = (s (T/64) + m/64) (C/256) + k/256.  The training calls work on a
 * caller-chosen list of tile numbers (device int32[n_tiles], n_tiles <=
 * max_tiles); an out-of-range number is recorded in the workspace (reported by
 * corr_cnn_check_device_errors) and that tile reads as zeros. */
#define CORR_CNN_PARAMS 2625

typedef struct corr_cnn corr_cnn_t;

typedef struct {
    int32_t max_tiles; /* largest tile list of a training call, 1..4096    */
    float lr;          /* Adam step size (> 0)                              */
    float beta1;       /* Adam moment decay rates, in [0, 1)                */
    float beta2;
    float eps;         /* Adam denominator offset (> 0)                     */
    int32_t reserved[7]; /* must be zero                                    */
} corr_cnn_desc_t;

/* Errors: NULL, INVALID, NOMEM. */
corr_status corr_cnn_create(const corr_cnn_desc_t *desc, corr_cnn_t **out);
void corr_cnn_destroy(corr_cnn_t *cnn);
/* Training scratch: activations and gradients of max_tiles tiles (about
 * 4.4 MB per tile).  Bind 256-byte-aligned device memory of at least this
 * size before the training calls.  Errors: NULL, ALIGN, WORKSPACE. */
size_t corr_cnn_workspace_bytes(const corr_cnn_t *cnn);
corr_status corr_cnn_bind_workspace(corr_cnn_t *cnn, void *d_ws, size_t bytes);

/* FP32 forward pass of the training path: logits [n_tiles][64][256] of the
 * listed tiles of d_power.  Errors: NULL, ALIGN, INVALID, WORKSPACE, DEVICE. */
corr_status corr_cnn_forward(corr_cnn_t *cnn, const float *d_params, const float *d_power, int32_t S, int64_t T,
                             int32_t C, const int32_t *d_tiles, int32_t n_tiles, float *d_logits, void *stream);
/* Mean BCE loss (d_loss, one float) and its gradient (d_grad, CORR_CNN_PARAMS
 * floats; NULL: kept in the workspace) over the listed tiles, labels from
 * d_labels [S][T][C] (0 = clean, nonzero = flagged).  Errors as above. */
corr_status corr_cnn_loss_grad(corr_cnn_t *cnn, const float *d_params, const float *d_power,
                               const uint8_t *d_labels, int32_t S, int64_t T, int32_t C, const int32_t *d_tiles,
                               int32_t n_tiles, float *d_loss, float *d_grad, void *stream);
/* One Adam update of d_params with moments d_m, d_v (CORR_CNN_PARAMS floats
 * each, zero before step 1) at step number `step` >= 1, from d_grad (NULL: the
 * gradient the last corr_cnn_loss_grad kept in the workspace).
 * Errors: NULL, INVALID, WORKSPACE, DEVICE. */
corr_status corr_cnn_adam(corr_cnn_t *cnn, float *d_params, float *d_m, float *d_v, const float *d_grad,
                          int64_t step, void *stream);
/* corr_cnn_loss_grad followed by corr_cnn_adam. */
corr_status corr_cnn_train_step(corr_cnn_t *cnn, float *d_params, float *d_m, float *d_v, int64_t step,
                                const float *d_power, const uint8_t *d_labels, int32_t S, int64_t T, int32_t C,
                                const int32_t *d_tiles, int32_t n_tiles, float *d_loss, void *stream);
/* Synchronise `stream`; CORR_ERR_DEVICE_ARG (and clear it) if a training call
 * saw an out-of-range tile number.  Errors: WORKSPACE, DEVICE. */
corr_status corr_cnn_check_device_errors(corr_cnn_t *cnn, void *stream);

/* Inference over every tile of d_power [S][T][C]: d_flags [S][T][C] uint8
 * (1 = flagged when sigmoid(z3) > threshold, 0 otherwise; ready for
 * corr_apply_flags) and optionally the logits d_logits [S][T][C] (NULL: not
 * written).  FP16 operands with FP32 accumulation on the matrix cores, so the
 * logits differ from the FP32 path by about 1e-3 of their scale.  Needs no
 * handle or workspace.  C is at most 2^22 (offsets inside a tile are 32-bit).
 * Errors: NULL, ALIGN, INVALID (shape, C above 2^22, threshold not in (0, 1)),
 * DEVICE; messages via corr_cnn_last_error(NULL). */
corr_status corr_cnn_infer(const float *d_params, const float *d_power, int32_t S, int64_t T, int32_t C,
                           float threshold, uint8_t *d_flags, float *d_logits, void *stream);
/* The same inference on FP16 power (as corr_fengine writes it with the plan's
 * power_fp16; any scale, the input normalisation divides it out), read as
 * FP16 and widened to FP32 before the normalisation.  2-byte aligned.
 * Errors as corr_cnn_infer. */
corr_status corr_cnn_infer_f16(const float *d_params, const void *d_power16, int32_t S, int64_t T, int32_t C,
                               float threshold, uint8_t *d_flags, float *d_logits, void *stream);
/* Inference with the column guard: a cell is also flagged when its tile
 * column is an outlier of the MAD column statistic (section 5, Eq. 3 and
 * Eq. 4 with M = guard_m on the tile's 256 channel means over its 64 spectra,
 * the means the network's input normalisation already forms).  The guard
 * catches weak persistent tones that the network's 7 x 7 view misses; it
 * leaves the logits unchanged.  guard_m = 0: no guard (corr_cnn_infer /
 * corr_cnn_infer_f16).  power_fp16 selects FP32 or FP16 cells.  Errors as
 * corr_cnn_infer, and INVALID for guard_m < 0 or not finite. */
corr_status corr_cnn_infer_guarded(const float *d_params, const void *d_power, int32_t power_fp16, int32_t S,
                                   int64_t T, int32_t C, float threshold, float guard_m, uint8_t *d_flags,
                                   float *d_logits, void *stream);

/* Save / load parameters and Adam state (each d_* CORR_CNN_PARAMS floats;
 * d_m and d_v may be NULL) to a little-endian binary file: magic "CORRCNN1",
 * int64 step, int32 count, then params, m, v as float32.  Both synchronise the
 * null stream.  Errors: NULL, IO (open / read / write), INVALID (not such a
 * file, or another parameter count), DEVICE (copies). */
corr_status corr_cnn_save(const char *path, const float *d_params, const float *d_m, const float *d_v,
                          int64_t step);
corr_status corr_cnn_load(const char *path, float *d_params, float *d_m, float *d_v, int64_t *step);

/* Last error of the handle (or of handle-free calls when cnn is NULL). */
const char *corr_cnn_last_error(const corr_cnn_t *cnn);

/* ------------------------------------------------------------------ misc */

/* Synchronise `stream` and report (and clear) device-side argument errors:
 * CORR_ERR_DEVICE_ARG if a delay was outside [0, max_delay] (such signals
 * are read with the delay clamped into range).  Errors: WORKSPACE, DEVICE. */
corr_status corr_check_device_errors(corr_plan_t *plan, void *stream);

const char *corr_status_string(corr_status st);
/* Last error message of the plan (or of plan creation when plan is NULL). */
const char *corr_last_error(const corr_plan_t *plan);

#ifdef __cplusplus
}
#endif
#endif /* CORR_H */
