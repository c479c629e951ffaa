/* swprobe.h -- VALU issue-rate probe of the device (libswprobe.so).
 *
 * Measures how many lane-instructions per second one kind of VALU
 * instruction sustains on a grid that fills the device, so that the peak a
 * roofline divides by can be checked on the machine itself.  Not part of the
 * alignment path. */
#ifndef SWPROBE_H
#define SWPROBE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SW_PROBE_PK_ADD_U16 = 0,   /* v_pk_add_u16: two 16-bit additions per lane-instruction */
    SW_PROBE_PK_MAX3_F16 = 1,  /* v_pk_maximum3_f16: two three-way maxima per lane-instruction */
    SW_PROBE_MAX3_U32 = 2,     /* v_max3_u32 */
    SW_PROBE_ADD_U32 = 3       /* v_add_u32 */
};

/* Launch `blocks` workgroups of 256 threads, each thread running `iters`
 * steps of 8 independent chains of the instruction; the second of two
 * launches is timed with HIP events.  *instr_per_s receives lane-instructions
 * per second.  Returns 0, -1 for bad arguments, -2 if device memory cannot be
 * allocated, -4 on a HIP error. */
int sw_probe_valu(int device, int kind, int iters, int blocks, double* instr_per_s);

#ifdef __cplusplus
}
#endif

#endif /* SWPROBE_H */
