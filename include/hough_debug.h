/*
 * hough_debug.h -- measurement hook exported only by the instrumented build of the library
 * (libhough_phases.so: the same sources compiled with HOUGH_PHASE_TIMING).  The product library
 * libhough.so does not export it.
 *
 * In the instrumented build, thread 0 of every workgroup of hough_run_batch's fused kernel
 * reads the GPU's constant-rate clock (hipDeviceAttributeWallClockRate kHz) after each
 * workgroup barrier and charges the interval to the phase that just ended; at kernel exit the
 * workgroup adds its totals to a device array.  Slots, in order:
 *   0 pop      taking the next event from the work counter
 *   1 setup    an event's keep bytes cleared (and the relative-threshold pass)
 *   2 vote     steps 1-3 of a theta tile (conformal map, theta sweep, votes into LDS)
 *   3 peaks    step 4's 3x3 test into peak bits
 *   4 list     peak listing in raster order and the dilated retention words
 *   5 retain   step 5 of a tile, while the tile is cleared for the next one
 *   6 finish   n_peaks and status of the event
 *   7 events   count of events processed
 *   8 staged   count of valid hits x theta tiles (a staged hit votes all 64 * groups columns)
 * Slots 0-6 are clock ticks summed over workgroups.
 */
#ifndef HOUGH_DEBUG_H
#define HOUGH_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOUGH_PHASE_SLOTS 9

/* Wait for the device, copy the first n (1 .. HOUGH_PHASE_SLOTS) slots to out (host), zero
 * every slot when reset is non-zero, and (clock_khz not NULL) store the clock's rate in kHz.
 * HOUGH_EINVAL for a bad argument, HOUGH_EDEVICE on a HIP failure. */
int hough_debug_phase_ticks(uint64_t *out, int32_t n, int32_t reset, uint32_t *clock_khz);

#ifdef __cplusplus
}
#endif

#endif /* HOUGH_DEBUG_H */
