// rr_internal.h -- hooks between the host-side translation units of the
// library (not exported: hidden visibility).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/rrmhd.h"

#define RR_HIDDEN __attribute__((visibility("hidden")))

extern "C" {
// single domain: geometry, storage, stream and whether a state is present
RR_HIDDEN int rr_handle_info(const rrmhd *h, int *nx, int *ny, int *storage,
                             hipStream_t *stream, int *ready);
RR_HIDDEN void rr_handle_set_ready(rrmhd *h, int ready);
// 1 when the handle has walls (the paired FP16 update is periodic only)
RR_HIDDEN int rr_handle_walls(const rrmhd *h);
// 1 when the handle streams in place in one population buffer
RR_HIDDEN int rr_handle_inplace(const rrmhd *h);
// 1 when the handle keeps its planes row-interleaved
RR_HIDDEN int rr_handle_rows(const rrmhd *h);
}
// record the HIP message of a device error for rrmhd_last_error_detail and
// map it to RRMHD_ENOMEM or RRMHD_EDEVICE
RR_HIDDEN int rr_device_error(hipError_t e, const char *what);
// Checkpoint files (synchronous, through one plane of host memory):
// write a header and `planes` planes of `row` bytes taken from device memory
// at base + p * pitch (with nrows > 1: as nrows rows of row / nrows bytes,
// rstride bytes apart); open a file and read its header; after the caller has
// checked the header, check the file size and read the planes back
// (*touched: some device memory was written before a failure); record a
// header mismatch (RRMHD_EINVAL, the field named in the error detail).
RR_HIDDEN int rr_ck_write(const char *path, const void *hdr, size_t hdr_bytes, const char *base,
                          size_t pitch, size_t row, int planes, size_t rstride = 0,
                          int nrows = 1);
RR_HIDDEN int rr_ck_open(const char *path, void *hdr, size_t hdr_bytes, FILE **f);
RR_HIDDEN int rr_ck_read_planes(FILE *f, const char *path, size_t hdr_bytes, char *base,
                                size_t pitch, size_t row, int planes, bool *touched,
                                size_t rstride = 0, int nrows = 1);
RR_HIDDEN int rr_ck_mismatch(const char *field);
extern "C" {
// batch: domain sizes (arrays may be NULL to query n and storage)
RR_HIDDEN int rr_batch_domains(const rrmhd_batch *b, int *n, int *storage, int *nx,
                               int *ny);
// batch: copy of the whole current state / restore it (frees the copy)
RR_HIDDEN int rr_batch_save(rrmhd_batch *b, void **copy);
RR_HIDDEN int rr_batch_restore(rrmhd_batch *b, void *copy, int64_t steps);
RR_HIDDEN hipStream_t rr_batch_stream(const rrmhd_batch *b);
}

namespace rr {
struct Domain;
}
extern "C" RR_HIDDEN int rr_launch_current_vorticity(int storage, const rr::Domain *D,
                                                     const void *src, double omega_m,
                                                     double *jz, double *wz, double *upl,
                                                     hipStream_t st, int swapped);
extern "C" RR_HIDDEN int rr_launch_impose_fluid(int storage, const rr::Domain *D, void *dst,
                                                const double *rho, const double *j,
                                                const double *b, hipStream_t st);
