// client.cpp: a native client of libtwofold.so through include/twofold.h
// alone (no Python, no torch): device memory from hipMalloc, one stream,
// the single-vector, multi-vector, segmented-plan and monitor entry points.
// Prints one
// "name status value error" line per result, values as C99 hex floats, for
// tests/test_gpu_c_client.py to check against exact rational sums.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "twofold.h"

#define HIP_OK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));          \
      exit(2);                                                                    \
    }                                                                             \
  } while (0)

static const int64_t kN = 1000003;

int main(void) {
  // x_i = 1 + (i mod 1000) * 2^-40 (rounds when summed), y_i = ((7 i) mod 201 - 100) / 32
  double* hx = (double*)malloc(sizeof(double) * kN);
  double* hy = (double*)malloc(sizeof(double) * kN);
  float* hf = (float*)malloc(sizeof(float) * kN);
  for (int64_t i = 0; i < kN; i++) {
    hx[i] = 1.0 + (double)(i % 1000) * 0x1p-40;
    hy[i] = (double)((7 * i) % 201 - 100) / 32.0;
    hf[i] = (float)(1.0 + (double)(i % 1000) * 0x1p-20);
  }
  hipStream_t st;
  HIP_OK(hipStreamCreate(&st));
  double *x, *y;
  float* xf;
  twofold_f64_t* out64;
  twofold_f32_t* out32;
  HIP_OK(hipMalloc((void**)&x, sizeof(double) * kN));
  HIP_OK(hipMalloc((void**)&y, sizeof(double) * kN));
  HIP_OK(hipMalloc((void**)&xf, sizeof(float) * kN));
  HIP_OK(hipMalloc((void**)&out64, sizeof(twofold_f64_t) * 8));
  HIP_OK(hipMalloc((void**)&out32, sizeof(twofold_f32_t) * 2));
  HIP_OK(hipMemcpy(x, hx, sizeof(double) * kN, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(y, hy, sizeof(double) * kN, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(xf, hf, sizeof(float) * kN, hipMemcpyHostToDevice));

  size_t wsb = twofold_workspace_bytes_single(8, 1, TWOFOLD_RIGOROUS, kN, NULL);
  size_t w2 = twofold_workspace_bytes_single(8, 0, TWOFOLD_RIGOROUS, kN, NULL);
  size_t w3 = twofold_workspace_bytes_single(4, 0, TWOFOLD_RIGOROUS, kN, NULL);
  if (w2 > wsb) wsb = w2;
  if (w3 > wsb) wsb = w3;
  void* ws;
  HIP_OK(hipMalloc(&ws, wsb));

  int rc[6];
  rc[0] = twofold_sum_f64(x, kN, TWOFOLD_RIGOROUS, NULL, &out64[0], ws, wsb, st);
  rc[1] = twofold_sum_f64(x, kN, TWOFOLD_PLAIN, NULL, &out64[1], ws, wsb, st);
  rc[2] = twofold_dot_f64(x, y, kN, TWOFOLD_RIGOROUS, NULL, &out64[2], ws, wsb, st);
  rc[3] = twofold_sum_f32(xf, kN, TWOFOLD_FAST, NULL, &out32[0], ws, wsb, st);

  // a segmented plan over four segments (one empty), dots
  const int64_t off_h[5] = {0, 10, 10, 1000, kN};
  twofold_seg_plan_t* plan = NULL;
  rc[4] = twofold_seg_plan_create(off_h, 4, 8, 1, TWOFOLD_RIGOROUS, NULL, &plan);
  void* pws = NULL;
  size_t pwsb = 0;
  if (rc[4] == TWOFOLD_OK) {
    pwsb = twofold_seg_plan_workspace_bytes(plan);
    HIP_OK(hipMalloc(&pws, pwsb));
    rc[4] = twofold_seg_plan_execute(plan, x, y, &out64[3], pws, pwsb, st);
  }
  // the precision monitor over the four segment results
  int64_t* doff;
  uint32_t* flags;
  int64_t* nflag;
  HIP_OK(hipMalloc((void**)&doff, sizeof(off_h)));
  HIP_OK(hipMalloc((void**)&flags, 4 * sizeof(uint32_t)));
  HIP_OK(hipMalloc((void**)&nflag, sizeof(int64_t)));
  HIP_OK(hipMemcpy(doff, off_h, sizeof(off_h), hipMemcpyHostToDevice));
  rc[5] = twofold_monitor(8, &out64[3], 4, doff, 0, 0.0, flags, nflag, st);

  // three dots in one multi-vector call: the whole pair, the pair from
  // element 1 on (both 8 bytes past a 16-byte line) and its first 1000
  // elements
  const double* mx[3] = {x, x + 1, x};
  const double* my[3] = {y, y + 1, y};
  const int64_t mn[3] = {kN, kN - 1, 1000};
  size_t mwsb = twofold_workspace_bytes_multi(8, 1, TWOFOLD_RIGOROUS, mn, 3, NULL);
  void* mws;
  twofold_f64_t* outm;
  HIP_OK(hipMalloc(&mws, mwsb));
  HIP_OK(hipMalloc((void**)&outm, sizeof(twofold_f64_t) * 3));
  const int rcm = twofold_multidot_f64(mx, my, mn, 3, TWOFOLD_RIGOROUS, NULL, outm, mws, mwsb, st);

  // binary64 results: the mixed-form dot of xf with itself, and double-word
  // sums of x and of x from element 1 on in one multi-vector call
  const double* wx[2] = {x, x + 1};
  const int64_t wn[2] = {kN, kN - 1};
  size_t xwsb = twofold_workspace_bytes_single(4, 1, TWOFOLD_MIXED, kN, NULL);
  size_t w4 = twofold_workspace_bytes_multi(8, 0, TWOFOLD_WIDE, wn, 2, NULL);
  if (w4 > xwsb) xwsb = w4;
  void* xws;
  twofold_f64_t* outw;
  HIP_OK(hipMalloc(&xws, xwsb));
  HIP_OK(hipMalloc((void**)&outw, sizeof(twofold_f64_t) * 3));
  const int rcx = twofold_dot_mixed_f32(xf, xf, kN, NULL, &outw[0], xws, xwsb, st);
  // the same workspace: calls on one stream run in order
  const int rcw = twofold_multisumd_f64(wx, wn, 2, NULL, &outw[1], xws, xwsb, st);

  // a mixed batch: the binary64 dot and the binary32 fast sum in one launch
  twofold_f64_t* outb64;
  twofold_f32_t* outb32;
  HIP_OK(hipMalloc((void**)&outb64, sizeof(twofold_f64_t)));
  HIP_OK(hipMalloc((void**)&outb32, sizeof(twofold_f32_t)));
  twofold_batch_item_t bi[2] = {{x, y, outb64, kN, 8, 1, TWOFOLD_RIGOROUS, 0},
                                {xf, NULL, outb32, kN, 4, 0, TWOFOLD_FAST, 0}};
  size_t bwsb = twofold_workspace_bytes_batch(bi, 2, NULL);
  void* bws;
  HIP_OK(hipMalloc(&bws, bwsb));
  const int rcb = twofold_batch(bi, 2, NULL, bws, bwsb, st);
  HIP_OK(hipStreamSynchronize(st));

  twofold_f64_t r64[8];
  twofold_f32_t r32[2];
  uint32_t hflags[4];
  int64_t hn;
  HIP_OK(hipMemcpy(r64, out64, sizeof(r64), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(r32, out32, sizeof(r32), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&hn, nflag, sizeof(hn), hipMemcpyDeviceToHost));

  printf("sum_f64_rigorous %d %a %a\n", rc[0], r64[0].value, r64[0].error);
  printf("sum_f64_plain %d %a %a\n", rc[1], r64[1].value, r64[1].error);
  printf("dot_f64_rigorous %d %a %a\n", rc[2], r64[2].value, r64[2].error);
  printf("sum_f32_fast %d %a %a\n", rc[3], (double)r32[0].value, (double)r32[0].error);
  for (int s = 0; s < 4; s++)
    printf("segdot_f64_rigorous_%d %d %a %a\n", s, rc[4], r64[3 + s].value, r64[3 + s].error);
  printf("monitor %d %u %u %u %u %lld\n", rc[5], hflags[0], hflags[1], hflags[2], hflags[3],
         (long long)hn);
  twofold_f64_t rm[3];
  HIP_OK(hipMemcpy(rm, outm, sizeof(rm), hipMemcpyDeviceToHost));
  for (int v = 0; v < 3; v++)
    printf("multidot_f64_rigorous_%d %d %a %a\n", v, rcm, rm[v].value, rm[v].error);
  twofold_f64_t rw[3];
  HIP_OK(hipMemcpy(rw, outw, sizeof(rw), hipMemcpyDeviceToHost));
  printf("dot_mixed_f32 %d %a %a\n", rcx, rw[0].value, rw[0].error);
  for (int v = 0; v < 2; v++)
    printf("multisumd_f64_%d %d %a %a\n", v, rcw, rw[1 + v].value, rw[1 + v].error);
  twofold_f64_t rb64;
  twofold_f32_t rb32;
  HIP_OK(hipMemcpy(&rb64, outb64, sizeof(rb64), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&rb32, outb32, sizeof(rb32), hipMemcpyDeviceToHost));
  printf("batch_dot_f64_rigorous %d %a %a\n", rcb, rb64.value, rb64.error);
  printf("batch_sum_f32_fast %d %a %a\n", rcb, (double)rb32.value, (double)rb32.error);

  HIP_OK(hipFree(x));
  HIP_OK(hipFree(y));
  HIP_OK(hipFree(xf));
  HIP_OK(hipFree(out64));
  HIP_OK(hipFree(out32));
  HIP_OK(hipFree(ws));
  if (pws) HIP_OK(hipFree(pws));
  HIP_OK(hipFree(doff));
  HIP_OK(hipFree(flags));
  HIP_OK(hipFree(nflag));
  HIP_OK(hipFree(mws));
  HIP_OK(hipFree(outm));
  HIP_OK(hipFree(xws));
  HIP_OK(hipFree(outb64));
  HIP_OK(hipFree(outb32));
  HIP_OK(hipFree(bws));
  HIP_OK(hipFree(outw));
  if (plan) twofold_seg_plan_destroy(plan);
  HIP_OK(hipStreamDestroy(st));
  free(hx);
  free(hy);
  free(hf);
  return 0;
}
