/* Host-side checks of the library's argument validation under AddressSanitizer
 * (the library's host code is built with -fsanitize=address; no GPU is used:
 * every call here returns before any device work).  Prints one line per check
 * and "all host checks ran"; ASan aborts the process on a memory error. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pic.h"
#include "pic2d.h"

#ifdef WITH_GPU
#include <hip/hip_runtime_api.h>
#endif

static int fails = 0;

static void expect(const char* what, pic_status got, pic_status want) {
  const char* msg = got != PIC_OK ? pic_last_error() : "";
  printf("%-44s %3d (want %3d) %s\n", what, (int)got, (int)want, msg ? msg : "(null)");
  if (got != want || (got != PIC_OK && (!msg || !msg[0]))) ++fails;
}

static pic_config c1(void) {
  pic_config c;
  memset(&c, 0, sizeof c);
  c.struct_size = sizeof c;
  c.precision = PIC_FP32;
  c.lambda_um = 0.8;
  c.cells_per_lambda = 100;
  c.ppc = 64;
  c.box_lambda = 20.0;
  c.cfl = 0.5;
  c.pol = PIC_CP;
  c.rr = 1;
  c.a0 = 200.0;
  c.t_rise = 5.0;
  c.t_fall = 5.0;
  c.n0 = 90.0;
  c.x_foil = 8.0;
  c.thickness = 1.0;
  c.mass_ratio = 1836.0;
  c.rr_compensated = 1;
  c.sort_interval = 16;
  c.seed = 1;
  c.jitter = 0.5;
  return c;
}

static pic2d_config d1(void) {
  pic2d_config c;
  memset(&c, 0, sizeof c);
  c.struct_size = sizeof c;
  c.precision = PIC_FP32;
  c.lambda_um = 0.8;
  c.cells_per_lambda = 32;
  c.ppc_x = c.ppc_y = 2;
  c.pol = PIC_LP;
  c.box_x = 10.0;
  c.box_y = 2.0;
  c.cfl = 0.5;
  c.rr = 1;
  c.rr_compensated = 1;
  c.a0 = 100.0;
  c.waist = 0.6;
  c.t_rise = c.t_fall = 3.0;
  c.n0 = 90.0;
  c.x_foil = 4.0;
  c.thickness = 1.0;
  c.mass_ratio = 1836.0;
  c.sort_interval = 16;
  c.seed = 1;
  c.jitter = 0.5;
  return c;
}

#ifdef WITH_GPU
/* Device part: a small run and a batch, with every host buffer allocated at
 * exactly the size the header documents, so that a write past it is caught. */
static void* must(size_t bytes) {
  void* p = calloc(1, bytes ? bytes : 1);
  if (!p) {
    printf("out of host memory\n");
    exit(2);
  }
  return p;
}

static void gpu_checks(void) {
  hipStream_t st;
  if (hipStreamCreate(&st) != hipSuccess) {
    printf("no HIP stream\n");
    ++fails;
    return;
  }
  pic_config c = c1();
  c.ppc = 16;
  c.box_lambda = 6.0;
  c.x_foil = 2.0;
  c.pol = PIC_LP;
  size_t n = 0;
  expect("gpu: workspace", pic_workspace_bytes(&c, &n), PIC_OK);
  void* ws = NULL;
  if (hipMalloc(&ws, n) != hipSuccess) {
    printf("hipMalloc failed\n");
    ++fails;
    return;
  }
  struct pic_run* r = NULL;
  expect("gpu: init", pic_init(&c, ws, n, st, &r), PIC_OK);
  expect("gpu: step 200", pic_step(r, 200, st), PIC_OK);
  pic_diag_out d;
  memset(&d, 0, sizeof d);
  expect("gpu: diag", pic_diag(r, &d, st), PIC_OK);
  pic_info info;
  memset(&info, 0, sizeof info);
  expect("gpu: info", pic_get_info(r, &info), PIC_OK);
  const long long cap = info.capacity, nc = info.n_cells;
  pic_state s;
  memset(&s, 0, sizeof s);
  for (int k = 0; k < 2; ++k) {
    s.sp[k].cell = (int32_t*)must(cap * sizeof(int32_t));
    s.sp[k].off = must(cap * sizeof(float));
    s.sp[k].ux = must(cap * sizeof(float));
    s.sp[k].uy = must(cap * sizeof(float));
    s.sp[k].uz = must(cap * sizeof(float));
    s.sp[k].w = must(cap * sizeof(float));
  }
  s.sp[0].rx = (float*)must(cap * sizeof(float));
  s.sp[0].ry = (float*)must(cap * sizeof(float));
  s.sp[0].rz = (float*)must(cap * sizeof(float));
  s.Ex = must((nc + 2) * sizeof(float));
  s.Ey = must((nc + 1) * sizeof(float));
  s.Ez = must((nc + 1) * sizeof(float));
  s.By = must((nc + 2) * sizeof(float));
  s.Bz = must((nc + 2) * sizeof(float));
  s.Ex_int = (int64_t*)must((nc + 2) * sizeof(int64_t));
  s.Jx_int = (int64_t*)must((nc + 2) * sizeof(int64_t));
  s.Jy_int = (int64_t*)must((nc + 3) * sizeof(int64_t));
  s.Jz_int = (int64_t*)must((nc + 3) * sizeof(int64_t));
  expect("gpu: get_state", pic_get_state(r, &s, st), PIC_OK);
  expect("gpu: set_state", pic_set_state(r, &s, st), PIC_OK);
  expect("gpu: step 16", pic_step(r, 16, st), PIC_OK);
  pic_species_state q;
  memset(&q, 0, sizeof q);
  q.cell = (int32_t*)must(100 * sizeof(int32_t));
  q.off = must(100 * sizeof(float));
  q.ux = must(100 * sizeof(float));
  expect("gpu: get_particles 100", pic_get_particles(r, 0, 0, 100, &q, st), PIC_OK);
  double* hist = (double*)must(64 * sizeof(double));
  expect("gpu: spectrum 64 bins", pic_spectrum(r, 64, 100.0, hist, st), PIC_OK);
  expect("gpu: spectrum, static 64 bins", pic_spectrum_static(r, 64, 100.0, hist, st), PIC_OK);

  /* a 2D run: state I/O at the documented sizes */
  {
    pic2d_config c2 = d1();
    size_t n2 = 0;
    expect("gpu: 2D workspace", pic2d_workspace_bytes(&c2, &n2), PIC_OK);
    void* ws2 = NULL;
    if (hipMalloc(&ws2, n2) != hipSuccess) {
      ++fails;
      return;
    }
    struct pic2d_run* r2 = NULL;
    expect("gpu: 2D init", pic2d_init(&c2, ws2, n2, st, &r2), PIC_OK);
    expect("gpu: 2D step 64", pic2d_step(r2, 64, st), PIC_OK);
    pic2d_info i2;
    memset(&i2, 0, sizeof i2);
    expect("gpu: 2D info", pic2d_get_info(r2, &i2), PIC_OK);
    const long long cap2 = i2.capacity, nx = i2.nx, ny = i2.ny;
    pic2d_state s2;
    memset(&s2, 0, sizeof s2);
    for (int k = 0; k < 2; ++k) {
      s2.sp[k].cell = (int32_t*)must(cap2 * sizeof(int32_t));
      s2.sp[k].ox = must(cap2 * sizeof(float));
      s2.sp[k].oy = must(cap2 * sizeof(float));
      s2.sp[k].ux = must(cap2 * sizeof(float));
      s2.sp[k].uy = must(cap2 * sizeof(float));
      s2.sp[k].uz = must(cap2 * sizeof(float));
      s2.sp[k].w = must(cap2 * sizeof(float));
    }
    s2.sp[0].rx = (float*)must(cap2 * sizeof(float));
    s2.sp[0].ry = (float*)must(cap2 * sizeof(float));
    s2.sp[0].rz = (float*)must(cap2 * sizeof(float));
    s2.Ex = must((nx + 2) * ny * sizeof(float));
    s2.Ey = must((nx + 1) * ny * sizeof(float));
    s2.Ez = must((nx + 1) * ny * sizeof(float));
    s2.Bx = must((nx + 1) * ny * sizeof(float));
    s2.By = must((nx + 2) * ny * sizeof(float));
    s2.Bz = must((nx + 2) * ny * sizeof(float));
    s2.Jx_int = (int64_t*)must((nx + 2) * ny * sizeof(int64_t));
    s2.Jy_int = (int64_t*)must((nx + 3) * ny * sizeof(int64_t));
    s2.Jz_int = (int64_t*)must((nx + 3) * ny * sizeof(int64_t));
    s2.charge_int = (int64_t*)must((nx + 1) * ny * sizeof(int64_t));
    expect("gpu: 2D get_state", pic2d_get_state(r2, &s2, st), PIC_OK);
    expect("gpu: 2D set_state", pic2d_set_state(r2, &s2, st), PIC_OK);
    expect("gpu: 2D step 8", pic2d_step(r2, 8, st), PIC_OK);
    pic_diag_out d2;
    memset(&d2, 0, sizeof d2);
    expect("gpu: 2D diag", pic2d_diag(r2, &d2, st), PIC_OK);
    pic2d_free(r2);
    (void)hipStreamSynchronize(st);
    (void)hipFree(ws2);
    for (int k = 0; k < 2; ++k) {
      free(s2.sp[k].cell); free(s2.sp[k].ox); free(s2.sp[k].oy); free(s2.sp[k].ux);
      free(s2.sp[k].uy); free(s2.sp[k].uz); free(s2.sp[k].w);
    }
    free(s2.sp[0].rx); free(s2.sp[0].ry); free(s2.sp[0].rz);
    free(s2.Ex); free(s2.Ey); free(s2.Ez); free(s2.Bx); free(s2.By); free(s2.Bz);
    free(s2.Jx_int); free(s2.Jy_int); free(s2.Jz_int); free(s2.charge_int);
  }

  /* a batch of two runs */
  size_t bw = 0;
  expect("gpu: batch workspace", pic_batch_workspace_bytes(PIC_FP32, 3, &bw), PIC_OK);
  void* bws = NULL;
  if (hipMalloc(&bws, bw) != hipSuccess) {
    ++fails;
    return;
  }
  pic_batch* b = NULL;
  expect("gpu: batch create", pic_batch_create(PIC_FP32, 3, 16, 1000000, 100000, bws, bw, st, &b), PIC_OK);
  struct pic_run* br[2] = {NULL, NULL};
  void* bwr[2] = {NULL, NULL};
  int32_t slot[2] = {-1, -1};
  for (int k = 0; k < 2; ++k) {
    pic_config ck = c;
    ck.seed = 7 + k;
    ck.a0 = 150.0 + 50.0 * k;
    if (hipMalloc(&bwr[k], n) != hipSuccess) {
      ++fails;
      return;
    }
    expect("gpu: batch run init", pic_init(&ck, bwr[k], n, st, &br[k]), PIC_OK);
    expect("gpu: admit", pic_batch_admit(b, br[k], 96 + 32 * k, st, &slot[k]), PIC_OK);
  }
  int64_t* steps = (int64_t*)must(3 * sizeof(int64_t));
  expect("gpu: batch step", pic_batch_step(b, 2, st), PIC_OK);
  expect("gpu: batch poll", pic_batch_poll(b, steps, st), PIC_OK);
  expect("gpu: batch poll queued", pic_batch_poll_async(b, st), PIC_OK);
  expect("gpu: batch poll wait", pic_batch_poll_wait(b, steps), PIC_OK);
  int64_t quanta = 0;
  expect("gpu: batch drain", pic_batch_drain(b, &quanta, st), PIC_OK);
  expect("gpu: batch persistent", pic_batch_set_persistent(b, 1), PIC_OK);
  expect("gpu: batch release 0", pic_batch_release(b, slot[0], st), PIC_OK);
  expect("gpu: batch release 1", pic_batch_release(b, slot[1], st), PIC_OK);
  pic_batch_free(b);
  for (int k = 0; k < 2; ++k) {
    expect("gpu: released run diag", pic_diag(br[k], &d, st), PIC_OK);
    pic_free(br[k]);
    (void)hipFree(bwr[k]);
  }
  pic_free(r);
  (void)hipStreamSynchronize(st);
  (void)hipFree(bws);
  (void)hipFree(ws);
  (void)hipStreamDestroy(st);
  for (int k = 0; k < 2; ++k) {
    free(s.sp[k].cell); free(s.sp[k].off); free(s.sp[k].ux); free(s.sp[k].uy); free(s.sp[k].uz);
    free(s.sp[k].w);
  }
  free(s.sp[0].rx); free(s.sp[0].ry); free(s.sp[0].rz);
  free(s.Ex); free(s.Ey); free(s.Ez); free(s.By); free(s.Bz);
  free(s.Ex_int); free(s.Jx_int); free(s.Jy_int); free(s.Jz_int);
  free(q.cell); free(q.off); free(q.ux); free(hist); free(steps);
}
#endif

int main(int argc, char** argv) {
  size_t n = 0;
  pic_config c = c1();
  expect("1D workspace, c1", pic_workspace_bytes(&c, &n), PIC_OK);
  c.precision = PIC_FP64;
  expect("1D workspace, c1 fp64", pic_workspace_bytes(&c, &n), PIC_OK);
  c = c1(); c.struct_size += 8;
  expect("1D struct_size mismatch", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.cfl = 0.6;
  expect("1D cfl above 0.5", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.ppc = 0;
  expect("1D no particles per cell", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.x_foil = 99.0;
  expect("1D foil outside the box", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.cells_per_lambda = 2;
  expect("1D too few cells per wavelength", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.jitter = 2.0;
  expect("1D jitter above 1", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.pol = 7;
  expect("1D unknown polarisation", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.precision = 3;
  expect("1D unknown precision", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.capacity = -5;
  expect("1D negative capacity", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.sort_interval = 0;
  expect("1D sort interval 0", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1(); c.ppc = 2000000000; c.thickness = 20.0; c.x_foil = 0.0;
  expect("1D particle count beyond the limits", pic_workspace_bytes(&c, &n), PIC_EINVAL);
  c = c1();
  expect("1D null output", pic_workspace_bytes(&c, NULL), PIC_EINVAL);
  expect("1D null config", pic_workspace_bytes(NULL, &n), PIC_EINVAL);
  struct pic_run* r = NULL;
  expect("1D init without a workspace", pic_init(&c, NULL, 0, NULL, &r), PIC_EINVAL);
  expect("1D step of a null run", pic_step(NULL, 1, NULL), PIC_EINVAL);
  expect("1D diag of a null run", pic_diag(NULL, NULL, NULL), PIC_EINVAL);

  pic2d_config d = d1();
  expect("2D workspace, d1", pic2d_workspace_bytes(&d, &n), PIC_OK);
  d = d1(); d.struct_size -= 4;
  expect("2D struct_size mismatch", pic2d_workspace_bytes(&d, &n), PIC_EINVAL);
  d = d1(); d.box_y = 0.01;
  expect("2D period below two rows", pic2d_workspace_bytes(&d, &n), PIC_EINVAL);
  d = d1(); d.ppc_x = 0;
  expect("2D empty lattice", pic2d_workspace_bytes(&d, &n), PIC_EINVAL);
  d = d1(); d.capacity = -1;
  expect("2D negative capacity", pic2d_workspace_bytes(&d, &n), PIC_EINVAL);
  expect("2D null config", pic2d_workspace_bytes(NULL, &n), PIC_EINVAL);
  d = d1(); d.field_kernel = 9;
  expect("2D unknown field kernel", pic2d_workspace_bytes(&d, &n), PIC_EINVAL);

  expect("batch workspace, 64 slots", pic_batch_workspace_bytes(PIC_FP32, 64, &n), PIC_OK);
  expect("batch workspace, 0 slots", pic_batch_workspace_bytes(PIC_FP32, 0, &n), PIC_EINVAL);
  expect("batch workspace, 100000 slots", pic_batch_workspace_bytes(PIC_FP32, 100000, &n), PIC_EINVAL);
  expect("batch workspace, bad precision", pic_batch_workspace_bytes(9, 4, &n), PIC_EINVAL);
  expect("rounding check without outputs", pic_check_rounding(0x3F800000u, 16, NULL, NULL), PIC_EINVAL);
#ifdef WITH_GPU
  if (argc > 1 && strcmp(argv[1], "--gpu") == 0) gpu_checks();
#else
  (void)argc;
  (void)argv;
#endif
  printf("all host checks ran: %d failed\n", fails);
  return fails ? 1 : 0;
}
