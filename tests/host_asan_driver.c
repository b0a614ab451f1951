/* Host-side checks of the library's argument validation under AddressSanitizer
 * (the library's host code is built with -fsanitize=address; no GPU is used:
 * every call here returns before any device work).  Prints one line per check
 * and "all host checks ran"; ASan aborts the process on a memory error. */
#include <stdio.h>
#include <string.h>

#include "pic.h"
#include "pic2d.h"

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

int main(void) {
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
  printf("all host checks ran: %d failed\n", fails);
  return fails ? 1 : 0;
}
