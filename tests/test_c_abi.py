"""The boundary from C: a C99 program built against include/tpfa.h and
linked to libtpfa.so calls the entry points that need no GPU (version, launch
resolution, argument validation, error strings) and checks what they return;
on the GPU, a C program allocates device memory with hipMalloc, calls
tpfa_jacobian and its outputs meet the oracle bound. No Python binding and no
torch are involved in either program."""
import os
import shutil
import subprocess

import pytest

from paper_2304_11274_amd import _lib as L

ROOT = os.path.join(os.path.dirname(__file__), "..")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "tpfa.h"

int main(void) {
  tpfa_grid_t g = {512, 512, 256, 10.0, 10.0, 2.0, 9.81, 0};
  tpfa_rock_t rock;
  memset(&rock, 0, sizeof rock);
  rock.kx = (const void *)&g; /* only presence is read */
  rock.ry = 1.0;
  rock.rz = 0.1;
  tpfa_launch_t out;
  int rc = tpfa_resolve_launch(&g, TPFA_OP_JACOBIAN, TPFA_FP64, &rock, NULL, &out);
  int tx = 0, ty = 0, th = 0;
  tpfa_tile_shape(out.tile, &tx, &ty, &th);
  printf("version %d rc %d tile %dx%d kz %d flags %d rows %lld %lld\n", tpfa_version(), rc, tx,
         ty, out.kz_chunk, out.flags, (long long)out.y_begin, (long long)out.y_end);
  /* argument errors are found on the host, before anything is enqueued */
  tpfa_fluid_t f = {1000.0, 1e-9, 1e7, 0.0};
  tpfa_state_t st = {(const void *)&g, NULL};
  rc = tpfa_residual(&g, &f, &rock, &st, TPFA_FP64, (void *)&g, NULL, NULL);
  printf("mu0 %d %s | %s\n", rc, tpfa_strerror(rc), tpfa_last_error());
  g.ldx = 100;
  rc = tpfa_resolve_launch(&g, TPFA_OP_JACOBIAN, TPFA_FP64, &rock, NULL, &out);
  printf("ldx %d\n", rc);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not available")
def test_c_program_against_the_header(tmp_path):
    L.load()  # builds nothing; fails loudly if the library is missing
    lib_dir = os.path.dirname(L.LIB_PATH)
    src = tmp_path / "use_tpfa.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_tpfa"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", lib_dir,
                    "-l:libtpfa.so", f"-Wl,-rpath,{lib_dir}"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    assert out[0] == "version 20100 rc 0 tile 64x8 kz 32 flags 0 rows 0 512", out
    assert out[1].startswith(f"mu0 {L.TPFA_ERR_PARAM} ") and "mu" in out[1], out
    assert out[2] == f"ldx {L.TPFA_ERR_SHAPE}", out


GPU_PROGRAM = r"""
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>
#include "tpfa.h"

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { \
  fprintf(stderr, "hip error %d at %d\n", (int)e_, __LINE__); return 2; } } while (0)

/* usage: prog nx ny nz in.bin out.bin; in.bin = p, kx (double), seal (uint8);
   out.bin = r, J[7] (double) */
int main(int argc, char **argv) {
  if (argc != 6) return 3;
  const int64_t nx = atoll(argv[1]), ny = atoll(argv[2]), nz = atoll(argv[3]);
  const size_t n = (size_t)(nx * ny * nz);
  double *h = (double *)malloc(8 * n * 9 + n);
  FILE *fi = fopen(argv[4], "rb");
  if (!h || !fi || fread(h, 1, 16 * n + n, fi) != 16 * n + n) return 4;
  fclose(fi);
  double *dp, *dk, *dr, *dJ;
  uint8_t *ds;
  CK(hipMalloc((void **)&dp, 8 * n));
  CK(hipMalloc((void **)&dk, 8 * n));
  CK(hipMalloc((void **)&ds, n));
  CK(hipMalloc((void **)&dr, 8 * n));
  CK(hipMalloc((void **)&dJ, 56 * n));
  CK(hipMemcpy(dp, h, 8 * n, hipMemcpyHostToDevice));
  CK(hipMemcpy(dk, h + n, 8 * n, hipMemcpyHostToDevice));
  CK(hipMemcpy(ds, (uint8_t *)(h + 2 * n), n, hipMemcpyHostToDevice));
  tpfa_grid_t g = {nx, ny, nz, 10.0, 10.0, 2.0, 9.81, 0};
  tpfa_fluid_t f = {1000.0, 1e-9, 1e7, 1e-3};
  tpfa_rock_t rock = {dk, NULL, NULL, 1.0, 0.1, ds, NULL, NULL, NULL};
  tpfa_state_t st = {dp, NULL};
  int rc = tpfa_jacobian(&g, &f, &rock, &st, TPFA_FP64, dr, dJ, NULL, NULL);
  if (rc) { fprintf(stderr, "tpfa_jacobian: %s\n", tpfa_last_error()); return 5; }
  CK(hipDeviceSynchronize());
  CK(hipMemcpy(h, dr, 8 * n, hipMemcpyDeviceToHost));
  CK(hipMemcpy(h + n, dJ, 56 * n, hipMemcpyDeviceToHost));
  FILE *fo = fopen(argv[5], "wb");
  if (!fo || fwrite(h, 8, 8 * n, fo) != 8 * n) return 6;
  fclose(fo);
  hipFree(dp); hipFree(dk); hipFree(ds); hipFree(dr); hipFree(dJ);
  free(h);
  printf("ok\n");
  return 0;
}
"""


@pytest.mark.gpu
def test_c_program_on_the_gpu(orc, tmp_path):
    """A C program allocates device memory with hipMalloc, calls tpfa_jacobian
    and copies r and J back; they meet the oracle bound (no torch involved)."""
    import numpy as np

    import geomodel
    from helpers import compare_full
    L.load()
    lib_dir = os.path.dirname(L.LIB_PATH)
    src = tmp_path / "use_tpfa_gpu.c"
    src.write_text(GPU_PROGRAM)
    exe = tmp_path / "use_tpfa_gpu"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I",
                    os.path.join(ROOT, "include"), "-I/opt/rocm/include", str(src), "-o", str(exe),
                    "-L", lib_dir, "-l:libtpfa.so", "-L/opt/rocm/lib", "-lamdhip64",
                    f"-Wl,-rpath,{lib_dir}:/opt/rocm/lib"], check=True)
    geo = geomodel.random_small(77, 37, 11, 9, sigma=1.5, seal_prob=0.05)
    g = geo.grid
    p = orc.pressure(geo)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(p, np.float64).tobytes())
        fh.write(np.ascontiguousarray(geo.kx, np.float64).tobytes())
        fh.write(np.ascontiguousarray(geo.seal, np.uint8).tobytes())
    print("C program on the GPU, 37x11x9", flush=True)
    res = subprocess.run([str(exe), str(g.nx), str(g.ny), str(g.nz), str(fin), str(fout)],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip() == "ok", (res.returncode, res.stderr)
    out = np.fromfile(fout, np.float64)
    n = g.nx * g.ny * g.nz
    r, J = out[:n].reshape(g.shape), out[n:].reshape((7,) + g.shape)
    rep = compare_full(orc, g, geo.fluid, geo.kx, p, r, J, tol=1e-12,
                       tau=1e-9 * float(np.abs(p).max()), ry=1.0, rz=0.1, seal=geo.seal)
    assert rep["max_err"] <= 1e-12, rep
