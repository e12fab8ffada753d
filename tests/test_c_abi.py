"""The boundary from C: a C99 program built against include/tpfa.h and
linked to libtpfa.so calls the entry points that need no GPU (version, launch
resolution, argument validation, error strings) and checks what they return.
No Python binding and no torch are involved."""
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
    assert out[0] == "version 20000 rc 0 tile 64x8 kz 32 flags 0 rows 0 512", out
    assert out[1].startswith(f"mu0 {L.TPFA_ERR_PARAM} ") and "mu" in out[1], out
    assert out[2] == f"ldx {L.TPFA_ERR_SHAPE}", out
