"""The boundary as a C caller sees it (no GPU needed): include/grmhd.h
compiles as C99 with warnings as errors, a C program links every declared
function against the built libgrmhd.so, sees the struct sizes the library
was built with, and gets EINVAL with a message for a bad descriptor before
any device call."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1810_04597_amd")


def _declared():
    with open(os.path.join(ROOT, "include", "grmhd.h")) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    return sorted(set(re.findall(r"\b(grmhd_[a-z0-9_]+)\s*\(", text)))


PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "grmhd.h"

int main(void) {
  void* fns[] = {%(fns)s};
  grmhd_grid_desc d;
  grmhd_grid* h = NULL;
  int rc;
  size_t i;
  for (i = 0; i < sizeof(fns) / sizeof(fns[0]); ++i)
    if (!fns[i]) return 10;
  printf("%%zu %%zu %%zu\n", sizeof(grmhd_grid_desc), sizeof(grmhd_diag), sizeof(grmhd_profile));
  memset(&d, 0, sizeof(d));
  for (i = 0; i < 3; ++i) {
    d.n[i] = 8;
    d.dx[i] = 0.125;
  }
  d.gamma_ad = 4.0 / 3.0;
  d.cfl = 0.4;
  d.newton_maxit = 50;
  d.newton_tol = 1e-14;
  d.ng = 3;                  /* the only bad field */
  rc = grmhd_init_grid(&d, NULL, &h);
  printf("%%d %%d %%s\n", rc == GRMHD_EINVAL, h == NULL, grmhd_last_error());
  return 0;
}
"""


def test_header_is_c_and_links():
    cc = shutil.which("gcc") or pytest.skip("no C compiler")
    lib = os.path.join(LIBDIR, "libgrmhd.so")
    if not os.path.exists(lib):
        pytest.fail("libgrmhd.so is not built (run __graft_entry__.build())")
    work = os.path.join(ROOT, "paper_1810_04597_amd", "_build")
    os.makedirs(work, exist_ok=True)
    src = os.path.join(work, "abi_c_check.c")
    exe = os.path.join(work, "abi_c_check")
    fns = ", ".join("(void*)&%s" % n for n in _declared())
    with open(src, "w") as f:
        f.write(PROGRAM % {"fns": fns})
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-Wno-pedantic",
                        "-I", os.path.join(ROOT, "include"), src, "-o", exe,
                        "-L", LIBDIR, "-lgrmhd", "-Wl,-rpath," + LIBDIR,
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = os.pathsep.join([LIBDIR, "/opt/rocm/lib", env.get("LD_LIBRARY_PATH", "")])
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=60)
    assert out.returncode == 0, (out.returncode, out.stderr)
    sizes, refusal = out.stdout.strip().splitlines()[:2]
    assert sizes.split() == ["184", "280", "272"]
    ok, null, msg = refusal.split(" ", 2)
    assert ok == "1" and null == "1" and "ng must be 4, 5 or 6" in msg
