"""include/lbm.h from plain C (CPU).

A small C99 program, compiled by gcc with -pedantic -Werror against the header
and linked against the built library, makes the host-only calls a C user
starts with: the workspace size, the compiled velocity set, the version, and a
rejected lbm_create (no workspace) with its error message.  None of these calls
reaches the GPU.  Their results must match what the Python binding reports for
the same arguments.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2302_04741_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stdio.h>
#include <string.h>

#include "lbm.h"

int main(void)
{
    lbm_params p;
    int32_t c[39 * 3];
    double w[39], r = 0.0;
    lbm_sim *s = (lbm_sim *)&p; /* lbm_create must clear it on failure */
    lbm_status st;
    size_t ws;
    int32_t q;

    memset(&p, 0, sizeof p);
    p.struct_size = (uint32_t)sizeof p;
    p.lattice = LBM_D3Q39;
    p.storage = LBM_F32;
    p.eq_order = 0;
    p.force_order = LBM_FORCE_N2;
    p.flags = 0;
    p.nx = 256;
    p.ny = 256;
    p.nz = 256;
    p.tau_hat = 0.8;
    p.rho0 = 1.0;

    ws = lbm_workspace_bytes(&p);
    q = lbm_lattice_table(LBM_D3Q39, c, w, &r);
    st = lbm_create(&p, NULL, ws, NULL, NULL, NULL, NULL, &s);
    printf("workspace %zu\n", ws);
    printf("q %d\n", (int)q);
    printf("r %.17g\n", r);
    printf("c1 %d %d %d\n", (int)c[3], (int)c[4], (int)c[5]);
    printf("w0 %.17g\n", w[0]);
    printf("create %d %s\n", (int)st, s == NULL ? "null" : "set");
    printf("error %s\n", lbm_last_error());
    printf("version %s\n", lbm_version());
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_compiles_as_c_and_links(tmp_path):
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2302_04741_amd import build

        build.build()
    src = tmp_path / "use_lbm.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_lbm"
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
           "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe),
           "-L" + libdir, "-Wl,-rpath," + libdir, "-l:" + os.path.basename(_lib.LIB_PATH)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    out = dict(line.split(" ", 1) for line in run.stdout.strip().splitlines())

    L = _lib.load()
    p = _lib.make_params("D3Q39", (256, 256, 256), 0.8, "f32", 0, 4, False, 1.0, False)
    assert int(out["workspace"]) == L.lbm_workspace_bytes(ctypes.byref(p))
    assert int(out["workspace"]) >= 2 * 39 * 4 * 256 ** 3

    c = (ctypes.c_int32 * (39 * 3))()
    w = (ctypes.c_double * 39)()
    rr = ctypes.c_double()
    assert L.lbm_lattice_table(1, c, w, ctypes.byref(rr)) == 39
    assert int(out["q"]) == 39
    assert float(out["r"]) == rr.value
    assert [int(v) for v in out["c1"].split()] == list(c[3:6])
    assert float(out["w0"]) == w[0]

    assert out["create"] == "%d null" % _lib.LBM_EINVAL
    assert "workspace" in out["error"]
    assert out["version"] == L.lbm_version().decode()
