"""The C ABI driven from plain C, with no PyTorch in the process (GPU).

A C program -- HIP runtime calls for memory and the stream, the library for
everything else -- creates a simulation from initial fields read from a file,
sets a uniform force, steps, reads the moments back and writes them out.  The
moments must match the FP64 oracle run on the same inputs to the parity bar of
the FP64 path (1e-12 relative on every field), as the Python-driven parity
tests require.  The program is compiled by gcc against include/lbm.h and the
built library; it checks every status and exits non-zero on the first failure.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2302_04741_amd import _lib, workloads

from _parity import oracle_run, rel_err

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"

PROGRAM = r"""
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbm.h"

#define HIP(call)                                                             \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
            return 1;                                                         \
        }                                                                     \
    } while (0)
#define LBM(call)                                                             \
    do {                                                                      \
        lbm_status s_ = (call);                                               \
        if (s_ != LBM_OK) {                                                   \
            fprintf(stderr, "%s: %d %s\n", #call, (int)s_, lbm_last_error()); \
            return 1;                                                         \
        }                                                                     \
    } while (0)

/* usage: lattice storage nx ny nz tau_hat gx gy gz steps in.bin out.bin
   in.bin / out.bin: float64 rho[N], u[D*N], theta[N] */
int main(int argc, char **argv)
{
    if (argc != 13) {
        fprintf(stderr, "expected 12 arguments\n");
        return 2;
    }
    lbm_params p = {0};
    p.struct_size = sizeof p;
    p.lattice = atoi(argv[1]);
    p.storage = atoi(argv[2]);
    p.nx = atoll(argv[3]);
    p.ny = atoll(argv[4]);
    p.nz = atoll(argv[5]);
    p.tau_hat = atof(argv[6]);
    p.eq_order = 0;
    p.force_order = LBM_FORCE_N2;
    p.rho0 = 1.0;
    const double g[3] = {atof(argv[7]), atof(argv[8]), atof(argv[9])};
    const long long steps = atoll(argv[10]);
    const int D = p.lattice == LBM_D2Q37 ? 2 : 3;
    const size_t N = (size_t)(p.nx * p.ny * p.nz), count = (size_t)(D + 2) * N;

    double *host = malloc(count * sizeof(double));
    FILE *fi = fopen(argv[11], "rb");
    if (!host || !fi || fread(host, sizeof(double), count, fi) != count) {
        fprintf(stderr, "cannot read %s\n", argv[11]);
        return 1;
    }
    fclose(fi);

    const size_t bytes = lbm_workspace_bytes(&p);
    if (bytes == 0) {
        fprintf(stderr, "invalid parameters: %s\n", lbm_last_error());
        return 1;
    }
    hipStream_t stream;
    void *ws;
    double *fin, *fout;
    HIP(hipSetDevice(0));
    HIP(hipStreamCreate(&stream));
    HIP(hipMalloc(&ws, bytes));
    HIP(hipMalloc((void **)&fin, count * sizeof(double)));
    HIP(hipMalloc((void **)&fout, count * sizeof(double)));
    HIP(hipMemcpy(fin, host, count * sizeof(double), hipMemcpyHostToDevice));

    lbm_sim *s = NULL;
    LBM(lbm_create(&p, ws, bytes, stream, fin, fin + N, fin + (size_t)(D + 1) * N, &s));
    LBM(lbm_set_force(s, LBM_G_UNIFORM, g, 0, 0));
    LBM(lbm_step(s, steps));
    LBM(lbm_moments(s, fout, fout + N, fout + (size_t)(D + 1) * N));
    HIP(hipStreamSynchronize(stream));
    if (lbm_step_count(s) != steps) {
        fprintf(stderr, "step count %lld\n", (long long)lbm_step_count(s));
        return 1;
    }
    HIP(hipMemcpy(host, fout, count * sizeof(double), hipMemcpyDeviceToHost));
    lbm_destroy(s);
    HIP(hipFree(fout));
    HIP(hipFree(fin));
    HIP(hipFree(ws));
    HIP(hipStreamDestroy(stream));

    FILE *fo = fopen(argv[12], "wb");
    if (!fo || fwrite(host, sizeof(double), count, fo) != count) {
        fprintf(stderr, "cannot write %s\n", argv[12]);
        return 1;
    }
    fclose(fo);
    free(host);
    puts("c driver: done");
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("c_driver")
    src = d / "lbm_c_driver.c"
    src.write_text(PROGRAM)
    exe = d / "lbm_c_driver"
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=gnu11", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + ROCM + "/include", str(src),
           "-o", str(exe), "-L" + libdir, "-Wl,-rpath," + libdir,
           "-l:" + os.path.basename(_lib.LIB_PATH), "-L" + ROCM + "/lib",
           "-Wl,-rpath," + ROCM + "/lib", "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("lattice,dims,seed", [("D2Q37", (24, 20, 1), 11),
                                               ("D3Q39", (10, 7, 6), 12)])
def test_c_program_matches_the_oracle(driver, tmp_path, oracle_mod, lattice, dims, seed):
    wl = workloads.random_smooth(lattice, dims, seed=seed, tau_hat=0.8, g_amp=1e-4)
    assert wl.force[0] == "uniform"
    g = list(np.asarray(wl.force[1], np.float64)) + [0.0] * (3 - wl.D)
    steps = 20
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([wl.rho, wl.u.reshape(-1), wl.theta]).astype(np.float64).tofile(fin)
    args = [str(driver), str(_lib.LATTICES[lattice]), str(_lib.STORAGES["f64"])] + \
        [str(d) for d in wl.dims] + [repr(wl.tau_hat)] + [repr(float(v)) for v in g[:3]] + \
        [str(steps), str(fin), str(fout)]
    print("c driver:", lattice, wl.dims, "seed", seed, flush=True)
    run = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    out = np.fromfile(fout, dtype=np.float64)
    N, D = wl.ncell, wl.D
    gpu = (out[:N], out[N:(D + 1) * N].reshape(D, N), out[(D + 1) * N:])

    ora = oracle_run(oracle_mod, wl, steps).moments()
    errs = rel_err(gpu, ora)
    assert max(errs) <= 1e-12, errs
