"""The C ABI used from plain C99: the header compiles without C++ and a C
program linked against liblbddf.so validates parameter sets and sizes the
caller's buffer (calls that need no GPU)."""
import os
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1109_6672_amd", "liblbddf.so")

PROGRAM = textwrap.dedent(r"""
    #include <stdio.h>
    #include <string.h>
    #include "lbddf.h"

    static lb_params periodic(int nx, int ny, int storage) {
        lb_params p;
        memset(&p, 0, sizeof p);
        p.nx = nx; p.ny = ny; p.storage = storage;
        p.energy = LB_ENERGY_TOTAL; p.heating = 1; p.correction = 1; p.coupled = 1;
        p.collision = LB_COLLIDE_MRT; p.visc = LB_VISC_CONST_TAU; p.rho_extrap = LB_RHO_PRESSURE;
        p.rho0 = 1.0; p.T0 = 1.0; p.R = 1.0 / 3.0; p.b = 3.0; p.Pr = 0.71; p.tau_f = 0.8;
        p.s_q = 1.5; p.tau_rho = 1.0; p.tau_j = 1.0; p.mu_ref = 0.1; p.T_ref = 1.0; p.visc_n = 1.0;
        for (int s = 0; s < 4; ++s) { p.side[s].kind = LB_BC_PERIODIC; p.side[s].T = 1.0; p.side[s].period = 1.0; }
        return p;
    }

    int main(void) {
        lb_params p = periodic(100, 70, LB_STORE_F32);
        lb_params q = periodic(100, 70, LB_STORE_F16);
        lb_params bad = periodic(100, 70, LB_STORE_F32);
        bad.tau_f = 0.5;
        printf("%d %zu %zu %d\n", (int)lb_validate(&p), lb_state_bytes(&p), lb_state_bytes(&q),
               (int)lb_validate(&bad));
        printf("%s\n", lb_last_error());
        return 0;
    }
""")


def test_c99_program_links_and_validates(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.dirname(LIB)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe), f"-L{libdir}", "-llbddf", f"-Wl,-rpath,{libdir}"])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    ok, b32, b16, bad = out[0].split()
    assert int(ok) == 0 and int(bad) == -1
    # 18 planes per buffer, two buffers, pitch rounded up to 64 nodes: the
    # 16-bit layout holds the populations in half the bytes
    assert int(b32) > 2 * 18 * 128 * 70 * 4 and int(b16) < int(b32)
    assert "tau" in out[1]
