"""Host-only checks of the C ABI: the library loads, exports every entry
point declared in include/gfmc.h, gfph.h, gfhy.h and gffo.h, and the binding's struct layouts equal the
C compiler's.  No compute call is made (there may be no GPU)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gfmc.h", "gfph.h", "gfhy.h", "gffo.h")]


def _declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def gfmc():
    from paper_1707_09073_amd import build, gfmc as G
    if not os.path.exists(G.LIB_PATH):
        build.build(force=True)
    return G


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("mc_init", "mc_step", "mc_tally", "poisson_update", "mc_workspace_bytes", "mc_destroy"):
        assert required in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol(gfmc):
    L = C.CDLL(gfmc.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(L, name), name
    assert sorted(gfmc.EXPORTS) == _declared_functions()


def test_struct_layouts_match_the_header(gfmc):
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "gfmc.h"
#include "gfph.h"
#include "gfhy.h"
#include "gffo.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(mc_material), sizeof(mc_config), sizeof(mc_tally_out),
         sizeof(mc_particles_view), offsetof(mc_config, seed));
  printf("%zu %zu %zu %zu\n", offsetof(mc_config, n_cells), offsetof(mc_config, Vds),
         offsetof(mc_tally_out, real), offsetof(mc_tally_out, flags));
  printf("%zu %zu %zu %zu\n", sizeof(mc_observables_out), offsetof(mc_observables_out, drift_velocity_ms),
         offsetof(mc_observables_out, half_se), offsetof(mc_observables_out, steady));
  printf("%zu %zu %zu %zu\n", sizeof(ph_mc_config), offsetof(ph_mc_config, seed), offsetof(ph_mc_config, n_packets),
         sizeof(ph_electrons));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(hy_config), offsetof(hy_config, n_packets), offsetof(hy_config, tol_K),
         sizeof(hy_record), offsetof(hy_record, hot_cell), offsetof(hy_record, packets_dropped));
  printf("%zu %zu %zu\n", sizeof(fo_config), offsetof(fo_config, R_K_m2KW), offsetof(fo_config, rtol));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", exe, src])
        out = subprocess.check_output([exe]).decode().split()
    want = [C.sizeof(gfmc.McMaterial), C.sizeof(gfmc.McConfig), C.sizeof(gfmc.McTallyOut),
            C.sizeof(gfmc.McParticlesView), gfmc.McConfig.seed.offset, gfmc.McConfig.n_cells.offset,
            gfmc.McConfig.Vds.offset, gfmc.McTallyOut.real.offset, gfmc.McTallyOut.flags.offset,
            C.sizeof(gfmc.McObservablesOut), gfmc.McObservablesOut.drift_velocity_ms.offset,
            gfmc.McObservablesOut.half_se.offset, gfmc.McObservablesOut.steady.offset,
            C.sizeof(gfmc.PhMcConfig), gfmc.PhMcConfig.seed.offset, gfmc.PhMcConfig.n_packets.offset,
            C.sizeof(gfmc.PhElectrons),
            C.sizeof(gfmc.HyConfig), gfmc.HyConfig.n_packets.offset, gfmc.HyConfig.tol_K.offset,
            C.sizeof(gfmc.HyRecord), gfmc.HyRecord.hot_cell.offset, gfmc.HyRecord.packets_dropped.offset,
            C.sizeof(gfmc.FoConfig), gfmc.FoConfig.R_K_m2KW.offset, gfmc.FoConfig.rtol.offset]
    assert [int(x) for x in out] == want


def test_workspace_sizing_and_validation_without_gpu(gfmc):
    from paper_1707_09073_amd import workloads as W
    ok = W.device_config(n_particles=200_000)
    assert gfmc.mc_workspace_bytes([ok]) > 200_000 * 28
    bad = dict(ok, capacity=10)
    assert gfmc.mc_workspace_bytes([bad]) == 0
    short = dict(ok, n_bins=100)            # table top 0.1 eV < 3 eV
    assert gfmc.mc_workspace_bytes([short]) == 0
    mixed = [ok, dict(ok, dt_fs=2.0)]       # instances must share the time step
    assert gfmc.mc_workspace_bytes(mixed) == 0
    assert gfmc.mc_workspace_bytes(W.bias_sweep(4, scale=0.1)) > 0


def test_binding_refuses_missing_library(gfmc, monkeypatch, tmp_path):
    monkeypatch.setattr(gfmc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gfmc, "_lib", None)
    with pytest.raises(RuntimeError):
        gfmc.lib()
