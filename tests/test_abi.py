"""The C ABI without a GPU: the built library loads and exports every function that
include/md.h declares, the ctypes mirrors of the structs match the header's layout, and the
host-side validation behind md_workspace_bytes accepts and rejects what the header says."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "md.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:md_status|const char\*)\s+(md_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def md():
    from paper_1001_3764_amd import md as m
    m.load()
    return m


def test_every_declared_function_is_exported(md):
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(md.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", md.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(names) <= exported


def test_struct_layouts_match_the_header(md, tmp_path):
    """sizeof and offsetof of every field, from a C program compiled against md.h."""
    structs = {"md_forcefield": md.md_forcefield, "md_config": md.md_config, "md_energy": md.md_energy,
               "md_obs_config": md.md_obs_config}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "md.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def config(md, n_chains=(10,), box=((44.376, 44.376, 44.376),), T0=(300.0,), **kw):
    args = dict(chain_len=300, dt=1.0, tau=100.0, precision="mixed", cell_div=1, lj_kernel=1, use_graph=False)
    args.update(kw)
    return md._Config(list(n_chains), np.asarray(box, float), list(T0), args.pop("chain_len"), args.pop("dt"),
                      args.pop("tau"), args.pop("precision"), args.pop("cell_div"), args.pop("lj_kernel"),
                      args.pop("use_graph"), **args)


def workspace(md, ff, cfg):
    n = ctypes.c_size_t()
    st = md.load().md_workspace_bytes(ctypes.byref(md.make_forcefield(ff)), ctypes.byref(cfg.c), ctypes.byref(n))
    return st, n.value


def test_workspace_bytes_and_validation(md, ff):
    st, n = workspace(md, ff, config(md))
    assert st == md.MD_OK and n > 0
    # the workspace grows with the system and with the FP64 payload
    _, n2 = workspace(md, ff, config(md, n_chains=(20,), box=((55.9, 55.9, 55.9),)))
    _, n64 = workspace(md, ff, config(md, precision="fp64"))
    assert n2 > n and n64 > n
    # neighbour-list mode needs the list arrays
    _, nnl = workspace(md, ff, config(md, cell_div=1, lj_kernel=0, nl_skin=1.0, nl_every=10))
    assert nnl > n
    # the half shell needs its int64 accumulators (24 B per atom); cell path only, R <= 2
    st_h, nh = workspace(md, ff, config(md, lj_kernel=md.MD_LJ_HALFSHELL))
    _, ntile = workspace(md, ff, config(md, lj_kernel=md.MD_LJ_CELLTILE))
    assert st_h == md.MD_OK and nh >= ntile + 24 * 3000
    assert workspace(md, ff, config(md, lj_kernel=md.MD_LJ_HALFSHELL, nl_skin=1.0, nl_every=10))[0] == md.MD_ERR_ARG
    assert workspace(md, ff, config(md, lj_kernel=md.MD_LJ_HALFSHELL, cell_div=3))[0] != md.MD_OK
    # both integrators and the COM removal are valid
    for integ in (md.MD_INT_VERLET_BERENDSEN, md.MD_INT_LEAPFROG_NH):
        for com in (False, True):
            assert workspace(md, ff, config(md, integrator=integ, remove_com=com))[0] == md.MD_OK
    bad = [
        dict(integrator=2),
        dict(dt=0.0),
        dict(tau=-1.0),
        dict(chain_len=3, n_chains=(1000,)),
        dict(cell_div=4),
        dict(lj_kernel=4),
        dict(lj_kernel=7),
        dict(nl_skin=-0.5),
        dict(nl_skin=1.0, nl_every=-1),
        dict(T0=(float("nan"),)),
        dict(box=((44.376, 0.0, 44.376),)),
    ]
    for kw in bad:
        assert workspace(md, ff, config(md, **kw))[0] == md.MD_ERR_ARG, kw
    # 2^25 atoms is the limit (the LJ candidate list packs sorted indices in 25 bits)
    big = (1 << 25) // 300 + 1
    assert workspace(md, ff, config(md, n_chains=(big,), box=((1000.0, 1000.0, 1000.0),)))[0] == md.MD_ERR_ARG
    assert workspace(md, ff, config(md, n_chains=(big - 1,), box=((1000.0, 1000.0, 1000.0),)))[0] == md.MD_OK
    cfg = config(md)
    cfg.c.remove_com = 2
    assert workspace(md, ff, cfg)[0] == md.MD_ERR_ARG
    # 25 A box: fewer than three cells of edge >= rc per dimension
    assert workspace(md, ff, config(md, n_chains=(1,), box=((25.0, 25.0, 25.0),)))[0] == md.MD_ERR_BOX_TOO_SMALL


def test_fixed_point_range_is_enforced(md, ff):
    """The mixed payload holds coordinates as int32 in 2^-25 A: (R + 2) * edge + skin must stay
    below 63 A (R stencil cells and the list's padding sentinel one edge further).  A 30 A
    cutoff fits at R = 3 (edges of 11.1 A) but not at R = 1 or 2 (33.3 and 16.7 A); a 45 A
    cutoff fits no tile stencil; FP64 has no such limit; the skin counts against it."""
    big = dict(n_chains=(10,), box=((100.0, 100.0, 100.0),))
    ff30 = dict(ff, rc=30.0)
    ff45 = dict(ff, rc=45.0)
    box150 = dict(n_chains=(10,), box=((150.0, 150.0, 150.0),))
    assert workspace(md, ff30, config(md, cell_div=1, **big))[0] == md.MD_ERR_ARG
    assert workspace(md, ff30, config(md, cell_div=2, lj_kernel=2, **big))[0] == md.MD_ERR_ARG
    assert workspace(md, ff30, config(md, cell_div=0, lj_kernel=0, **big))[0] == md.MD_ERR_ARG
    assert workspace(md, ff30, config(md, cell_div=3, lj_kernel=1, **big))[0] == md.MD_OK
    assert workspace(md, ff30, config(md, cell_div=1, precision="fp64", **big))[0] == md.MD_OK
    assert workspace(md, ff45, config(md, cell_div=0, lj_kernel=0, **box150))[0] == md.MD_ERR_ARG
    assert workspace(md, ff45, config(md, cell_div=0, lj_kernel=0, precision="fp64", **box150))[0] == md.MD_OK
    # neighbour lists, R = 1: a 2 A skin gives 14.8 A cells (3 * 14.8 + 2 < 63); a 25 A skin in a
    # 200 A box gives 40 A cells (3 * 40 + 25 >= 63)
    assert workspace(md, ff, config(md, cell_div=1, lj_kernel=0, nl_skin=2.0, nl_every=0))[0] == md.MD_OK
    assert workspace(md, ff, config(md, n_chains=(200,), box=((200.0, 200.0, 200.0),), cell_div=1, lj_kernel=0,
                                    nl_skin=25.0, nl_every=0))[0] == md.MD_ERR_ARG


def test_static_setup_refusals(md, ff):
    """md_init_system_static refuses, before touching the device, a graph, the autotuner and a
    workspace larger than its array (the pointers below are never dereferenced)."""
    lib = md.load()
    fake = ctypes.c_void_p(1 << 20)
    mff = md.make_forcefield(ff)

    def init(cfg):
        ctx = ctypes.c_void_p()
        st = lib.md_init_system_static(ctypes.byref(mff), ctypes.byref(cfg.c), fake, fake, fake, None,
                                       ctypes.byref(ctx))
        assert not ctx.value
        return st

    assert init(config(md, use_graph=True)) == md.MD_ERR_ARG
    assert init(config(md, cell_div=0)) == md.MD_ERR_ARG
    assert init(config(md, lj_kernel=0)) == md.MD_ERR_ARG
    assert init(config(md, dt=0.0)) == md.MD_ERR_ARG
    small = config(md, cell_div=2, lj_kernel=2)
    big = config(md, n_chains=(4000,), box=((327.0, 327.0, 327.0),), cell_div=2, lj_kernel=2)
    assert workspace(md, ff, small)[1] <= md.MD_STATIC_WORKSPACE_BYTES < workspace(md, ff, big)[1]
    assert init(big) == md.MD_ERR_WORKSPACE


def test_status_strings(md):
    lib = md.load()
    for st in (md.MD_OK, md.MD_ERR_ARG, md.MD_ERR_BOX_TOO_SMALL, md.MD_ERR_NONFINITE, md.MD_ERR_WORKSPACE,
               md.MD_ERR_HIP, md.MD_ERR_STATE, md.MD_ERR_NLIST):
        s = lib.md_status_string(st).decode()
        assert s and s != "unknown status"
    assert lib.md_status_string(12345).decode() == "unknown status"
    assert lib.md_last_error(None).decode() == ""


def test_missing_library_fails_loudly(tmp_path):
    """No CPU fallback: a missing library is an error at load time."""
    code = ("import os; os.environ['PAPER_1001_3764_AMD_LIB'] = %r\n"
            "from paper_1001_3764_amd import md\n"
            "try:\n    md.load()\nexcept RuntimeError as e:\n    print('raised', e)\n" % str(tmp_path / "none.so"))
    out = subprocess.run(["python3", "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert "raised" in out.stdout, out.stderr
