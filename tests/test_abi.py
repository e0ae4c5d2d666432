"""The C-ABI library loads and exports every entry point of include/grpic.h
(no compute calls: runs without a GPU)."""
import ctypes as C
import subprocess

import pytest

import paper_2602_07452_amd as G


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = G.exported_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_config_default():
    cfg = G.config_default()
    assert cfg.tol == 1e-13 and cfg.kmax == 50 and cfg.tile_r == 32 and cfg.tile_th == 16
    assert abs(cfg.theta0 - 3.141592653589793 / 200) < 1e-15


@pytest.mark.parametrize("cls,cname", [(G.Config, "grpic_config"),
                                       (G.InitSpec, "grpic_init_spec"),
                                       (G.Diag, "grpic_diag"),
                                       (G.MlpTrainConfig, "grpic_mlp_train_config"),
                                       (G.TuneResult, "grpic_tune_result"),
                                       (G.StateHeader, "grpic_state_header")])
def test_struct_layout_matches_header(cls, cname, tmp_path):
    """The ctypes mirrors have the C structs' size and field offsets."""
    fields = [f[0] for f in cls._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{G.HEADER}"',
           'int main(void) {', f'printf("%zu\\n", sizeof({cname}));']
    src += [f'printf("%zu\\n", offsetof({cname}, {f}));' for f in fields]
    src += ['return 0; }']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-o", str(exe), str(c)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == C.sizeof(cls)
    assert vals[1:] == [getattr(cls, f).offset for f in fields]


def test_cfl_limit_host_side():
    cfg = G.config_default(a=0.99, nr=64, nth=64, r_in=1.03, r_out=20.0)
    dt = G.cfl_dt(cfg)
    assert 1e-3 < dt < 5e-2
    # refining the grid lowers the limit
    cfg2 = G.config_default(a=0.99, nr=128, nth=128, r_in=1.03, r_out=20.0)
    assert G.cfl_dt(cfg2) < dt


def test_invalid_config_is_rejected_without_gpu():
    cfg = G.config_default(a=1.5)
    with pytest.raises(G.GrpicError):
        G.Context(cfg)


def test_grids_beyond_the_index_limits_are_rejected_without_gpu():
    """Field arrays are indexed with 32-bit byte offsets: (nr + 1)(nth + 1)
    may not exceed 2^30 and neither dimension 2^22 - 2."""
    for nr, nth in ((1 << 22) - 1, 2), (2, (1 << 22) - 1), (1 << 15, 1 << 15):
        cfg = G.config_default(a=0.5, nr=nr, nth=nth, r_in=1.0, r_out=10.0,
                               field_mode=G.FIELDS_STATIC)
        with pytest.raises(G.GrpicError, match="grid too large"):
            G.Context(cfg)


def test_paper_deposit_and_cleaning_need_evolving_fields():
    for kw in (dict(deposit_mode=G.DEPOSIT_PAPER), dict(clean_every=25),
               dict(deposit_mode=7, field_mode=G.FIELDS_EVOLVE)):
        base = dict(a=0.9, nr=16, nth=16, r_in=1.3, r_out=10.0, field_mode=G.FIELDS_STATIC)
        base.update(kw)
        with pytest.raises(G.GrpicError):
            G.Context(G.config_default(**base))


def test_kernel_group_names_match_the_header():
    """The binding sizes the timing buffers by its list of group names."""
    import re
    text = open(G.HEADER).read()
    count = int(re.search(r"GRPIC_K_COUNT\s*=\s*(\d+)", text).group(1))
    assert count == len(G.KERNEL_NAMES)


def test_step_is_marked_with_trace_ranges():
    """The library marks the parts of a step (the sub-steps of Sec. 2.1, the
    sort, cleaning and injection) with roctx ranges for tracing tools: it
    imports the range calls, and the range names are in the library."""
    out = subprocess.run(["nm", "-D", G.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    undefined = {l.split()[-1] for l in out.splitlines() if " U " in l}
    assert {"roctxRangePushA", "roctxRangePop"} <= undefined
    data = open(G.LIB_PATH, "rb").read()
    for name in (b"grpic sub-steps 1-4", b"grpic sub-step 5", b"grpic sub-step 6",
                 b"grpic sub-steps 7-10", b"grpic tile sort"):
        assert name in data
