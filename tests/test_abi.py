"""The C ABI library loads, exports every entry point declared in include/sdmm.h, and
rejects bad arguments on the host before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdmm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdmm_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_13094_amd import sdmm
    if not os.path.exists(sdmm.LIB_PATH):
        pytest.fail("libsdmm.so is not built (run __graft_entry__.build())")
    return sdmm.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sdmm_fit_mixtures", "sdmm_condition_prepare", "sdmm_condition", "sdmm_pdf", "sdmm_sample",
              "sdmm_condition_sample_pdf", "sdmm_fit_grad", "sdmm_fit_workspace_size", "sdmm_status_string"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_version(lib):
    assert lib.sdmm_status_string(0) == b"ok"
    assert lib.sdmm_status_string(-3) == b"workspace too small"
    assert lib.sdmm_version().startswith(b"sdmm")


def test_workspace_size_and_argument_errors(lib):
    from paper_2111_13094_amd import sdmm
    o = sdmm.default_opts(16)
    ws = lib.sdmm_fit_workspace_size(4096, 16, 4_000_000, C.byref(o))
    assert ws > 4096 * 16 * 32 * 4
    assert lib.sdmm_fit_workspace_size(0, 16, 10, C.byref(o)) == 0
    assert lib.sdmm_fit_workspace_size(1, 65, 10, C.byref(o)) == 0
    m = sdmm.Mixtures()
    st = sdmm.EmState()
    # null pointers are rejected before any device work
    assert lib.sdmm_fit_mixtures(None, None, 0, C.byref(m), C.byref(st), C.byref(o), None, None, 0, None) == -1
    assert lib.sdmm_condition(None, 1, 16, None, None, 1, None, None, None) == -1
    assert lib.sdmm_condition(C.c_void_p(8), 1, 16, None, None, 0, None, None, None) == 0  # empty
    assert lib.sdmm_pdf(C.c_void_p(8), 1, 65, None, 1, None, None, 1, None, None, None) == -1
    # a workspace below the reported size is refused
    m.n_cells, m.K = 1, 16
    m.weights = m.mean_dir = m.mean_pos = m.cov = C.c_void_p(256)
    st.s0 = st.s2 = st.sw = st.step = C.c_void_p(256)
    need = lib.sdmm_fit_workspace_size(1, 16, 100, C.byref(o))
    rc = lib.sdmm_fit_mixtures(C.c_void_p(256), C.c_void_p(256), 100, C.byref(m), C.byref(st), C.byref(o),
                               C.c_void_p(256), C.c_void_p(256), need - 1, None)
    assert rc == -3
    o.K = 8  # K mismatch between options and mixtures
    assert lib.sdmm_fit_mixtures(C.c_void_p(256), C.c_void_p(256), 100, C.byref(m), C.byref(st), C.byref(o),
                                 C.c_void_p(256), C.c_void_p(256), need, None) == -1
    # the FMA probe refuses other widths, empty launches and null pointers on the host
    ms = C.c_double()
    assert lib.sdmm_probe_fma(16, 1, 1, C.c_void_p(256), C.byref(ms), None) == -1
    assert lib.sdmm_probe_fma(32, 0, 1, C.c_void_p(256), C.byref(ms), None) == -1
    assert lib.sdmm_probe_fma(64, 1, 0, C.c_void_p(256), C.byref(ms), None) == -1
    assert lib.sdmm_probe_fma(32, 1, 1, None, C.byref(ms), None) == -1


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets that a C
    compiler gives the header's structures."""
    import subprocess
    from paper_2111_13094_amd import sdmm
    src = tmp_path / "layout.c"
    fields = [("sdmm_fit_opts", f) for f, _ in sdmm.FitOpts._fields_] + \
             [("sdmm_mixtures", f) for f, _ in sdmm.Mixtures._fields_] + \
             [("sdmm_em_state", f) for f, _ in sdmm.EmState._fields_] + \
             [("sdmm_tree", f) for f, _ in sdmm.Tree._fields_]
    body = "".join(f'printf("%s.%s %zu\\n", offsetof({t}, {f}));\n'.replace("%s.%s", f"{t}.{f}") for t, f in fields)
    body += "".join(f'printf("{t} %zu\\n", sizeof({t}));\n' for t in ("sdmm_fit_opts", "sdmm_mixtures", "sdmm_em_state",
                                                                     "sdmm_tree"))
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "sdmm.h"\nint main(void) {\n' + body + "return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for cls, name in ((sdmm.FitOpts, "sdmm_fit_opts"), (sdmm.Mixtures, "sdmm_mixtures"),
                      (sdmm.EmState, "sdmm_em_state"), (sdmm.Tree, "sdmm_tree")):
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_binding_rejects_undersized_tensors():
    """The C ABI sees bare pointers, so the binding checks every tensor against the size
    its layout needs before anything reaches the library."""
    import torch
    from paper_2111_13094_amd import sdmm
    K, n_cells, nq = 16, 4, 8
    full = n_cells * K * sdmm.COND_TABLE_STRIDE
    qcell = torch.zeros(nq, dtype=torch.int32)
    with pytest.raises(ValueError, match="table"):
        sdmm.condition(torch.zeros(full - 1), n_cells, K, torch.zeros(3, nq), qcell)
    with pytest.raises(ValueError, match="qpos"):
        sdmm.condition(torch.zeros(full), n_cells, K, torch.zeros(3, nq - 1), qcell)
    cw, cm = torch.zeros(nq, K), torch.zeros(nq, K, 2)
    with pytest.raises(ValueError, match="dirs"):
        sdmm.pdf(torch.zeros(full), n_cells, K, qcell, cw, cm, torch.zeros(3, nq * 2 - 1), 2)
    with pytest.raises(ValueError, match="cond_m"):
        sdmm.pdf(torch.zeros(full), n_cells, K, qcell, cw, cm[:-1], torch.zeros(3, nq * 2), 2)
    with pytest.raises(ValueError, match="uniforms"):
        sdmm.sample(torch.zeros(full), n_cells, K, qcell, cw, cm, 4, uniforms=torch.zeros(3, nq * 4 - 1))
    off = torch.tensor([0, 1, 2, 3, 4], dtype=torch.int64)
    with pytest.raises(ValueError, match="status"):
        sdmm.fit_mixtures(off, torch.zeros(7, 4), {}, {}, sdmm.default_opts(K), status=torch.zeros(3, dtype=torch.int32))


def test_binding_rejects_undersized_product_and_parameter_tensors():
    import torch
    from paper_2111_13094_amd import sdmm
    K, Kb, n_cells, n_bsdf, nq, ns = 16, 16, 2, 3, 5, 4
    st = sdmm.COND_TABLE_STRIDE
    table, btable = torch.zeros(n_cells * K * st), torch.zeros(n_bsdf * Kb * st)
    qpos, bpar, frames = torch.zeros(3, nq), torch.zeros(3, nq), torch.zeros(9, nq)
    qcell, bcell = torch.zeros(nq, dtype=torch.int32), torch.zeros(nq, dtype=torch.int32)
    args = dict(table=table, n_cells=n_cells, K=K, qpos=qpos, qcell=qcell, btable=btable, n_bsdf=n_bsdf, Kb=Kb,
                bpar=bpar, bcell=bcell, frames=frames)
    for key, bad in (("btable", btable[:-1]), ("frames", frames[:, :-1]), ("bpar", bpar[:, :-1]),
                     ("bcell", bcell[:-1]), ("table", table[:-1])):
        with pytest.raises(ValueError, match=key):
            sdmm.product_sample(**{**args, key: bad}, ns=ns)
    with pytest.raises(ValueError, match="uniforms"):
        sdmm.product_sample(**args, ns=ns, uniforms=torch.zeros(3, nq * ns - 1))
    with pytest.raises(ValueError, match="btable"):  # (the draw count is taken from dirs' shape)
        sdmm.product_pdf(**{**args, "btable": btable[:-1]}, dirs=torch.zeros(3, nq * 2))
    n = n_cells * K
    f64 = dict(dtype=torch.float64)
    with pytest.raises(ValueError, match="jac"):
        sdmm.grad_to_params(torch.zeros(n_cells, K, 15, **f64), torch.zeros(n * 4 - 1, **f64),
                            torch.zeros(n * 2, **f64), torch.zeros(n * 15, **f64))
    with pytest.raises(ValueError, match="delta"):
        sdmm.mixture_from_params(torch.zeros(n_cells, K, **f64), torch.zeros(n * 3, **f64),
                                 torch.zeros(n * 2 - 1, **f64), torch.zeros(n * 3, **f64), torch.zeros(n * 15, **f64))


def test_binding_rejects_wrong_element_types():
    """A tensor of the right element count but a narrower type would let a kernel write
    past its end (an FP64 kernel into a float32 buffer), so the binding checks the element
    type of every tensor the caller supplies, before anything reaches the library."""
    import torch
    from paper_2111_13094_amd import sdmm
    K, n_cells, nq, ns = 16, 4, 8, 4
    n = nq * ns
    full = n_cells * K * sdmm.COND_TABLE_STRIDE
    table, qpos, qcell = torch.zeros(full), torch.zeros(3, nq), torch.zeros(nq, dtype=torch.int32)
    cw, cm = torch.zeros(nq, K), torch.zeros(nq, K, 2)
    with pytest.raises(TypeError, match="table"):
        sdmm.condition(table.double(), n_cells, K, qpos, qcell)
    with pytest.raises(TypeError, match="qcell"):
        sdmm.condition(table, n_cells, K, qpos, qcell.long())
    with pytest.raises(TypeError, match="cond_w"):
        sdmm.pdf(table, n_cells, K, qcell, cw.double(), cm, torch.zeros(3, nq * 2), 2)
    with pytest.raises(TypeError, match="uniforms"):
        sdmm.sample(table, n_cells, K, qcell, cw, cm, ns, uniforms=torch.zeros(3, n, dtype=torch.float64))
    out = (torch.zeros(3, n), torch.zeros(n), torch.zeros(n, dtype=torch.uint8))
    for i, (what, bad) in enumerate((("dirs", torch.zeros(3, n, dtype=torch.float64)),
                                     ("pdf", torch.zeros(n, dtype=torch.float64)),
                                     ("valid", torch.zeros(n, dtype=torch.int32)))):
        o = list(out)
        o[i] = bad
        with pytest.raises(TypeError, match=what):
            sdmm.condition_sample_pdf(table, n_cells, K, qpos, qcell, ns, out=tuple(o))
    Kb, n_bsdf = 16, 3
    args = dict(table=table, n_cells=n_cells, K=K, qpos=qpos, qcell=qcell,
                btable=torch.zeros(n_bsdf * Kb * sdmm.COND_TABLE_STRIDE), n_bsdf=n_bsdf, Kb=Kb,
                bpar=torch.zeros(3, nq), bcell=torch.zeros(nq, dtype=torch.int32), frames=torch.zeros(9, nq))
    pout = (torch.zeros(3, n), torch.zeros(n), torch.zeros(n, dtype=torch.uint8), torch.zeros(n, dtype=torch.int32))
    for i, (what, bad) in enumerate((("dirs", torch.zeros(3, n, dtype=torch.float64)),
                                     ("pdf", torch.zeros(n, dtype=torch.float64)),
                                     ("valid", torch.zeros(n, dtype=torch.int32)),
                                     ("pair", torch.zeros(n, dtype=torch.float32)))):
        o = list(pout)
        o[i] = bad
        with pytest.raises(TypeError, match=what):
            sdmm.product_sample(**args, ns=ns, out=tuple(o))
    with pytest.raises(TypeError, match="frames"):
        sdmm.product_pdf(**{**args, "frames": torch.zeros(9, nq, dtype=torch.float64)}, dirs=torch.zeros(3, nq * 2))
    nc = n_cells * K
    with pytest.raises(TypeError, match="jac"):
        sdmm.grad_to_params(torch.zeros(n_cells, K, 15, dtype=torch.float64), torch.zeros(nc * 4),
                            torch.zeros(nc * 2, dtype=torch.float64), torch.zeros(nc * 15, dtype=torch.float64))
    f64 = dict(dtype=torch.float64)
    with pytest.raises(TypeError, match="L"):
        sdmm.mixture_from_params(torch.zeros(n_cells, K, **f64), torch.zeros(nc * 3, **f64),
                                 torch.zeros(nc * 2, **f64), torch.zeros(nc * 3, **f64), torch.zeros(nc * 15))
    off = torch.tensor([0, 1, 2, 3, 4], dtype=torch.int64)
    mix = {"pi": torch.zeros(nc, **f64), "mu_dir": torch.zeros(nc * 3, **f64), "mu_pos": torch.zeros(nc * 3, **f64),
           "cov": torch.zeros(nc * 15)}
    with pytest.raises(TypeError, match="cov"):
        sdmm.fit_mixtures(off, torch.zeros(7, 4), mix, sdmm.new_state(n_cells, K, device="cpu"), sdmm.default_opts(K))
    with pytest.raises(TypeError, match="cell_offsets"):
        sdmm.fit_mixtures(off.int(), torch.zeros(7, 4), mix, sdmm.new_state(n_cells, K, device="cpu"),
                          sdmm.default_opts(K))


def test_noalloc_entry_rejects_on_the_host(lib):
    """The entry point without a workspace checks its arguments and its size limit before
    it looks up the device array, so these return without a GPU."""
    from paper_2111_13094_amd import sdmm
    m, st = sdmm.Mixtures(), sdmm.EmState()
    m.n_cells, m.K = 4, 16
    m.weights = m.mean_dir = m.mean_pos = m.cov = C.c_void_p(256)
    st.s0 = st.s2 = st.sw = st.step = C.c_void_p(256)
    p = C.c_void_p(256)
    o = sdmm.default_opts(16, schedule=sdmm.SCHED_PER_CELL)
    assert lib.sdmm_fit_mixtures_noalloc(p, p, 100, C.byref(m), C.byref(st), C.byref(o), p, None) == -1
    o = sdmm.default_opts(16, use_graph=1)
    assert lib.sdmm_fit_mixtures_noalloc(p, p, 100, C.byref(m), C.byref(st), C.byref(o), p, None) == -1
    o = sdmm.default_opts(16, min_range=16, max_ranges=1 << 20)
    n = 1 << 22
    assert lib.sdmm_fit_workspace_size(4, 16, n, C.byref(o)) > sdmm.NOALLOC_SCRATCH_BYTES
    assert lib.sdmm_fit_mixtures_noalloc(p, p, n, C.byref(m), C.byref(st), C.byref(o), p, None) == -3
    assert lib.sdmm_fit_mixtures_noalloc(None, p, 100, C.byref(m), C.byref(st), C.byref(o), p, None) == -1
