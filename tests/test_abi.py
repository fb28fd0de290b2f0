"""CPU checks of the C-ABI boundary: the library is built, loads, and exports
every function the headers under include/ declare.  No compute call is made (no GPU
here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "\n".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(shock_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for must in ("shock_leaf_search", "shock_leaf_search_ex", "shock_opts_init", "shock_last_stats",
                 "shock_rf_leaf_search_ex", "shock_leaf_query", "shock_rice_encode", "shock_rice_decode"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2308_09561_amd as shock
    lib = shock.lib()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(shock.binding.EXPORTED) >= set(_declared_functions())


def test_library_is_a_gfx950_build():
    import paper_2308_09561_amd as shock
    blob = open(shock.lib_path(), "rb").read()
    assert b"gfx950" in blob


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    import paper_2308_09561_amd as shock
    k = torch.zeros(4, dtype=torch.int64)
    o = torch.tensor([0, 4], dtype=torch.int64)
    with pytest.raises(ValueError):
        shock.leaf_search(k, o)


def test_oracle_is_not_imported_by_the_package():
    pkg = os.path.join(ROOT, "paper_2308_09561_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "shock_oracle" not in src, f


def test_ctypes_structs_match_the_headers(tmp_path):
    """Every struct the binding passes across the boundary has the size and
    field offsets the C compiler gives the header's typedef (compiled here
    with gcc against include/)."""
    import ctypes
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    from paper_2308_09561_amd import binding as b
    pairs = [(b.ShockOpts, "shock_opts"), (b.ShockStats, "shock_stats"), (b.BipStats, "shock_bip_stats"),
             (b.MphfParams, "shock_mphf_params"), (b.MphfStats, "shock_mphf_stats"),
             (b.QueueParams, "shock_queue_params"), (b.TicketInfo, "shock_ticket_info"),
             (b.QueueStats, "shock_queue_stats")]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "shockleaf.h"', '#include "shockmphf.h"',
             "int main(void) {"]
    want = []
    for cls, cname in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f}));')
            want.append(getattr(cls, f).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want


def test_noalloc_limits_match_the_header():
    """The binding's copies of the no-allocation limits are the header's."""
    from paper_2308_09561_amd import binding as b
    text = open(os.path.join(ROOT, "include", "shockleaf.h")).read()
    want = {}
    for name in ("SHOCK_NOALLOC_MAX_LEAVES", "SHOCK_NOALLOC_MAX_WORKERS", "SHOCK_NOALLOC_SCRATCH_BYTES"):
        m = re.search(r"#define\s+" + name + r"\s+\(?(\d+)u?(?:\s*<<\s*(\d+))?\)?", text)
        assert m, name
        want[name] = int(m.group(1)) << int(m.group(2) or 0)
        assert getattr(b, name) == want[name], name


def test_binding_rejects_short_outputs_and_empty_keys_with_leaves():
    torch = pytest.importorskip("torch")
    from paper_2308_09561_amd import binding as b
    k = torch.zeros(4, dtype=torch.int64)
    o = torch.tensor([0, 2, 4], dtype=torch.int64)
    with pytest.raises(ValueError):
        b._check_out(torch.zeros(1, dtype=torch.int64), 2, torch.int64, k.device, "out_seeds")
    with pytest.raises(ValueError):
        b._check_out(torch.zeros(2, dtype=torch.int32), 2, torch.int64, k.device, "out_seeds")
    with pytest.raises(ValueError):
        b._check_out(torch.zeros(4, dtype=torch.int64)[::2], 2, torch.int64, k.device, "out_seeds")
    b._check_out(torch.zeros(2, dtype=torch.int64), 2, torch.int64, k.device, "out_seeds")
    assert o.numel() == 3
