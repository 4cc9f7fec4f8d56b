"""Build-time guard for the direct HBM-to-LDS loads.  A direct load takes its LDS destination from
the m0 register; some loads are written as inline asm that sets m0 itself (so the compiler does not
add its blanket wait for every direct load before each LDS read), others come from the compiler's
builtin.  The compiler warns that an asm clobber of m0 may not be honoured, which would break a
builtin load that relied on an m0 value set before an asm block.  This test compiles every HIP
source to gfx950 assembly (CPU only) and checks that no load depends on m0 across anything:

* every instruction that names m0 is `s_mov_b32 m0, s<n>`, and no instruction reads m0 implicitly
  (relative indexing, messages, GWS / append counters, buffer loads into LDS);
* within a basic block, every m0 write is followed by a direct load before any other m0 write,
  direct load, label or branch, and every direct load is preceded by its own m0 write under the
  same rule (one m0 write per load, set in the same straight-line code).
"""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_20870_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

M0_WRITE = re.compile(r"^s_mov_b32 m0, s\d+$")
# instructions that read m0 without naming it (relative indexing, messages, GWS/ordered/append
# counters, interpolation, buffer loads into LDS)
IMPLICIT_M0 = re.compile(r"^(s_movrel|v_movrel|s_sendmsg|ds_gws|ds_ordered_count|ds_append|ds_consume|v_interp|"
                         r"buffer_load\S*\s.*\blds\b|buffer_store_lds)")


def _assembly(src, out_dir):
    from paper_2602_20870_amd.build import FLAGS
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    flags = [f for f in FLAGS if f not in ("-fPIC",)]
    r = subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", src, "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def _instructions(path):
    """(kind, text) per line: 'label' for labels, 'ins' for instructions (comments and directives dropped)."""
    out = []
    for raw in open(path):
        line = raw.split(";")[0].strip()
        if not line or line.startswith("."):
            if line.startswith(".LBB") and line.endswith(":"):
                out.append(("label", line))
            continue
        out.append(("label", line) if line.endswith(":") else ("ins", line))
    return out


def _ends_block(kind, text):
    return kind == "label" or text.startswith(("s_branch", "s_cbranch", "s_setpc", "s_endpgm"))


def _check(ins):
    problems, writes, loads = [], 0, 0
    for k, (kind, text) in enumerate(ins):
        if kind != "ins":
            continue
        toks = re.split(r"[\s,]+", text)
        is_load = text.startswith("global_load_lds")
        if IMPLICIT_M0.match(text):
            problems.append(f"instruction that reads m0 implicitly: {text}")
        if "m0" in toks:
            writes += 1
            if not M0_WRITE.match(text):
                problems.append(f"instruction other than an m0 write names m0: {text}")
                continue
            j = k + 1
            while j < len(ins):
                kj, tj = ins[j]
                if kj == "ins" and tj.startswith("global_load_lds"):
                    break
                if _ends_block(kj, tj) or (kj == "ins" and "m0" in re.split(r"[\s,]+", tj)):
                    problems.append(f"m0 write not followed by its direct load: {text} ... {tj}")
                    break
                j += 1
        if is_load:
            loads += 1
            j = k - 1
            while j >= 0:
                kj, tj = ins[j]
                if kj == "ins" and M0_WRITE.match(tj):
                    break
                if _ends_block(kj, tj) or (kj == "ins" and tj.startswith("global_load_lds")):
                    problems.append(f"direct load without its own m0 write in the same block: {text}")
                    break
                j -= 1
    return problems, writes, loads


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_every_direct_load_sets_its_own_m0(tmp_path):
    total_loads = 0
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        problems, writes, loads = _check(_instructions(_assembly(src, str(tmp_path))))
        assert not problems, f"{os.path.basename(src)}: {problems[:5]}"
        assert writes == loads, (os.path.basename(src), writes, loads)
        total_loads += loads
    assert total_loads > 0      # the kernels do use direct loads: the check is not vacuous


def test_guard_catches_a_load_that_relies_on_an_earlier_m0():
    """The rule itself, on hand-written listings: a builtin load after an asm block's m0 write."""
    ok = [("ins", "s_mov_b32 m0, s4"), ("ins", "v_add_u32_e32 v1, 4, v1"), ("ins", "global_load_lds_dwordx4 v[2:3], off")]
    assert _check(ok)[0] == []
    shared = [("ins", "s_mov_b32 m0, s4"), ("ins", "global_load_lds_dwordx4 v[2:3], off"),
              ("ins", "global_load_lds_dwordx4 v[4:5], off")]
    assert _check(shared)[0]
    across_label = [("ins", "s_mov_b32 m0, s4"), ("label", ".LBB0_3:"), ("ins", "global_load_lds_dwordx4 v[2:3], off")]
    assert _check(across_label)[0]
    other_use = [("ins", "s_movrels_b32 s0, s1"), ("ins", "v_movreld_b32_e32 v0, m0")]
    assert _check(other_use)[0]
