"""The gfx950 code the library is built from, checked without a GPU.

Every dense kernel instance is compiled to assembly with the library's own
flags; no taken branch may leave a matrix-core result (or operand) short of
the wait states the compiler uses on straight-line code, and the bf16 forms
must not spill registers to scratch.  The checker itself is pinned on small
hand-written snippets.
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

import asm_hazards
from paper_1410_0342_amd import build as B

HIPCC = B.HIPCC if os.path.exists(B.HIPCC) else shutil.which("hipcc")


def test_checker_flags_a_result_read_right_after_a_taken_branch():
    text = """
    v_mfma_f32_16x16x4_f32 a[4:7], v6, v58, 0
    s_cbranch_vccnz .L1
    v_mov_b32_e32 v1, v2
.L1:
    v_accvgpr_read_b32 v61, a7
    """
    found, _ = asm_hazards.check(text, {"v_mfma_f32_16x16x4_f32": 10})
    assert len(found) == 1 and found[0][4] == 1


def test_checker_accepts_enough_wait_states_and_unrelated_reads():
    ok = """
    v_mfma_f32_16x16x4_f32 a[4:7], v6, v58, 0
    s_cbranch_vccnz .L1
    v_mov_b32_e32 v1, v2
.L1:
    s_nop 8
    v_accvgpr_read_b32 v61, a7
    v_accvgpr_read_b32 v60, a9
    """
    found, _ = asm_hazards.check(ok, {"v_mfma_f32_16x16x4_f32": 10})
    assert found == []
    other = """
    v_mfma_f32_16x16x4_f32 a[4:7], v6, v58, 0
    s_cbranch_vccnz .L1
.L1:
    v_accvgpr_read_b32 v60, a9
    """
    assert asm_hazards.check(other, {"v_mfma_f32_16x16x4_f32": 10})[0] == []


def test_checker_learns_the_straight_line_requirement():
    text = """
    v_mfma_f32_16x16x32_bf16 a[0:3], v[2:5], v[6:9], 0
    s_nop 7
    v_accvgpr_read_b32 v10, a3
    v_mfma_f32_16x16x32_bf16 a[0:3], v[2:5], v[6:9], 0
    s_cbranch_scc1 .L2
.L2:
    s_nop 5
    v_accvgpr_read_b32 v11, a0
    """
    found, need = asm_hazards.check(text)
    assert need["v_mfma_f32_16x16x32_bf16"] == 8
    assert len(found) == 1 and found[0][4] == 7


def test_checker_flags_a_vector_write_feeding_a_product_across_a_branch():
    text = """
    v_cvt_pk_bf16_f32 v20, v1, v2
    s_cbranch_execz .L3
.L3:
    v_mfma_f32_16x16x16_bf16 a[0:3], v[20:21], v[22:23], a[0:3]
    """
    assert len(asm_hazards.check(text)[0]) == 1


UNITS = [(p, l) for p in (0, 1, 3) for l in (0, 1)]


def _asm(unit, tmp):
    prec, lks = unit
    out = os.path.join(tmp, "dense_prec%d_%d.s" % unit)
    cmd = [HIPCC] + B.FLAGS + B.dense_prec_flags(prec, lks) + ["-x", "hip", "--cuda-device-only", "-S",
                               os.path.join(B.CSRC, "dense_prec.hip"), "-o", out,
                               "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return unit, open(out).read(), r.stderr


@pytest.fixture(scope="module")
def dense_asm(tmp_path_factory):
    if not HIPCC:
        pytest.skip("hipcc not available")
    tmp = str(tmp_path_factory.mktemp("asm"))
    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        return {u: (text, remarks) for u, text, remarks in ex.map(lambda u: _asm(u, tmp), UNITS)}


@pytest.fixture(scope="module")
def learned_needs(dense_asm):
    """The compiler's straight-line wait states, learned over every unit (a
    unit may lack a sample of some product)."""
    need = {}
    for text, _ in dense_asm.values():
        for op, n in asm_hazards.straight_line_needs(asm_hazards.parse(text)[0]).items():
            need[op] = max(need.get(op, 0), n)
    return need


@pytest.mark.parametrize("unit", UNITS)
def test_no_short_wait_paths_in_the_dense_kernels(dense_asm, learned_needs, unit):
    assert len(learned_needs) >= 3, learned_needs
    found, _ = asm_hazards.check(dense_asm[unit][0], learned_needs)
    assert found == [], found[:5]


def _scratch(remarks):
    out, name = {}, None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    return out


@pytest.mark.parametrize("unit", [u for u in UNITS if u[0] != 0])
def test_bf16_forms_do_not_spill(dense_asm, unit):
    sc = _scratch(dense_asm[unit][1])
    assert len(sc) > 20
    assert {k: v for k, v in sc.items() if v} == {}


@pytest.mark.parametrize("src", ["proxprox.hip", "linalg.hip"])
def test_no_short_wait_paths_in_the_other_matrix_core_kernels(dense_asm, learned_needs, src, tmp_path):
    """The prox-prox passes and the linear-algebra kernels use fp32 matrix-core
    products too; their paths are held to the same wait states (learned from
    the dense units and from the file itself)."""
    out = str(tmp_path / (src + ".s"))
    cmd = [HIPCC] + B.FLAGS + ["-x", "hip", "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    text = open(out).read()
    need = dict(learned_needs)
    for op, n in asm_hazards.straight_line_needs(asm_hazards.parse(text)[0]).items():
        need[op] = max(need.get(op, 0), n)
    found, _ = asm_hazards.check(text, need)
    assert found == [], found[:5]
