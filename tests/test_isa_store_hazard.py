"""Regression check on the library's own gfx950 machine code (CPU only).

A vector-memory store of more than 64 bits reads its data registers one
instruction after it issues.  If the very next instruction overwrites those
registers, the low part of the stored data can be the new value instead of
the intended one.  The compiler inserts the needed wait for buffer stores
whose scalar offset is the constant 0 but not for stores with a register
scalar offset, so the kernels pass the whole offset per lane for wide stores.
This test disassembles the built library's device code (every translation
unit's offload bundle) and fails if any wide store is followed directly by an
instruction that writes its data.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1407_0674_amd", "libpnpcdft.so")
LLVM = "/opt/rocm/llvm/bin"

WIDE = ("buffer_store_dwordx3", "buffer_store_dwordx4", "global_store_dwordx3",
        "global_store_dwordx4", "flat_store_dwordx3", "flat_store_dwordx4")


def _vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def _disassemble():
    if not (os.path.exists(LIB) and os.path.exists(os.path.join(LLVM, "llvm-objdump"))):
        pytest.skip("library or ROCm LLVM tools not present")
    tmp = tempfile.mkdtemp()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    try:
        fat, dummy = (os.path.join(tmp, x) for x in ("fat.bin", "dummy.so"))
        subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fat}", LIB, dummy],
                       check=True, capture_output=True)
        blob = open(fat, "rb").read()
        # one offload bundle per translation unit, concatenated (with padding)
        starts = []
        i = blob.find(magic)
        while i >= 0:
            starts.append(i)
            i = blob.find(magic, i + 1)
        out = []
        for k, st in enumerate(starts):
            part, co = os.path.join(tmp, f"b{k}.bin"), os.path.join(tmp, f"b{k}.co")
            with open(part, "wb") as f:
                f.write(blob[st:starts[k + 1] if k + 1 < len(starts) else len(blob)])
            subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={part}",
                            "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                           check=True, capture_output=True)
            out.append(subprocess.run([f"{LLVM}/llvm-objdump", "-d", "--no-show-raw-insn", co],
                                      check=True, capture_output=True, text=True).stdout)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return "\n".join(out)


def test_no_wide_store_data_overwritten_by_next_instruction():
    text = _disassemble()
    insns = []
    for line in text.splitlines():
        s = line.strip()
        if not s or s.endswith(">:") or s.startswith(("Disassembly", ";")) or ":" in s.split()[0]:
            continue
        insns.append(s.split("//")[0].strip())
    wide = 0
    bad = []
    for k, ins in enumerate(insns[:-1]):
        op = ins.split()[0]
        if op not in WIDE:
            continue
        wide += 1
        ops = [o.strip() for o in ins.split(None, 1)[1].split(",")]
        data = _vregs(ops[0] if op.startswith("buffer") else ops[1])
        nxt = insns[k + 1].split()
        if nxt and nxt[0].startswith("v_") and len(nxt) > 1 and (_vregs(nxt[1].rstrip(",")) & data):
            bad.append(f"{ins}  ->  {insns[k + 1]}")
    assert wide > 100, "no wide stores found: disassembly not parsed"
    assert not bad, f"{len(bad)} wide stores overwritten at once, e.g. {bad[:3]}"
