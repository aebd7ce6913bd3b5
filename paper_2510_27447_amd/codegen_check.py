"""Build-time check of the generated gfx950 code for one known miscompilation.

When a wavefront leaves a divergent region (an if, or a loop whose lanes exit
at different iterations) the code restores the execution mask (EXEC) at the
start of the join block.  In register-starved kernels the compiler has been
seen to place spill code (AGPR copies, scratch stores) at the top of such a
block *before* that restore.  Those instructions run with the mask of the
region just left -- empty when every lane has exited a loop -- so they store
nothing for the other lanes, whose values are later reloaded stale: results
then depend on what earlier waves left in scratch or registers.

This module scans the device assembly that the build saves beside each object
(-save-temps) and reports every lane-masked vector write that sits in a block
reached by s_cbranch_execz before that block writes EXEC.  The build fails on
any finding.  The step kernels are written without divergent branches in
their per-step work, so a finding means the compiler has introduced one.
"""
from __future__ import annotations

import re

# instructions that write EXEC: "s_<op>_b64 exec, ..." and the *_saveexec_* forms
_EXEC_WRITE = re.compile(r"^s_(\w+_b64\s+exec\s*,|\w*saveexec\w*\s)")
_LABEL = re.compile(r"^(\.LBB\w+):")
_BLOCK_START = re.compile(r"^(\.LBB\w+:|; %bb\.\d+:)")
_BLOCK_END = ("s_endpgm", "s_branch", "s_cbranch_", "s_setpc")
_FUNC = re.compile(r"^(_Z\w+|\w+):\s*(;.*)?$")
# instructions that do not depend on EXEC or write no vector lane
_EXEMPT = ("v_writelane", "v_readlane", "v_readfirstlane", "s_", "buffer_wbl2", "buffer_inv")


def lane_masked_writes_before_exec_restore(asm_text: str):
    """List of (function, label, line number, instruction) findings."""
    lines = asm_text.splitlines()
    targets = set(re.findall(r"s_cbranch_execz\s+(\.LBB\w+)", asm_text))
    found = []
    func = None
    i = 0
    while i < len(lines):
        line = lines[i]
        fm = _FUNC.match(line)
        if fm and not line.startswith(".") and not line.startswith(";"):
            func = fm.group(1)
        lm = _LABEL.match(line)
        if lm and lm.group(1) in targets:
            j = i + 1
            while j < len(lines):
                t = lines[j].split(";")[0].strip()
                if _BLOCK_START.match(lines[j]) or t.startswith(_BLOCK_END):
                    break
                if _EXEC_WRITE.match(t):
                    break
                if t and not t.startswith(".") and not t.startswith(_EXEMPT):
                    found.append((func, lm.group(1), j + 1, t))
                j += 1
        i += 1
    return found


def check_file(path: str):
    with open(path) as f:
        return lane_masked_writes_before_exec_restore(f.read())
