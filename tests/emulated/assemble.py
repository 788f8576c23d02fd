"""Assemble the host build of the accept kernel: the library's device header
(without its MFMA section and address-space casts) and the text of k_accept,
with a wavefront rendezvous between the loads and the stores of a sweep chunk
(the hardware runs a wavefront's lanes in lockstep; host threads do not).

Usage: assemble.py <repository root> <output header>"""
import re, sys
root = sys.argv[1]
dev = open(f"{root}/paper_1901_01047_amd/csrc/dcax_dev.h").read()
dev = dev.replace('#include <hip/hip_runtime.h>', '')
dev = dev.replace('#include "dcax.h"', '#include "dcax.h"')
# drop the MFMA section (clang vector types and builtins)
i0 = dev.index('// ------------------------------------------------------------------ MFMA')
i1 = dev.index('// ------------------------------------------------------------ generator')
dev = dev[:i0] + dev[i1:]
dev = dev.replace('__attribute__((address_space(1)))', '')
win = open(f"{root}/paper_1901_01047_amd/csrc/dcax_window.hip").read()
i0 = win.index('constexpr int MAX_ATTEMPTS')
i1 = win.index('// --------------------------------------------------------- Y = N g_{I,c}')
acc = win[i0:i1]
# wave lockstep between the loads and the stores of a sweep chunk
pat = '          v1[u] = T_s[1][r * LS + lane];\n        }\n'
assert pat in acc
acc = acc.replace(pat, pat + '        EMU_WAVE_SYNC();\n')
out = '#include "emu_hip.h"\n' + dev.replace('namespace dcax {', 'namespace dcax {', 1)
# append the kernel inside the namespace
k = out.rindex('}  // namespace dcax')
out = out[:k] + acc + '\n' + out[k:]
open(sys.argv[2], 'w').write(out)
