#!/usr/bin/env python3
"""Compression-ratio cost of the stream's format constants (a study, not a
test): the residual quantization radius R and the longest Huffman codeword
were 512 and 12 when this study was written (one workgroup builds a
codebook, one 4096-entry table decodes it; the format now allows 16-bit
codewords, decoded through the same table plus a per-length search for the
rare long ones).  Longer codewords (16, 24) and the wider radius
R = 32768 are built from the CPU oracle with the constants overridden, and
compress the same crops of the wind and turbulence workloads; CR is printed
for each (Huffman stream, and with the zero-byte-elision stage), with the
change against R 512 / 12 bits.

Usage: python tests/format_cost_study.py   (about a minute on one core)
"""
import json
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
VARIANTS = [("R512_L12", 512, 12), ("R512_L16", 512, 16), ("R512_L24", 512, 24), ("R32768_L24", 32768, 24)]
CASES = [(1, (360, 720, 8), 1e-3), (1, (360, 720, 8), 1e-2), (2, (512, 512, 8), 1e-3), (2, (512, 512, 8), 1e-2)]

WORKER = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import oracle, synthfields
oracle._SO = sys.argv[2]
out = []
for cfg, shape, eb in json.loads(sys.argv[3]):
    f, m = synthfields.workload(cfg, shape=tuple(shape))
    fn = f.numpy()
    dt = m["dt_dx"]
    b = oracle.compress(fn, eb, dt_dx=dt, dt_dy=dt)
    c = oracle.compress(fn, eb, dt_dx=dt, dt_dy=dt, backend=1)
    info = oracle.stream_info(b)
    out.append(dict(workload=cfg, shape=shape, eb=eb, CR=fn.size * 4 / len(b), CR_stage=fn.size * 4 / len(c),
                    raw_words=int(info["n_raw"]), residual_codes=int(info["n_q"])))
print(json.dumps(out))
"""


def main():
    res = {}
    with tempfile.TemporaryDirectory() as tmp:
        for name, r, l in VARIANTS:
            so = os.path.join(tmp, "libcpo_%s.so" % name)
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                                   "-DCPO_QR=%d" % r, "-DCPO_MAXLEN=%d" % l, "-o", so,
                                   os.path.join(ROOT, "oracle", "cpo.c"), "-lm"])
            out = subprocess.run([sys.executable, "-c", WORKER, ROOT, so, json.dumps(CASES)], capture_output=True,
                                 text=True, check=True).stdout
            res[name] = json.loads(out.strip().splitlines()[-1])
    for i, row in enumerate(res[VARIANTS[0][0]]):
        cells = []
        for name, _, _ in VARIANTS:
            alt = res[name][i]
            cells.append("%s CR %.3f (%+.2f%%), with the stage %.3f, raw words %d" %
                         (name, alt["CR"], 100 * (alt["CR"] / row["CR"] - 1), alt["CR_stage"], alt["raw_words"]))
        print("workload %d %s eb %g: %s" % (row["workload"], "x".join(map(str, row["shape"])), row["eb"],
                                            "; ".join(cells)))

if __name__ == "__main__":
    main()
