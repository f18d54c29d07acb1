#!/usr/bin/env python3
"""Compression-ratio cost of the stream's format constants (a study, not a
test): the residual quantization radius R and the longest Huffman codeword
are 512 and 12 in this implementation (one workgroup builds a codebook, one
4096-entry table decodes it); the alternative R = 32768 with 24-bit codes
keeps more residuals out of the raw-float store at tight bounds.  Both are
built from the CPU oracle with the constants overridden, and compress the
same crops of the wind and turbulence workloads; CR is printed for each
(Huffman stream, and with the zero-byte-elision stage).

Usage: python tests/format_cost_study.py   (about a minute on one core)
"""
import json
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
VARIANTS = [("R512_L12", 512, 12), ("R32768_L24", 32768, 24)]
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
    base = res[VARIANTS[0][0]]
    for i, row in enumerate(base):
        alt = res[VARIANTS[1][0]][i]
        print("workload %d %s eb %g: CR %.3f (R 512, 12 bits) vs %.3f (R 32768, 24 bits), %+.2f%%; "
              "with the stage %.3f vs %.3f; raw words %d vs %d" %
              (row["workload"], "x".join(map(str, row["shape"])), row["eb"], row["CR"], alt["CR"],
               100 * (alt["CR"] / row["CR"] - 1), row["CR_stage"], alt["CR_stage"], row["raw_words"],
               alt["raw_words"]))


if __name__ == "__main__":
    main()
