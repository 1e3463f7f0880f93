"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The C oracle: a separate process loads a build of the same source made here
  with gcc and the sanitizers (their runtimes preloaded) and runs a tiny
  Argmax, a key switch at every level, the Phoenix path, slot packing and a
  bootstrap.  Leak checking is off: the Python interpreter itself holds memory
  to exit.
* The host C++ that builds the bootstrapping tables (binary128), in a small
  driver over every group of both transforms.
Any sanitizer report fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    sys.path.insert(0, {tests!r})
    import numpy as np
    import workload as W
    from conftest import make_oracle
    from oracle.ckks import argmax_rotation_steps
    o = make_oracle("tiny")
    o.keygen(3, sorted(set(argmax_rotation_steps(4, 8, o.slots)) | set(range(1, 9)) | set(o.slots - j for j in range(1, 9))))
    y = W.logits(9, 1, 3, 5)
    lo, hi = W.d_bounds(3)
    z = o.eval_argmax(o.encrypt_logits(y, 4), 3, 5, lo, hi, 5)
    o.decrypt_decode(z, 5)
    pr = [int(v) for v in o.primes]
    rng = np.random.default_rng(1)
    for lvl in range(o.n_q):
        d = np.stack([rng.integers(0, pr[t], o.n, dtype=np.uint64) for t in range(lvl + 1)])
        o.key_switch(0, d)
    zp = o.eval_argmax_phoenix(o.encrypt_logits(y, 6), 3, 5, lo, hi, 7)
    blocks = [W.logits(9, 20 + i, K, C) for i, (K, C) in enumerate([(2, 3), (3, 4)])]
    oc = o.encrypt_packed(blocks, 8)
    o.eval_argmax_packed(oc, [(2, 3), (3, 4)], [W.d_bounds(2)[0], W.d_bounds(3)[0]],
                         [W.d_bounds(2)[1], W.d_bounds(3)[1]], 9)
    b = make_oracle("tiny_boot")
    b.keygen(11, b.boot_steps())
    ct = b.lower(b.encrypt(b.encode(rng.uniform(-1, 1, b.slots), 2.0**49), 2.0**49, 12), 2)
    b.bootstrap(ct)
    print("sanitized oracle run complete")
""")


def _build_sanitized(out_path):
    """The oracle source built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code, gcc) into out_path."""
    src = os.path.join(ROOT, "oracle", "ckks_oracle.c")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", out_path, src,
           "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    lib = _build_sanitized(str(tmp_path / "libckks_oracle_san.so"))
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, tests=HERE)], env=env,
                       capture_output=True, text=True, timeout=880)
    report = r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr, report
    assert "runtime error" not in r.stderr, report
    assert r.returncode == 0, report
    assert "sanitized oracle run complete" in r.stdout


DRIVER = r"""
#include <cstdio>
#include "boot_tables.h"
int main() {
  // every group of both transforms at N = 2^10 and N = 2^12, 2 and 3 groups,
  // full-slot and sparse-slot (n = 8 and 32: the widened groups included)
  double cheb[64];
  for (int log_n : {10, 12})
    for (int log_ns : {log_n - 1, 3, 5})
      for (int groups : {2, 3})
        for (int inverse : {0, 1})
          for (int g = 0; g < groups; ++g) {
            secpe::BootGroupTable t = secpe::boot_group_table(log_n, log_ns, groups, 12, 8, inverse, g);
            if (t.diags.empty()) return 2;
            for (const secpe::BootDiag& d : t.diags)
              if ((int)d.re.size() != t.ns || d.off < 0 || d.off >= t.ns) return 3;
          }
  secpe::boot_cheb_coeffs(24, 4, 31, cheb);
  std::printf("tables ok %.3f\n", cheb[1]);
  return 0;
}
"""


@pytest.mark.timeout(600)
def test_boot_tables_under_asan_and_ubsan(tmp_path):
    """The host C++ that builds the bootstrapping tables (binary128), under
    AddressSanitizer and UndefinedBehaviorSanitizer."""
    csrc = os.path.join(ROOT, "paper_2502_00847_amd", "csrc")
    drv = tmp_path / "drv.cpp"
    drv.write_text(DRIVER)
    exe = str(tmp_path / "drv")
    subprocess.run(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-std=gnu++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", csrc, str(drv), os.path.join(csrc, "boot_tables.cpp"),
                    "-o", exe, "-lquadmath"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=580,
                       env=dict(os.environ, ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1"))
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "tables ok" in r.stdout, (r.returncode, r.stderr[-2000:])

