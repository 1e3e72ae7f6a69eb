"""libnhdc shares torch's HIP runtime: only one libamdhip64 is mapped."""
import subprocess
import sys


def test_single_hip_runtime_in_process():
    code = ("from paper_2511_02021_amd import nhdc; nhdc.lib();"
            "maps=open('/proc/self/maps').read();"
            "libs={l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l};"
            "print(len(libs)); print(sorted(libs))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=__import__("os").path.dirname(__import__("os").path.dirname(
                           __import__("os").path.abspath(__file__))))
    assert r.returncode == 0, r.stderr
    assert r.stdout.splitlines()[0] == "1", r.stdout
