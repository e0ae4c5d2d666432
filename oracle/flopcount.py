"""FP64 operation counts of one particle step, measured on the oracle
(test infrastructure; see flopcount.cpp).

``counts()`` compiles flopcount.cpp -- the oracle's own C sources built as C++
with every double replaced by a counting scalar type -- into a temporary
directory, runs it, and returns its per-particle counts: for each piece
(RK4 step, energy, deposit weights, one Picard or Newton iteration of the
implicit midpoint rule, one discrete-gradient iteration, gather, metric,
equations of motion) the additions/subtractions, multiplications, divisions,
square roots and transcendental calls, and their sum ``flop``.
"""
import json
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def counts(particles: int = 4096) -> dict:
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "flopcount")
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-o", exe,
                               os.path.join(HERE, "flopcount.cpp"), "-lm"], cwd=HERE)
        out = subprocess.run([exe, str(particles)], check=True, capture_output=True,
                             text=True).stdout
    return json.loads(out)


if __name__ == "__main__":
    print(json.dumps(counts(), indent=1))
