#!/bin/sh
# Builds the CPU oracle (test infrastructure) as a shared library next to
# this script.  binary64 semantics are kept: no fast-math, no FMA contraction.
set -e
here=$(cd "$(dirname "$0")" && pwd)
gcc -O2 -fopenmp -fPIC -shared -ffp-contract=off -fno-fast-math \
    -Wall -Wextra -o "$here/liboracle.so" "$here/oracle.c" -lquadmath -lm
