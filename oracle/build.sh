#!/bin/sh
# Builds the CPU oracle library (test infrastructure only).
set -e
cd "$(dirname "$0")"
gcc -std=c11 -D_GNU_SOURCE -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared \
    -Wall -Wextra -o liboracle.so start_oracle.c -lm
