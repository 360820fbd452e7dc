#!/bin/sh
# Builds the CPU oracle (test infrastructure) into oracle/liboracle.so.
set -e
cd "$(dirname "$0")"
gcc -O2 -fPIC -shared -std=gnu11 -fopenmp -ffp-contract=off -fno-fast-math -Wall -Wno-unused-function \
    -o liboracle.so.tmp fmm_oracle.c -lm
mv liboracle.so.tmp liboracle.so
