#!/bin/sh
# Builds the CPU oracle library (test infrastructure only).
#   sh build.sh            liboracle.so
#   sh build.sh sanitize   liboracle_san.so: the same sources with AddressSanitizer
#                          and UndefinedBehaviorSanitizer, every finding fatal
set -e
cd "$(dirname "$0")"
if [ "$1" = "sanitize" ]; then
    gcc -std=c11 -D_GNU_SOURCE -O1 -g -fno-omit-frame-pointer -ffp-contract=off -fno-fast-math -fopenmp -fPIC \
        -shared -fsanitize=address,undefined -fno-sanitize-recover=all -Wall -Wextra \
        -o liboracle_san.so start_oracle.c -lm
else
    gcc -std=c11 -D_GNU_SOURCE -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared \
        -Wall -Wextra -o liboracle.so start_oracle.c -lm
fi
