"""Host test of the launch over the ring of wall tiles (csrc/ring.h): for many
grid and tile shapes, the block -> tile map of a ring launch must be a
bijection onto the tiles that are not of the fast kind, so every wall tile is
swept exactly once.  The header is compiled with the host C++ compiler."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1709_05458_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <vector>
#include "ring.h"
using namespace dk;
int main() {
    const int tiles[][2] = {{32, 8}, {16, 16}, {64, 4}, {8, 32}, {8, 8}, {32, 16}, {14, 14}};
    long checked = 0, ringed = 0;
    for (int nx = 3; nx <= 150; nx += (nx < 40 ? 1 : 7))
        for (int ny = 3; ny <= 150; ny += (ny < 40 ? 3 : 11))
            for (auto &t : tiles)
                for (int per = 0; per < 4; per++)
                    for (int nxcd : {8, 1, 3}) {
                        const bool px = per & 1, py = per & 2;
                        const int TX = t[0], TY = t[1];
                        const int gx = (nx + TX - 1) / TX, gy = (ny + TY - 1) / TY;
                        long nfast = 0;
                        for (int ty = 0; ty < gy; ty++)
                            for (int tx = 0; tx < gx; tx++)
                                nfast += tile_fast(true, px, py, nx, ny, tx * TX, ty * TY, TX, TY);
                        const Ring r = ring_make(true, px, py, nx, ny, TX, TY);
                        checked++;
                        if (!r.on) {
                            if (nfast != 0 && nfast != (long)gx * gy) { printf("FAIL off %d %d\n", nx, ny); return 1; }
                            continue;
                        }
                        ringed++;
                        if (r.ng != (long)gx * gy - nfast) { printf("FAIL count %d %d\n", nx, ny); return 1; }
                        std::vector<int> seen((size_t)gx * gy, 0);
                        for (int b = 0; b < r.ng; b++) {
                            int tx, ty;
                            ring_tile_of(r, nxcd, b, tx, ty);
                            if (tx < 0 || tx >= gx || ty < 0 || ty >= gy) { printf("FAIL range %d %d %d\n", nx, ny, b); return 1; }
                            if (tile_fast(true, px, py, nx, ny, tx * TX, ty * TY, TX, TY)) { printf("FAIL fast %d %d\n", nx, ny); return 1; }
                            if (seen[(size_t)ty * gx + tx]++) { printf("FAIL twice %d %d\n", nx, ny); return 1; }
                        }
                    }
    printf("OK %ld %ld\n", checked, ringed);
    return 0;
}
'''


def test_ring_launch_covers_every_wall_tile_once(tmp_path):
    src = tmp_path / "ring_driver.cpp"
    exe = tmp_path / "ring_driver"
    src.write_text(DRIVER)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    ok, checked, ringed = out.stdout.split()
    assert ok == "OK" and int(ringed) > 1000
