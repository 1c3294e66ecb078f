// Tile shapes of the column-marching cell kernels.  2D: one wavefront of 64
// lanes, two x-columns each, marched along y; 3D: 128 x 4 (x, y) columns
// (four wavefronts) marched along z.  The
// march length (cells per tile along the march direction) is chosen by the
// planner at run time.
#pragma once
#define TILE_X 128  // 64 lanes x 2 cells
#define TILE3_Y 4
#define MARCH2_DEFAULT 32
#define MARCH3_DEFAULT 32
#define ROW_ALIGN_DEFAULT 32
