// Tile shapes of the cell kernels (one thread per cell of a tile).
#pragma once
#define TILE2_X 64
#define TILE2_Y 4
#define TILE3_X 64
#define TILE3_Y 4
#define TILE3_Z 1
